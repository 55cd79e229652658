// Dense local matrices in packed lower-triangular tile storage.
//
//  * Dirichlet matrices A_j = R_j A R_j^T (Sec. 3) over D_j, read from the
//    global CSR matrix, symmetrically scaled by D^{-1/2} (unit diagonal),
//    stored in FP32 (mixed mode) or FP64.
//  * Shifted matrices C_j = A_N,j - sigma X_j A^o_j X_j over N_j (the matrix
//    of the shift-and-invert transform of Sec. 4.4), FP64.
// The caller clears the tiles (one device-wide fill, or for the shifted
// matrices just their envelope tiles, found from the patterns first); the
// grid is
// (subdomain[, group of 256 rows]) and every thread owns whole rows (a unit
// diagonal first, the identity on padding rows, then the row's entries), so
// no two threads write the same entry.
//
// Tile envelope.  Each fill also records, per tile row i of a matrix, the
// first tile column E(i) that holds an entry of the matrix's pattern
// (atomic minimum over the rows of the tile row, from E(i) = i).  A
// Cholesky factor has no entries left of the first entry of each row of
// its matrix, so tiles (i, jj < E(i)) of the factor are zero.
// k_env_finish then makes E nondecreasing (E(i) = min over rows >= i: a
// superset of the nonzero tiles) and forms R(k) = the last tile row i with
// E(i) <= k, the last nonzero tile of tile column k.  Box subdomains in
// lexicographic order give banded matrices: E(i) trails i by about the
// band width in tiles.
#include "internal.h"

namespace geneo {

__global__ __launch_bounds__(256) void k_env_init(int* __restrict__ env,
                                                  const int64_t* __restrict__ doff,
                                                  const int* __restrict__ ntl,
                                                  const int* __restrict__ jobs) {
  const int j = jobs ? jobs[blockIdx.x] : blockIdx.x, nt = ntl[j];
  int* E = env + doff[j];
  for (int i = threadIdx.x; i < nt; i += blockDim.x) E[i] = i;
}

__global__ __launch_bounds__(64) void k_env_finish(int* __restrict__ envE, int* __restrict__ envR,
                                                   const int64_t* __restrict__ doff,
                                                   const int* __restrict__ ntl,
                                                   const int* __restrict__ jobs, int njobs) {
  const int q = blockIdx.x * 64 + threadIdx.x;
  if (q >= njobs) return;
  const int j = jobs ? jobs[q] : q;
  const int nt = ntl[j];
  int* E = envE + doff[j];
  int* R = envR + doff[j];
  int m = nt;
  for (int i = nt - 1; i >= 0; --i) {
    m = min(m, min(E[i], i));
    E[i] = max(m, 0);
  }
  int i = nt - 1;
  for (int k = nt - 1; k >= 0; --k) {
    while (E[i] > k) --i;  // stops at i = k at the latest (E(k) <= k)
    R[k] = i;
  }
}

hipError_t launch_env_init(int* env, const int64_t* doff, const int* nt, const int* jobs,
                           int njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_env_init, dim3(njobs), dim3(256), 0, st, env, doff, nt, jobs);
  return hipGetLastError();
}

hipError_t launch_env_finish(int* envE, int* envR, const int64_t* doff, const int* nt,
                             const int* jobs, int njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_env_finish, dim3((njobs + 63) / 64), dim3(64), 0, st, envE, envR, doff, nt,
                     jobs, njobs);
  return hipGetLastError();
}

template <typename T>
__device__ __forceinline__ T* tile_elem(T* base, int r, int c) {
  return base + tile_idx(r / TS, c / TS) * TSQ + (r % TS) * TS + (c % TS);
}

// bsearch_row for 8 keys at once: branch-free halving steps, the same
// number for every key, so the 8 probes of a step are in flight together.
// pos[u] = index of key[u] in the sorted a[0..n), or -1.
__device__ __forceinline__ void bsearch_row8(const int* a, int n, const int (&key)[8],
                                             int (&pos)[8]) {
  int base[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) base[u] = 0;
  for (int len = n; len > 1;) {
    const int half = len >> 1;
    int v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = a[base[u] + half];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (v[u] <= key[u]) base[u] += half;
    len -= half;
  }
  int v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = n > 0 ? a[base[u]] : key[u] + 1;
#pragma unroll
  for (int u = 0; u < 8; ++u) pos[u] = v[u] == key[u] ? base[u] : -1;
}

template <typename T>
__global__ __launch_bounds__(256) void k_densify_dirichlet(
    T* __restrict__ tiles, const int64_t* __restrict__ toff, const int* __restrict__ ntl,
    const int* __restrict__ voff, const int* __restrict__ jobs, const int* __restrict__ sub_ptr,
    const int* __restrict__ sub_idx, const int* __restrict__ dmap, const int* __restrict__ dglob,
    const double* __restrict__ dscale, const int* __restrict__ rowptr,
    const int* __restrict__ col, const double* __restrict__ val, int* __restrict__ env,
    const int64_t* __restrict__ doff) {
  const int j = jobs[blockIdx.x];
  const int nt = ntl[j];
  T* base = tiles + toff[j] * TSQ;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  const int v0 = voff[j];
  const int* Nj = sub_idx + s0;
  for (int d = blockIdx.y * blockDim.x + threadIdx.x; d < nt * TS; d += blockDim.x * gridDim.y) {
    *tile_elem(base, d, d) = (T)1;
    int g = dglob[v0 + d];
    if (g < 0) continue;
    double sd = dscale[v0 + d];
    int first = d;
    // the row's entries in batches of 8, each level of loads (index and
    // value, the searches' probes, dmap, dscale) in flight together
    const int p1 = rowptr[g + 1];
    for (int p0 = rowptr[g]; p0 < p1; p0 += 8) {
      int key[8], a8[8], dc8[8];
      double v8[8], sc8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int p = min(p0 + u, p1 - 1);
        key[u] = col[p];
        v8[u] = val[p];
      }
      bsearch_row8(Nj, n, key, a8);
#pragma unroll
      for (int u = 0; u < 8; ++u) dc8[u] = p0 + u < p1 && a8[u] >= 0 ? dmap[s0 + a8[u]] : -1;
#pragma unroll
      for (int u = 0; u < 8; ++u) sc8[u] = dscale[v0 + max(dc8[u], 0)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int dc = dc8[u];
        if (dc < 0 || dc > d) continue;
        *tile_elem(base, d, dc) = (T)(v8[u] * sd * sc8[u]);
        first = min(first, dc);
      }
    }
    if (env && first / TS < d / TS) atomicMin(env + doff[j] + d / TS, first / TS);
  }
}

hipError_t launch_densify_dirichlet(bool fp32, void* tiles, const int64_t* toff, const int* nt,
                                    const int* voff, const int* jobs, int njobs,
                                    const int* sub_ptr, const int* sub_idx, const int* dmap,
                                    const int* dglob, const double* dscale, const geneo_csr_t* A,
                                    int ntmax, int* env, const int64_t* doff, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  const dim3 grid(njobs, std::max(1, (ntmax * TS + 255) / 256));
  if (fp32)
    hipLaunchKernelGGL(k_densify_dirichlet<float>, grid, dim3(256), 0, st, (float*)tiles,
                       toff, nt, voff, jobs, sub_ptr, sub_idx, dmap, dglob, dscale, A->rowptr,
                       A->col, A->val, env, doff);
  else
    hipLaunchKernelGGL(k_densify_dirichlet<double>, grid, dim3(256), 0, st,
                       (double*)tiles, toff, nt, voff, jobs, sub_ptr, sub_idx, dmap, dglob,
                       dscale, A->rowptr, A->col, A->val, env, doff);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_densify_shifted(
    double* __restrict__ tiles, const int64_t* __restrict__ toff, const int* __restrict__ ntl,
    const int* __restrict__ sub_ptr, const double* __restrict__ pou,
    const int* __restrict__ an_rp, const int* __restrict__ an_col,
    const double* __restrict__ an_val, const int* __restrict__ ao_rp,
    const int* __restrict__ ao_col, const double* __restrict__ ao_val, double sigma,
    int* __restrict__ env, const int64_t* __restrict__ doff) {
  const int j = blockIdx.x;
  const int nt = ntl[j];
  double* base = tiles + toff[j] * TSQ;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  for (int a = blockIdx.y * blockDim.x + threadIdx.x; a < nt * TS; a += blockDim.x * gridDim.y) {
    *tile_elem(base, a, a) = 1.0;
    if (a >= n) continue;
    int first = a;
    // entries in batches of 8, each level of loads in flight together
    // (the columns of a row are distinct, so a batch's updates are too)
    const int pa1 = an_rp[s0 + a + 1];
    for (int p0 = an_rp[s0 + a]; p0 < pa1; p0 += 8) {
      int c8[8];
      double v8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int p = min(p0 + u, pa1 - 1);
        c8[u] = an_col[p];
        v8[u] = an_val[p];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (p0 + u >= pa1 || c8[u] > a) continue;
        *tile_elem(base, a, c8[u]) = v8[u];
        first = min(first, c8[u]);
      }
    }
    double mua = pou[s0 + a];
    if (mua != 0.0) {
      const int po1 = ao_rp[s0 + a + 1];
      for (int p0 = ao_rp[s0 + a]; p0 < po1; p0 += 8) {
        int c8[8];
        double v8[8], m8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int p = min(p0 + u, po1 - 1);
          c8[u] = ao_col[p];
          v8[u] = ao_val[p];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) m8[u] = pou[s0 + c8[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (p0 + u >= po1 || c8[u] > a) continue;
          *tile_elem(base, a, c8[u]) -= sigma * mua * v8[u] * m8[u];
          first = min(first, c8[u]);
        }
      }
    }
    if (env && first / TS < a / TS) atomicMin(env + doff[j] + a / TS, first / TS);
  }
}

// Envelope of the shifted matrices from the patterns alone (the first
// column of each row among the entries of A_N,j and A^o_j at or left of the
// diagonal; padding rows: the diagonal), without writing a tile: a pass
// over the column indices, so that only the envelope tiles need clearing
// before the fill.  Grid (subdomain, group of 256 rows).
__global__ __launch_bounds__(256) void k_env_shifted(const int* __restrict__ ntl,
                                                     const int* __restrict__ sub_ptr,
                                                     const int* __restrict__ an_rp,
                                                     const int* __restrict__ an_col,
                                                     const int* __restrict__ ao_rp,
                                                     const int* __restrict__ ao_col,
                                                     int* __restrict__ env,
                                                     const int64_t* __restrict__ doff) {
  const int j = blockIdx.x;
  const int nt = ntl[j];
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  const int a = blockIdx.y * blockDim.x + threadIdx.x;
  if (a >= nt * TS) return;
  int first = a;
  if (a < n) {
    for (int p = an_rp[s0 + a]; p < an_rp[s0 + a + 1]; ++p) first = min(first, an_col[p]);
    for (int p = ao_rp[s0 + a]; p < ao_rp[s0 + a + 1]; ++p) first = min(first, ao_col[p]);
  }
  if (first / TS < a / TS) atomicMin(env + doff[j] + a / TS, first / TS);
}

// Zeroes tiles E(i) .. i of tile row blockIdx.y of matrix blockIdx.x (they
// are consecutive in the packed layout).
__global__ __launch_bounds__(256) void k_env_clear(double* __restrict__ tiles,
                                                   const int64_t* __restrict__ toff,
                                                   const int* __restrict__ ntl,
                                                   const int* __restrict__ envE,
                                                   const int64_t* __restrict__ doff) {
  const int j = blockIdx.x, i = blockIdx.y;
  if (i >= ntl[j]) return;
  const int e = envE[doff[j] + i];
  double2* t = reinterpret_cast<double2*>(tiles + (toff[j] + tile_idx(i, e)) * TSQ);
  const int nv = (i - e + 1) * TSQ / 2;
  for (int v = threadIdx.x; v < nv; v += blockDim.x) t[v] = make_double2(0.0, 0.0);
}

hipError_t launch_env_shifted(const int* nt, int nsub, int ntmax, const int* sub_ptr,
                              const geneo_csr_batch_t* An, const geneo_csr_batch_t* Ao, int* env,
                              const int64_t* doff, hipStream_t st) {
  if (nsub <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_env_shifted, dim3(nsub, (ntmax * TS + 255) / 256), dim3(256), 0, st, nt,
                     sub_ptr, An->rowptr, An->col, Ao->rowptr, Ao->col, env, doff);
  return hipGetLastError();
}

hipError_t launch_env_clear(double* tiles, const int64_t* toff, const int* nt, int nsub,
                            int ntmax, const int* envE, const int64_t* doff, hipStream_t st) {
  if (nsub <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_env_clear, dim3(nsub, ntmax), dim3(256), 0, st, tiles, toff, nt, envE,
                     doff);
  return hipGetLastError();
}

hipError_t launch_densify_shifted(double* tiles, const int64_t* toff, const int* nt, int nsub,
                                  const int* sub_ptr, const double* pou,
                                  const geneo_csr_batch_t* An, const geneo_csr_batch_t* Ao,
                                  double sigma, int* env, const int64_t* doff, hipStream_t st) {
  // one workgroup per subdomain: measured faster here than splitting the
  // rows over several (the Dirichlet fill, launched for fewer matrices,
  // splits them)
  hipLaunchKernelGGL(k_densify_shifted, dim3(nsub), dim3(256), 0, st, tiles, toff, nt, sub_ptr,
                     pou, An->rowptr, An->col, An->val, Ao->rowptr, Ao->col, Ao->val, sigma, env,
                     doff);
  return hipGetLastError();
}

}  // namespace geneo
