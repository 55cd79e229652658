// Coarse matrix A_H = Z^T A Z (Def. 2) computed from local data (Sec. 4.5).
//
// For a basis vector phi supported on D_j (interior dofs of Omega_j), A phi
// is supported on N_j and equals A_N,j phi there, so W_j = A_N,j Z_j is a
// local sparse product and the block (i, j) of A_H is Z_i^T W_j summed over
// the dofs shared by D_i and N_j.  Only pairs of subdomains that share a dof
// are visited (A_H is zero elsewhere); the result goes straight into the
// packed tile storage of the coarse Cholesky (lower triangle).
#include "internal.h"

namespace geneo {

__device__ __forceinline__ int bsearch_sorted(const int* a, int n, int key) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    int v = a[mid];
    if (v == key) return mid;
    if (v < key) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// W_j[a][c] = sum_b A_N,j[a][b] Z_j[dmap(b)][c], rows a over N_j; grid
// (subdomain, chunk of 256 outputs), one thread per output.
__global__ __launch_bounds__(256) void k_galerkin_w(const int* __restrict__ rp,
                                                    const int* __restrict__ colx,
                                                    const double* __restrict__ val,
                                                    const int* __restrict__ sub_ptr,
                                                    const int* __restrict__ dmap,
                                                    const double* __restrict__ Z,
                                                    const int* __restrict__ zoff,
                                                    const int* __restrict__ m,
                                                    const int* __restrict__ woff,
                                                    double* __restrict__ W) {
  const int j = blockIdx.x;
  const int mj = m[j];
  if (mj == 0) return;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  const double* Zj = Z + zoff[j];
  double* Wj = W + woff[j];
  for (int t = blockIdx.y * blockDim.x + threadIdx.x; t < n * mj; t += blockDim.x * gridDim.y) {
    int a = t / mj, c = t % mj;
    double s = 0.0;
    // entries in batches of 8: index and value loads, then the dmap
    // gathers, then the Z gathers, each level in flight together; the sum
    // keeps the entry order (entries outside D_j load row 0 and are skipped)
    const int p1 = rp[s0 + a + 1];
    for (int p0 = rp[s0 + a]; p0 < p1; p0 += 8) {
      int dd[8];
      double vv[8], zv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int p = min(p0 + u, p1 - 1);
        dd[u] = colx[p];
        vv[u] = val[p];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) dd[u] = p0 + u < p1 ? dmap[s0 + dd[u]] : -1;
#pragma unroll
      for (int u = 0; u < 8; ++u) zv[u] = Zj[(int64_t)max(dd[u], 0) * mj + c];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (dd[u] >= 0) s += vv[u] * zv[u];
    }
    Wj[(int64_t)a * mj + c] = s;
  }
}

hipError_t launch_galerkin_w(const geneo_csr_batch_t* An, const int* sub_ptr, const int* dmap,
                             const double* Z, const int* zoff, const int* m, const int* woff,
                             int nsub, int64_t maxwork, double* W, hipStream_t st) {
  const unsigned ny = (unsigned)std::max<int64_t>(1, (maxwork + 255) / 256);
  hipLaunchKernelGGL(k_galerkin_w, dim3(nsub, ny), dim3(256), 0, st, An->rowptr, An->col,
                     An->val, sub_ptr, dmap, Z, zoff, m, woff, W);
  return hipGetLastError();
}

#define CB_CHUNK 2048

// Block (i, j), j <= i, of A_H into the tiled lower triangle: the rows d of
// D_i found in N_j (binary search, in chunks of CB_CHUNK) contribute
// Z_i(d, p) W_j(b(d), q).
__global__ __launch_bounds__(256) void k_coarse_blocks(
    const int2* __restrict__ pairs, const int* __restrict__ sub_ptr,
    const int* __restrict__ sub_idx, const int* __restrict__ didx,
    const int* __restrict__ dvoff, const int* __restrict__ nd, const double* __restrict__ Z,
    const int* __restrict__ zoff, const double* __restrict__ W, const int* __restrict__ woff,
    const int* __restrict__ m, const int* __restrict__ coff, double* __restrict__ AHt) {
  const int i = pairs[blockIdx.x].x, j = pairs[blockIdx.x].y;
  const int mi = m[i], mj = m[j];
  if (mi == 0 || mj == 0) return;
  __shared__ int match[CB_CHUNK];
  const int si = sub_ptr[i];
  const int sj = sub_ptr[j], nj = sub_ptr[j + 1] - sj;
  const int ndi = nd[i];
  const double* Zi = Z + zoff[i];
  const double* Wj = W + woff[j];
  const int npq = mi * mj;
  if (npq <= 256) {
    // thread = (output pq, row group rg): P >= npq outputs padded to a
    // power of two, G = 256 / P row groups each taking every G-th row of
    // D_i; the G partial sums of an output are added in a fixed order
    __shared__ double red[256];
    int P = 1;
    while (P < npq) P <<= 1;
    const int G = 256 / P;
    const int pq = threadIdx.x % P, rg = threadIdx.x / P;
    const int p = pq / mj, q = pq % mj;
    double s = 0.0;
    for (int base = 0; base < ndi; base += CB_CHUNK) {
      const int cnt = min(CB_CHUNK, ndi - base);
      __syncthreads();
      for (int d = threadIdx.x; d < cnt; d += blockDim.x) {
        int a = didx[dvoff[i] + base + d];
        int g = sub_idx[si + a];
        match[d] = bsearch_sorted(sub_idx + sj, nj, g);
      }
      __syncthreads();
      if (pq < npq)
        // rows in batches of 8: the batch's loads are all in flight before
        // the first product (rows outside N_j load row 0 of W_j and are
        // skipped); the sum keeps the row order
        for (int d0 = rg; d0 < cnt; d0 += 8 * G) {
          int bb[8];
          double zv[8], wv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int d = min(d0 + u * G, cnt - 1);
            bb[u] = d0 + u * G < cnt ? match[d] : -1;
            zv[u] = Zi[(int64_t)(base + d) * mi + p];
            wv[u] = Wj[(int64_t)max(bb[u], 0) * mj + q];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (bb[u] >= 0) s += zv[u] * wv[u];
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (rg == 0 && pq < npq) {
      double t = 0.0;
      for (int g2 = 0; g2 < G; ++g2) t += red[g2 * P + pq];
      const int R = coff[i] + p, C = coff[j] + q;
      if (R >= C) AHt[tile_idx(R / TS, C / TS) * TSQ + (R % TS) * TS + (C % TS)] = t;
    }
    return;
  }
  // larger blocks: each thread owns up to 16 (p, q) outputs
  double acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = 0.0;
  for (int base = 0; base < ndi; base += CB_CHUNK) {
    const int cnt = min(CB_CHUNK, ndi - base);
    __syncthreads();
    for (int d = threadIdx.x; d < cnt; d += blockDim.x) {
      int a = didx[dvoff[i] + base + d];
      int g = sub_idx[si + a];
      match[d] = bsearch_sorted(sub_idx + sj, nj, g);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      int t = threadIdx.x + u * 256;
      if (t >= npq) break;
      int p = t / mj, q = t % mj;
      double s = 0.0;
      // batches of 8 rows, as above
      for (int d0 = 0; d0 < cnt; d0 += 8) {
        int bb[8];
        double zv[8], wv[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const int d = min(d0 + v, cnt - 1);
          bb[v] = d0 + v < cnt ? match[d] : -1;
          zv[v] = Zi[(int64_t)(base + d) * mi + p];
          wv[v] = Wj[(int64_t)max(bb[v], 0) * mj + q];
        }
#pragma unroll
        for (int v = 0; v < 8; ++v)
          if (bb[v] >= 0) s += zv[v] * wv[v];
      }
      acc[u] += s;
    }
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    int t = threadIdx.x + u * 256;
    if (t >= npq) break;
    int p = t / mj, q = t % mj;
    int R = coff[i] + p, C = coff[j] + q;
    if (R < C) continue;
    AHt[tile_idx(R / TS, C / TS) * TSQ + (R % TS) * TS + (C % TS)] = acc[u];
  }
}

hipError_t launch_coarse_blocks(const int2* pairs, int npairs, const int* sub_ptr,
                                const int* sub_idx, const int* didx, const int* dvoff,
                                const int* nd, const double* Z, const int* zoff,
                                const double* W, const int* woff, const int* m,
                                const int* coff, double* AHt, hipStream_t st) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_blocks, dim3(npairs), dim3(256), 0, st, pairs, sub_ptr, sub_idx,
                     didx, dvoff, nd, Z, zoff, W, woff, m, coff, AHt);
  return hipGetLastError();
}

// Zero the tiles, unit diagonal on the padding rows nc .. ntc*TS-1.
__global__ void k_coarse_init(double* __restrict__ AHt, int64_t nel, int ntc, int nc) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nel) return;
  int64_t t = e / TSQ;
  int r = (int)((e % TSQ) / TS), c = (int)(e % TS);
  // tile (ti, tk) of index t
  int ti = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while ((int64_t)ti * (ti + 1) / 2 > t) --ti;
  int tk = (int)(t - (int64_t)ti * (ti + 1) / 2);
  int R = ti * TS + r, C = tk * TS + c;
  AHt[e] = (R == C && R >= nc) ? 1.0 : 0.0;
}

hipError_t launch_coarse_init(double* AHt, int ntc, int nc, hipStream_t st) {
  int64_t nel = tri_tiles(ntc) * TSQ;
  hipLaunchKernelGGL(k_coarse_init, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, st, AHt,
                     nel, ntc, nc);
  return hipGetLastError();
}

// Pivot threshold of the coarse Cholesky: a pivot at or below
// nc * eps * max_k (A_H)_kk marks A_H as numerically singular (the rounding
// of the factorisation alone leaves pivots of up to about (k+1) u (A_H)_kk
// where the exact one vanishes, as for a repeated basis vector).
__global__ void k_coarse_pivtol(const double* __restrict__ AHt, int nc, double* __restrict__ tol) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int k = threadIdx.x; k < nc; k += blockDim.x)
    mx = fmax(mx, AHt[tile_idx(k / TS, k / TS) * TSQ + (k % TS) * (TS + 1)]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *tol = (double)nc * 2.220446049250313e-16 * red[0];
}

hipError_t launch_coarse_pivtol(const double* AHt, int nc, double* tol, hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_pivtol, dim3(1), dim3(256), 0, st, AHt, nc, tol);
  return hipGetLastError();
}

__global__ void k_coarse_to_dense(const double* __restrict__ AHt, int nc, double* __restrict__ out) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)nc * nc) return;
  int R = (int)(e / nc), C = (int)(e % nc);
  int r = R >= C ? R : C, c = R >= C ? C : R;
  out[e] = AHt[tile_idx(r / TS, c / TS) * TSQ + (r % TS) * TS + (c % TS)];
}

hipError_t launch_coarse_to_dense(const double* AHt, int ntc, int nc, double* out,
                                  hipStream_t st) {
  (void)ntc;
  int64_t n2 = (int64_t)nc * nc;
  if (n2 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_to_dense, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st,
                     AHt, nc, out);
  return hipGetLastError();
}

}  // namespace geneo
