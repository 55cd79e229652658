// Index bookkeeping on the device: prefix sums, the D_j maps of the local
// Dirichlet problems, diagonal scaling, the dof -> (subdomain, local index)
// owner lists used by the deterministic overlap sums, and subdomain
// adjacency (which subdomain pairs share a dof).
#include "internal.h"

namespace geneo {

void LocalLayout::build(const std::vector<int>& rows) {
  n = (int)rows.size();
  nrow = rows;
  nt.assign(n, 0);
  toff.assign(n, 0);
  doff.assign(n, 0);
  voff.assign(n, 0);
  ntiles = ndiag = nvec = 0;
  maxnt = 0;
  for (int j = 0; j < n; ++j) {
    int t = (rows[j] + TS - 1) / TS;
    if (t < 1) t = 1;
    nt[j] = t;
    toff[j] = ntiles;
    doff[j] = ndiag;
    voff[j] = (int)nvec;
    ntiles += tri_tiles(t);
    ndiag += t;
    nvec += (int64_t)t * TS;
    if (t > maxnt) maxnt = t;
  }
}

// ------------------------------------------------------------ prefix sums
#define SCAN_BS 1024
#define SCAN_PER 4
#define SCAN_CHUNK (SCAN_BS * SCAN_PER)

__device__ int block_excl_scan(int v, int* sh, int* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_BS; off <<= 1) {
    int x = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  int incl = sh[t];
  if (total) *total = sh[SCAN_BS - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(SCAN_BS) void k_scan_chunks(const int* __restrict__ in,
                                                         int* __restrict__ out, int64_t n,
                                                         int* __restrict__ bsum) {
  __shared__ int sh[SCAN_BS];
  __shared__ int tot;
  int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int v[SCAN_PER], s = 0;
  for (int q = 0; q < SCAN_PER; ++q) {
    v[q] = (base + q < n) ? in[base + q] : 0;
    s += v[q];
  }
  int ex = block_excl_scan(s, sh, &tot);
  for (int q = 0; q < SCAN_PER; ++q) {
    if (base + q < n) out[base + q] = ex;
    ex += v[q];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BS) void k_scan_add(int* __restrict__ out, int64_t n,
                                                      const int* __restrict__ boff) {
  int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int add = boff[blockIdx.x];
  for (int q = 0; q < SCAN_PER; ++q)
    if (base + q < n) out[base + q] += add;
}

__global__ void k_scan_total(const int* __restrict__ in, const int* __restrict__ out, int64_t n,
                             int* __restrict__ outn, int* __restrict__ total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int t = n > 0 ? out[n - 1] + in[n - 1] : 0;
    outn[n] = t;
    if (total) *total = t;
  }
}

// Exclusive scan of n ints; out has n+1 entries (out[n] = total).  The
// recursion allocates its block-sum buffers with hipMallocAsync.
hipError_t scan_exclusive_i32(const int* in, int* out, int64_t n, int* total_dev,
                              hipStream_t st) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, in, out, (int64_t)0, out,
                       total_dev);
    return hipGetLastError();
  }
  int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
  int* bsum = nullptr;
  int* boff = nullptr;
  hipError_t e = hipMallocAsync((void**)&bsum, (nb + 1) * sizeof(int), st);
  if (e != hipSuccess) return e;
  e = hipMallocAsync((void**)&boff, (nb + 1) * sizeof(int), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nb), dim3(SCAN_BS), 0, st, in, out, n, bsum);
  if (nb > 1) {
    e = scan_exclusive_i32(bsum, boff, nb, nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_BS), 0, st, out, n, boff);
  }
  hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, in, out, n, out, total_dev);
  e = hipGetLastError();
  hipFreeAsync(bsum, st);
  hipFreeAsync(boff, st);
  return e;
}

// ----------------------------------------------------------- D_j maps ---
// dmap[sub_ptr[j] + a] = position of local dof a in D_j, or -1; nd[j] = |D_j|.
__global__ __launch_bounds__(SCAN_BS) void k_dmap(const int* __restrict__ sub_ptr,
                                                  const uint8_t* __restrict__ flags,
                                                  int* __restrict__ dmap, int* __restrict__ nd) {
  __shared__ int sh[SCAN_BS];
  __shared__ int tot;
  const int j = blockIdx.x;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  int carry = 0;
  for (int base = 0; base < n; base += SCAN_BS) {
    int a = base + threadIdx.x;
    int f = (a < n) ? (flags[s0 + a] & 1) : 0;
    int ex = block_excl_scan(f, sh, &tot);
    if (a < n) dmap[s0 + a] = f ? carry + ex : -1;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) nd[j] = carry;
}

hipError_t launch_dmap(const int* sub_ptr, const uint8_t* flags, int nsub, int* dmap, int* nd,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_dmap, dim3(nsub), dim3(SCAN_BS), 0, st, sub_ptr, flags, dmap, nd);
  return hipGetLastError();
}

// Binary search of `key` in the ascending array a[0..n); -1 if absent.
__device__ __forceinline__ int bsearch_i32(const int* a, int n, int key) {
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

// Padded per-subdomain vectors over D_j: global dof (or -1 on padding), the
// N_j-local index, and the diagonal scaling 1/sqrt(A_gg) (0 on padding).
__global__ void k_dvec(const int* __restrict__ sub_ptr, const int* __restrict__ sub_idx,
                       const int* __restrict__ dmap, const int* __restrict__ voff,
                       const int* __restrict__ nt, const int* __restrict__ rowptr,
                       const int* __restrict__ col, const double* __restrict__ val,
                       int* __restrict__ dglob, int* __restrict__ didx,
                       double* __restrict__ dscale) {
  const int j = blockIdx.x;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  const int v0 = voff[j], npad = nt[j] * TS;
  for (int d = threadIdx.x; d < npad; d += blockDim.x) {
    dglob[v0 + d] = -1;
    didx[v0 + d] = -1;
    dscale[v0 + d] = 0.0;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    int d = dmap[s0 + a];
    if (d < 0) continue;
    int g = sub_idx[s0 + a];
    int r0 = rowptr[g], r1 = rowptr[g + 1];
    int p = bsearch_i32(col + r0, r1 - r0, g);
    double diag = p >= 0 ? val[r0 + p] : 0.0;
    dglob[v0 + d] = g;
    didx[v0 + d] = a;
    dscale[v0 + d] = diag > 0.0 ? 1.0 / sqrt(diag) : 0.0;
  }
}

hipError_t launch_dvec(const int* sub_ptr, const int* sub_idx, const int* dmap,
                       const int* voff, const int* nt, int nsub, const geneo_csr_t* A,
                       int* dglob, int* didx, double* dscale, hipStream_t st) {
  hipLaunchKernelGGL(k_dvec, dim3(nsub), dim3(256), 0, st, sub_ptr, sub_idx, dmap, voff, nt,
                     A->rowptr, A->col, A->val, dglob, didx, dscale);
  return hipGetLastError();
}

// ------------------------------------------------------------- owners ---
// For every global dof g the list of (subdomain j, N_j-local index a) with
// g in N_j, sorted by j: optr [ndof+1], olist [nloc].
__global__ void k_owner_count(const int* __restrict__ sub_ptr, const int* __restrict__ sub_idx,
                              int* __restrict__ cnt) {
  const int j = blockIdx.x;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  for (int a = threadIdx.x; a < n; a += blockDim.x) atomicAdd(&cnt[sub_idx[s0 + a]], 1);
}

__global__ void k_owner_fill(const int* __restrict__ sub_ptr, const int* __restrict__ sub_idx,
                             const int* __restrict__ optr, int* __restrict__ fill,
                             int2* __restrict__ olist) {
  const int j = blockIdx.x;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    int g = sub_idx[s0 + a];
    int slot = optr[g] + atomicAdd(&fill[g], 1);
    olist[slot] = make_int2(j, a);
  }
}

__global__ void k_owner_sort(const int* __restrict__ optr, int2* __restrict__ olist, int ndof) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ndof) return;
  int p0 = optr[g], p1 = optr[g + 1];
  for (int p = p0 + 1; p < p1; ++p) {
    int2 key = olist[p];
    int q = p - 1;
    while (q >= p0 && olist[q].x > key.x) {
      olist[q + 1] = olist[q];
      --q;
    }
    olist[q + 1] = key;
  }
}

hipError_t launch_owners(const int* sub_ptr, const int* sub_idx, int nsub, int64_t nloc,
                         int ndof, int* optr, int* ocount, int2* olist, hipStream_t st) {
  hipError_t e = hipMemsetAsync(ocount, 0, sizeof(int) * (size_t)ndof, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_owner_count, dim3(nsub), dim3(256), 0, st, sub_ptr, sub_idx, ocount);
  e = scan_exclusive_i32(ocount, optr, ndof, nullptr, st);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(ocount, 0, sizeof(int) * (size_t)ndof, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_owner_fill, dim3(nsub), dim3(256), 0, st, sub_ptr, sub_idx, optr, ocount,
                     olist);
  hipLaunchKernelGGL(k_owner_sort, dim3((ndof + 255) / 256), dim3(256), 0, st, optr, olist,
                     ndof);
  return hipGetLastError();
}

// ---------------------------------------------------------- adjacency ---
// adj[i*nsub + j] = 1 when N_i and N_j share a dof.
__global__ void k_adjacency(const int* __restrict__ optr, const int2* __restrict__ olist,
                            int ndof, int nsub, uint8_t* __restrict__ adj) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ndof) return;
  int p0 = optr[g], p1 = optr[g + 1];
  for (int p = p0; p < p1; ++p)
    for (int q = p0; q < p1; ++q) adj[(int64_t)olist[p].x * nsub + olist[q].x] = 1;
}

hipError_t launch_adjacency(const int* optr, const int2* olist, int ndof, int nsub,
                            uint8_t* adj, hipStream_t st) {
  hipError_t e = hipMemsetAsync(adj, 0, (size_t)nsub * nsub, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adjacency, dim3((ndof + 255) / 256), dim3(256), 0, st, optr, olist, ndof,
                     nsub, adj);
  return hipGetLastError();
}

// Pairs (i, j) with j <= i and adj[i][j], row by row in ascending j.
__global__ void k_pair_count(const uint8_t* __restrict__ adj, int nsub, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsub) return;
  int c = 0;
  for (int j = 0; j <= i; ++j) c += adj[(int64_t)i * nsub + j];
  cnt[i] = c;
}

__global__ void k_pair_fill(const uint8_t* __restrict__ adj, int nsub, const int* __restrict__ off,
                            int2* __restrict__ pairs) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsub) return;
  int p = off[i];
  for (int j = 0; j <= i; ++j)
    if (adj[(int64_t)i * nsub + j]) pairs[p++] = make_int2(i, j);
}

hipError_t launch_pairs(const uint8_t* adj, int nsub, int* cnt, int* off, int2* pairs,
                        int* npairs_dev, hipStream_t st, bool count_only) {
  if (count_only) {
    hipLaunchKernelGGL(k_pair_count, dim3((nsub + 255) / 256), dim3(256), 0, st, adj, nsub, cnt);
    return scan_exclusive_i32(cnt, off, nsub, npairs_dev, st);
  }
  hipLaunchKernelGGL(k_pair_fill, dim3((nsub + 255) / 256), dim3(256), 0, st, adj, nsub, off,
                     pairs);
  return hipGetLastError();
}

}  // namespace geneo
