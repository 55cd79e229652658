// Solve-phase kernels: CSR SpMV, the pieces of the preconditioner apply that
// move data between the global vector and the per-subdomain blocks, and
// the PCG recurrences with their scalars kept on the device.
//
// Every reduction is two-stage with a fixed partition (per-block partial
// sums, then one block adds them in a fixed order), so results do not
// depend on scheduling.  Every kernel that runs inside the iteration reads
// the `done` flag first and returns once the iteration has stopped, which
// lets a captured graph of several iterations run past convergence.
#include "internal.h"
#include "pcg.h"

namespace geneo {

// ---------------------------------------------------------------- SpMV ---
template <int LPR>
__global__ __launch_bounds__(256) void k_spmv(int n, const int* __restrict__ rp,
                                              const int* __restrict__ col,
                                              const double* __restrict__ val,
                                              const double* __restrict__ x,
                                              double* __restrict__ y,
                                              const int* __restrict__ done) {
  if (done && *done) return;
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = gl / LPR, sub = gl % LPR;
  double s = 0.0;
  if (row < n) {
    const int p1 = rp[row + 1];
    // a lane's entries in batches of 4: the index and value loads, then the
    // gathers, all in flight before the first product; the sum keeps the
    // entry order
    for (int p = rp[row] + sub; p < p1; p += 4 * LPR) {
      int cc[4];
      double vv[4], xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = min(p + u * LPR, p1 - 1);  // in range; extra terms unused
        cc[u] = col[q];
        vv[u] = val[q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = x[cc[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (p + u * LPR < p1) s += vv[u] * xv[u];
    }
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR);
  if (row < n && sub == 0) y[row] = s;
}

hipError_t spmv(const geneo_csr_t* A, const double* x, double* y, int lpr, const int* done,
                hipStream_t st) {
  const int n = A->n;
  const int64_t thr = (int64_t)n * lpr;
  const dim3 grid((unsigned)((thr + 255) / 256)), blk(256);
  switch (lpr) {
    case 4: hipLaunchKernelGGL(k_spmv<4>, grid, blk, 0, st, n, A->rowptr, A->col, A->val, x, y, done); break;
    case 8: hipLaunchKernelGGL(k_spmv<8>, grid, blk, 0, st, n, A->rowptr, A->col, A->val, x, y, done); break;
    case 16: hipLaunchKernelGGL(k_spmv<16>, grid, blk, 0, st, n, A->rowptr, A->col, A->val, x, y, done); break;
    default: hipLaunchKernelGGL(k_spmv<32>, grid, blk, 0, st, n, A->rowptr, A->col, A->val, x, y, done); break;
  }
  return hipGetLastError();
}

int spmv_lanes(const geneo_csr_t* A) {
  double avg = A->n > 0 ? (double)A->nnz / A->n : 1.0;
  if (avg <= 10) return 4;
  if (avg <= 30) return 8;
  if (avg <= 60) return 16;
  return 32;
}

// ------------------------------------------------------- apply pieces ---
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
  __syncthreads();
  return t;
}

// Sum over the block, returned to every thread (fixed order).
__device__ __forceinline__ double block_allsum(double v, double* sh) {
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) sh[4] = t;
  __syncthreads();
  const double r = sh[4];
  __syncthreads();
  return r;
}

// Sum of nb partial sums, returned to every thread of the block (the same
// order in every block, so every block gets the same value).
__device__ double allsum_partials(const double* partial, int nb, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  return block_allsum(s, sh);
}

__device__ double sum_partials(const double* partial, int nb, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  return block_sum(s, sh);
}

__global__ void k_gather_local(const double* __restrict__ r, const int* __restrict__ dglob,
                               const double* __restrict__ dscale, int64_t nvec,
                               double* __restrict__ xl, const int* __restrict__ done) {
  if (done && *done) return;
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nvec) return;
  int g = dglob[e];
  xl[e] = g >= 0 ? dscale[e] * r[g] : 0.0;
}

hipError_t gather_local(const double* r, const int* dglob, const double* dscale, int64_t nvec,
                        double* xl, const int* done, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_local, dim3((unsigned)((nvec + 255) / 256)), dim3(256), 0, st, r,
                     dglob, dscale, nvec, xl, done);
  return hipGetLastError();
}

// r_H entries of subdomain j, (Z_j^T R_j r)_c for c < m_j, by one block of
// 256 threads: thread t takes the rows t, t + 256, ... of the D_j block of Z
// (row-major, m_j entries a row, read contiguously) with r at their global
// dofs, for up to 16 columns at a time; the column sums are reduced within
// each wavefront and then over the 4 wavefronts in a fixed order.
__device__ __forceinline__ void restrict_block(int j, const double* __restrict__ r,
                                               const double* __restrict__ Z,
                                               const int* __restrict__ zoff,
                                               const int* __restrict__ m,
                                               const int* __restrict__ nd,
                                               const int* __restrict__ dglob,
                                               const int* __restrict__ dvoff,
                                               const int* __restrict__ coff,
                                               double* __restrict__ rH) {
  __shared__ double sred[4][16];
  const int mj = m[j];
  if (mj == 0) return;
  const int n = nd[j];
  const double* Zj = Z + zoff[j];
  const int* gj = dglob + dvoff[j];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c0 = 0; c0 < mj; c0 += 16) {
    const int nc = min(16, mj - c0);
    double s[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) s[c] = 0.0;
    // rows in batches of 4 (stride 256): the index loads, then the gathers
    // of r, all in flight before the first product; rows in order
    for (int d0 = threadIdx.x; d0 < n; d0 += 4 * 256) {
      double rv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) rv[u] = r[gj[min(d0 + 256 * u, n - 1)]];
#pragma unroll 1
      for (int u = 0; u < 4; ++u) {
        const int d = d0 + 256 * u;
        if (d >= n) break;
        const double* zr = Zj + (int64_t)d * mj + c0;
        // the row's 16 loads issued together (columns past nc read column
        // nc - 1 and feed only accumulators that are never stored)
        double zv[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) zv[c] = zr[min(c, nc - 1)];
#pragma unroll
        for (int c = 0; c < 16; ++c) s[c] += zv[c] * rv[u];
      }
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if (c >= nc) break;
      for (int o = 32; o > 0; o >>= 1) s[c] += __shfl_xor(s[c], o);
    }
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < nc) sred[w][c] = s[c];
    }
    __syncthreads();
    if (threadIdx.x < nc)
      rH[coff[j] + c0 + threadIdx.x] =
          sred[0][threadIdx.x] + sred[1][threadIdx.x] + sred[2][threadIdx.x] + sred[3][threadIdx.x];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_restrict(const double* __restrict__ r,
                                                  const double* __restrict__ Z,
                                                  const int* __restrict__ zoff,
                                                  const int* __restrict__ m,
                                                  const int* __restrict__ nd,
                                                  const int* __restrict__ dglob,
                                                  const int* __restrict__ dvoff,
                                                  const int* __restrict__ coff,
                                                  double* __restrict__ rH,
                                                  const int* __restrict__ done) {
  if (done && *done) return;
  restrict_block(blockIdx.x, r, Z, zoff, m, nd, dglob, dvoff, coff, rH);
}

hipError_t restrict_coarse(const double* r, const double* Z, const int* zoff, const int* m,
                           const int* nd, const int* dglob, const int* dvoff, const int* coff,
                           int nsub, double* rH, const int* done, hipStream_t st) {
  hipLaunchKernelGGL(k_restrict, dim3(nsub), dim3(256), 0, st, r, Z, zoff, m, nd, dglob, dvoff,
                     coff, rH, done);
  return hipGetLastError();
}

// Owner entries of the combine, resolved once per setup: for the owner
// entry (j, local index a) of a dof, e = the D_j-vector position of a (or -1
// when a is not in D_j), the offset of its row of Z_j, the coarse offset of
// subdomain j and m_j.
__global__ __launch_bounds__(256) void k_owner_entries(const int2* __restrict__ olist,
                                                       int64_t nent,
                                                       const int* __restrict__ sub_ptr,
                                                       const int* __restrict__ dmap,
                                                       const int* __restrict__ dvoff,
                                                       const int* __restrict__ zoff,
                                                       const int* __restrict__ m,
                                                       const int* __restrict__ coff,
                                                       int4* __restrict__ oent) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= nent) return;
  const int2 o = olist[p];
  const int j = o.x;
  const int d = dmap[sub_ptr[j] + o.y];
  const int mj = m[j];
  oent[p] = d < 0 ? make_int4(-1, 0, 0, 0)
                  : make_int4(dvoff[j] + d, zoff[j] + d * mj, coff[j], mj);
}

hipError_t owner_entries(const int2* olist, int64_t nent, const int* sub_ptr, const int* dmap,
                         const int* dvoff, const int* zoff, const int* m, const int* coff,
                         int4* oent, hipStream_t st) {
  if (nent <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_owner_entries, dim3((unsigned)((nent + 255) / 256)), dim3(256), 0, st,
                     olist, nent, sub_ptr, dmap, dvoff, zoff, m, coff, oent);
  return hipGetLastError();
}

// z[g] = sum over the subdomains j owning g (in ascending j) of
//        s_d y_j[d] + Z_j[d][:] . yH[coff_j :]          (d = dmap_j(g) >= 0)
// and z[g] = r[g] for a dof in no D_j (an eliminated Dirichlet dof: its row
// of A is a unit row, so the operator stays SPD on every dof).  The owner
// entries come resolved (k_owner_entries): one load each, then independent
// loads of the scale, the local value and the coarse row.
__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ r,
                                                 const int* __restrict__ optr,
                                                 const int4* __restrict__ oent,
                                                 const double* __restrict__ dscale,
                                                 const double* __restrict__ yl,
                                                 const double* __restrict__ Z,
                                                 const double* __restrict__ yH, int ndof,
                                                 int use_coarse, double* __restrict__ z,
                                                 const int* __restrict__ done,
                                                 double* __restrict__ rz_partial) {
  if (done && *done) return;
  __shared__ double sh[4];
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  double zg = 0.0, rg = 0.0;
  if (g < ndof) {
    double s = 0.0;
    bool covered = false;
    for (int p = optr[g]; p < optr[g + 1]; ++p) {
      const int4 o = oent[p];
      if (o.x < 0) continue;
      covered = true;
      s += dscale[o.x] * yl[o.x];
      if (use_coarse) {
        // columns in batches of 8: the batch's loads are all in flight
        // before the first product (one round trip per batch, not per
        // column); the sum keeps the column order
        const double* zr = Z + o.y;
        const double* yh = yH + o.z;
        for (int c0 = 0; c0 < o.w; c0 += 8) {
          double zv[8], hv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int c = min(c0 + u, o.w - 1);  // in range; extra terms unused
            zv[u] = zr[c];
            hv[u] = yh[c];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (c0 + u < o.w) s += zv[u] * hv[u];
        }
      }
    }
    rg = r[g];
    zg = covered ? s : rg;
    z[g] = zg;
  }
  if (rz_partial) {
    // this block's share of r.z (rows 256 b .. 256 b + 255), fixed order
    const double t = block_sum(rg * zg, sh);
    if (threadIdx.x == 0) rz_partial[blockIdx.x] = t;
  }
}

hipError_t combine(const double* r, const int* optr, const int4* oent, const double* dscale,
                   const double* yl, const double* Z, const double* yH, int ndof, int use_coarse,
                   double* z, const int* done, double* rz_partial, hipStream_t st) {
  hipLaunchKernelGGL(k_combine, dim3((ndof + 255) / 256), dim3(256), 0, st, r, optr, oent, dscale,
                     yl, Z, yH, ndof, use_coarse, z, done, rz_partial);
  return hipGetLastError();
}

// -------------------------------------------------------- PCG kernels ---
// partial[b] = sum over the fixed row range of block b of x.y
__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ x,
                                                     const double* __restrict__ y, int n,
                                                     double* __restrict__ partial,
                                                     const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Start of PCG on the device (no host round trip).  stage 0: b.b from the
// partial sums; every scalar reset, tol2 = rtol^2 b.b, done = (b = 0).
// stage 1: r0.r0; done (and converged) when it is already within tol2.
__global__ __launch_bounds__(256) void k_pcg_start(const double* __restrict__ partial, int nb,
                                                   int stage, PcgScalars* __restrict__ sc,
                                                   int* __restrict__ done, double rtol2,
                                                   int maxit) {
  __shared__ double sh[4];
  const double s = sum_partials(partial, nb, sh);
  if (threadIdx.x != 0) return;
  if (stage == 0) {
    PcgScalars z{};
    z.bb = s;
    z.tol2 = rtol2 * s;
    z.maxit = maxit;
    z.converged = s == 0.0 ? 1 : 0;
    *sc = z;
    *done = z.converged;
  } else {
    sc->rr = s;
    if (!*done && s <= sc->tol2) {
      sc->converged = 1;
      *done = 1;
    }
  }
}

hipError_t dot_partial(const double* x, const double* y, int n, double* partial, const int* done,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial, dim3(PCG_NB), dim3(256), 0, st, x, y, n, partial, done);
  return hipGetLastError();
}

hipError_t pcg_start(const double* partial, int stage, PcgScalars* sc, int* done, double rtol2,
                     int maxit, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(256), 0, st, partial, PCG_NB, stage, sc, done,
                     rtol2, maxit);
  return hipGetLastError();
}

// ------------------------------------------------ fused PCG iteration ---
// The scalars of an iteration are not formed by separate one-thread
// kernels: every block of the kernel that needs one sums the fixed-order
// partial sums itself (identical in every block); block 0 records it.

// alpha = (r.z) / (p.A p); x += alpha p, r -= alpha q; partial sums of r.r.
__global__ __launch_bounds__(256) void k_update_xr_a(double* __restrict__ x,
                                                     double* __restrict__ r,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q, int n,
                                                     const double* __restrict__ pq_part, int npq,
                                                     const double* __restrict__ rz_part, int nrz,
                                                     PcgScalars* __restrict__ sc,
                                                     double* __restrict__ alphas,
                                                     double* __restrict__ rr_part,
                                                     const int* __restrict__ done) {
  if (*done) return;
  __shared__ double sh[8];
  const double pq = allsum_partials(pq_part, npq, sh);
  const double rz = allsum_partials(rz_part, nrz, sh);
  const double alpha = rz / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->pq = pq;
    sc->rz = rz;
    sc->alpha = alpha;
    alphas[sc->iters] = alpha;
    sc->iters += 1;
  }
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) rr_part[blockIdx.x] = s;
}

// Convergence check on r.r, then the first pieces of the apply: blocks
// [0, ngather) gather the scaled local vectors, the next nrestrict blocks
// form the coarse restriction of one subdomain each.
__global__ __launch_bounds__(256) void k_check_apply_in(const double* __restrict__ r,
                                                        const int* __restrict__ dglob,
                                                        const double* __restrict__ dscale,
                                                        int64_t nvec, double* __restrict__ xl,
                                                        int ngather, const double* __restrict__ Z,
                                                        const int* __restrict__ zoff,
                                                        const int* __restrict__ m,
                                                        const int* __restrict__ nd,
                                                        const int* __restrict__ dvoff,
                                                        const int* __restrict__ coff,
                                                        double* __restrict__ rH,
                                                        const double* __restrict__ rr_part, int nrr,
                                                        PcgScalars* __restrict__ sc,
                                                        int* __restrict__ done) {
  if (*done) return;
  __shared__ double sh[8];
  const double rr = allsum_partials(rr_part, nrr, sh);
  const bool conv = rr <= sc->tol2;
  const bool stop = conv || sc->iters >= sc->maxit || !(rr == rr);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rr = rr;
    if (conv) sc->converged = 1;
    if (stop) *done = 1;
  }
  if (stop) return;
  if ((int)blockIdx.x < ngather) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < nvec) {
      const int g = dglob[e];
      xl[e] = g >= 0 ? dscale[e] * r[g] : 0.0;
    }
  } else {
    restrict_block(blockIdx.x - ngather, r, Z, zoff, m, nd, dglob, dvoff, coff, rH);
  }
}

// One launch for the start of a PCG iteration: beta = (r.z)_new / (r.z)_old
// (none on the first iteration, where p = z), p = z + beta p, q = A p and
// the partial sums of p.q.  A row needs p at its neighbours: those entries
// are formed again from z and the previous p, which stays untouched in the
// other buffer (pin and pout alternate between iterations), so no block
// reads an entry that another block rewrites; every copy of an entry is the
// same expression of the same inputs, hence the same value.  LPR lanes per
// row in the summation order of k_spmv; the block takes row groups in
// grid-stride order and leaves its rows' p.q in pq_part[blockIdx.x].
template <int LPR>
__global__ __launch_bounds__(256) void k_p_spmv(int n, const int* __restrict__ rp,
                                                const int* __restrict__ col,
                                                const double* __restrict__ val,
                                                const double* __restrict__ z,
                                                const double* __restrict__ pin,
                                                double* __restrict__ pout, double* __restrict__ q,
                                                const double* __restrict__ rz_part, int nrz,
                                                PcgScalars* __restrict__ sc,
                                                double* __restrict__ betas,
                                                double* __restrict__ pq_part,
                                                const int* __restrict__ done) {
  if (*done) return;
  __shared__ double sh[8];
  const int it = sc->iters;
  double beta = 0.0;
  if (it > 0) {
    beta = allsum_partials(rz_part, nrz, sh) / sc->rz;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->beta = beta;
      betas[it - 1] = beta;
    }
  }
  auto pnew = [&](int j) { return it > 0 ? z[j] + beta * pin[j] : z[j]; };
  constexpr int RPB = 256 / LPR;  // rows per block and pass
  const int sub = threadIdx.x % LPR;
  double dot = 0.0;
  for (int r0 = blockIdx.x * RPB; r0 < n; r0 += gridDim.x * RPB) {
    const int row = r0 + threadIdx.x / LPR;
    double s = 0.0;
    if (row < n) {
      const int p1 = rp[row + 1];
      // batches of 4 entries per lane, as in k_spmv
      for (int k = rp[row] + sub; k < p1; k += 4 * LPR) {
        int cc[4];
        double vv[4], pv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = min(k + u * LPR, p1 - 1);
          cc[u] = col[q];
          vv[u] = val[q];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) pv[u] = pnew(cc[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (k + u * LPR < p1) s += vv[u] * pv[u];
      }
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR);
    if (row < n && sub == 0) {
      const double pr = pnew(row);
      pout[row] = pr;
      q[row] = s;
      dot += pr * s;
    }
  }
  dot = block_sum(dot, sh);
  if (threadIdx.x == 0) pq_part[blockIdx.x] = dot;
}

hipError_t p_spmv(const geneo_csr_t* A, int lpr, const double* z, const double* pin,
                  double* pout, double* q, const double* rz_part, int nrz, PcgScalars* sc,
                  double* betas, double* pq_part, int npq, const int* done, hipStream_t st) {
  const dim3 grid(npq), blk(256);
  const int n = A->n;
#define GENEO_P_SPMV(L)                                                                        \
  hipLaunchKernelGGL(k_p_spmv<L>, grid, blk, 0, st, n, A->rowptr, A->col, A->val, z, pin, pout, \
                     q, rz_part, nrz, sc, betas, pq_part, done)
  switch (lpr) {
    case 4: GENEO_P_SPMV(4); break;
    case 8: GENEO_P_SPMV(8); break;
    case 16: GENEO_P_SPMV(16); break;
    default: GENEO_P_SPMV(32); break;
  }
#undef GENEO_P_SPMV
  return hipGetLastError();
}

hipError_t update_xr_alpha(double* x, double* r, const double* p, const double* q, int n,
                           const double* pq_part, int npq, const double* rz_part, int nrz,
                           PcgScalars* sc, double* alphas, double* rr_part, const int* done,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_update_xr_a, dim3(PCG_NB), dim3(256), 0, st, x, r, p, q, n, pq_part, npq,
                     rz_part, nrz, sc, alphas, rr_part, done);
  return hipGetLastError();
}

hipError_t check_apply_in(const double* r, const int* dglob, const double* dscale, int64_t nvec,
                          double* xl, const double* Z, const int* zoff, const int* m, const int* nd,
                          const int* dvoff, const int* coff, double* rH, int nrestrict,
                          const double* rr_part, PcgScalars* sc, int* done, hipStream_t st) {
  const int ngather = (int)((nvec + 255) / 256);
  hipLaunchKernelGGL(k_check_apply_in, dim3(ngather + nrestrict), dim3(256), 0, st, r, dglob,
                     dscale, nvec, xl, ngather, Z, zoff, m, nd, dvoff, coff, rH, rr_part, PCG_NB,
                     sc, done);
  return hipGetLastError();
}

// r = b - q (q = A x0), used to start the iteration
__global__ void k_residual0(const double* __restrict__ b, const double* __restrict__ q,
                            double* __restrict__ r, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - q[i];
}

hipError_t residual0(const double* b, const double* q, double* r, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_residual0, dim3((n + 255) / 256), dim3(256), 0, st, b, q, r, n);
  return hipGetLastError();
}

// r = b - A x with each row's sum carried to twice the working precision
// and rounded once at the end: error-free products (p + e = a x exactly,
// e by a fused multiply-add) and error-free sums (Knuth's TwoSum) as in
// the Dot2 algorithm of Ogita, Rump and Oishi ("Accurate sum and dot
// product", SIAM J. Sci. Comput. 26, 2005).  The explicit _rn operations
// keep the compiler from contracting the products into the sums.  LPR
// lanes per row, each over every LPR-th entry, their double-double partial
// sums combined in a fixed order: used a few times per solve, for the
// residuals of iterative refinement and the reported true residual.
template <int LPR>
__global__ __launch_bounds__(256) void k_residual_dd(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ r) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) / LPR, sub = threadIdx.x % LPR;
  // lane sub of row i: b_i (lane 0) minus its share of the entries (every
  // LPR-th), as a double-double (s, c)
  double s = 0.0, c = 0.0;
  if (i < n) {
    if (sub == 0) s = b[i];
    for (int k = rp[i] + sub; k < rp[i + 1]; k += LPR) {
      const double a = val[k], xv = x[col[k]];
      const double p = __dmul_rn(a, xv);
      const double ep = fma(a, xv, -p);            // a xv = p + ep
      const double t = __dadd_rn(s, -p);
      const double bv = __dsub_rn(t, s);
      const double es = __dadd_rn(__dsub_rn(s, __dsub_rn(t, bv)), __dsub_rn(-p, bv));  // s - p = t + es
      s = t;
      c = __dadd_rn(c, __dsub_rn(es, ep));
    }
  }
  // the lanes' pairs added in a fixed tree: s by an error-free sum (the
  // same in both lanes of each exchange), the errors into c
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) {
    const double s2 = __shfl_xor(s, o, LPR), c2 = __shfl_xor(c, o, LPR);
    const double t = __dadd_rn(s, s2);
    const double bv = __dsub_rn(t, s);
    const double e = __dadd_rn(__dsub_rn(s, __dsub_rn(t, bv)), __dsub_rn(s2, bv));
    s = t;
    c = __dadd_rn(__dadd_rn(c, c2), e);
  }
  if (i < n && sub == 0) r[i] = __dadd_rn(s, c);
}

hipError_t residual_dd(const geneo_csr_t* A, const double* b, const double* x, double* r,
                       hipStream_t st) {
  constexpr int LPR = 8;
  hipLaunchKernelGGL(k_residual_dd<LPR>, dim3((A->n + 256 / LPR - 1) / (256 / LPR)), dim3(256), 0,
                     st, A->n, A->rowptr, A->col, A->val, b, x, r);
  return hipGetLastError();
}

// x += d
__global__ void k_add_into(double* __restrict__ x, const double* __restrict__ d, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += d[i];
}

hipError_t add_into(double* x, const double* d, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_add_into, dim3((n + 255) / 256), dim3(256), 0, st, x, d, n);
  return hipGetLastError();
}

// Fill kernel used instead of memset inside code a caller may capture.
__global__ void k_fill_i32(int* __restrict__ p, int v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t fill_i32(int* p, int v, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

}  // namespace geneo
