// Triangular products and solves with the packed tile factors.
//
//  * k_trmv_lower / k_trmv_upperT: t = X x and y = X^T t for the inverse
//    factors X = L^{-1} of the local Dirichlet matrices (and of the coarse
//    matrix).  One wavefront per (matrix, tile row) resp. (matrix, tile
//    column); loads are whole 64-byte row segments (lower) or coalesced row
//    reads by 32 lanes (transposed); accumulation in FP64.  These stream
//    the factors once each and are HBM-bound.
//  * k_trsm_fwd / k_trsm_bwd: X = G^{-1} R and X = G^{-T} R with b right-hand
//    sides for the shift-and-invert eigen sweeps (FP64, one workgroup per
//    subdomain, blocked substitution with the inverted diagonal tiles and
//    MFMA quadrant products split over tile slices).
//  * k_bapply: Y = X_j A^o_j X_j X (the B-matrix of the GenEO eigenproblem).
#include "internal.h"

namespace geneo {

template <typename T> struct Seg16;
template <> struct Seg16<float> {
  static __device__ __forceinline__ void load(const float* p, double* o) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float4 v = q[u];
      o[4 * u + 0] = v.x; o[4 * u + 1] = v.y; o[4 * u + 2] = v.z; o[4 * u + 3] = v.w;
    }
  }
};
template <> struct Seg16<double> {
  static __device__ __forceinline__ void load(const double* p, double* o) {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      double2 v = q[u];
      o[2 * u + 0] = v.x; o[2 * u + 1] = v.y;
    }
  }
};

template <typename T>
__global__ __launch_bounds__(64) void k_trmv_lower(const T* __restrict__ X,
                                                   const int64_t* __restrict__ toff,
                                                   const int* __restrict__ ntl,
                                                   const int* __restrict__ voff,
                                                   const int* __restrict__ jobs,
                                                   const double* __restrict__ xin,
                                                   double* __restrict__ tout,
                                                   const int* __restrict__ done) {
  if (done && *done) return;
  const int j = jobs[blockIdx.y];
  const int i = blockIdx.x;
  const int nt = ntl[j];
  if (i >= nt) return;
  const int lane = threadIdx.x, row = lane >> 1, half = lane & 1;
  const T* Xr = X + (toff[j] + tile_idx(i, 0)) * TSQ + row * TS + half * 16;
  const double* xv = xin + voff[j] + half * 16;
  double s = 0.0;
  for (int k = 0; k <= i; ++k) {
    double m[16];
    Seg16<T>::load(Xr + (int64_t)k * TSQ, m);
    const double* xk = xv + k * TS;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += m[q] * xk[q];
  }
  s += __shfl_xor(s, 1);
  if (half == 0) tout[voff[j] + i * TS + row] = s;
}

template <typename T>
__global__ __launch_bounds__(64) void k_trmv_upperT(const T* __restrict__ X,
                                                    const int64_t* __restrict__ toff,
                                                    const int* __restrict__ ntl,
                                                    const int* __restrict__ voff,
                                                    const int* __restrict__ jobs,
                                                    const double* __restrict__ tin,
                                                    double* __restrict__ yout,
                                                    const int* __restrict__ done) {
  if (done && *done) return;
  const int j = jobs[blockIdx.y];
  const int k = blockIdx.x;
  const int nt = ntl[j];
  if (k >= nt) return;
  const int lane = threadIdx.x, c = lane & 31, h = lane >> 5;
  const T* base = X + toff[j] * TSQ + (h * 16) * TS + c;
  const double* tv = tin + voff[j] + h * 16;
  double s = 0.0;
  for (int i = k; i < nt; ++i) {
    const T* tile = base + tile_idx(i, k) * TSQ;
    const double* ti = tv + i * TS;
#pragma unroll
    for (int r = 0; r < 16; ++r) s += (double)tile[r * TS] * ti[r];
  }
  s += __shfl_xor(s, 32);
  if (h == 0) yout[voff[j] + k * TS + c] = s;
}

hipError_t trmv_lower(bool fp32, const void* X, const int64_t* toff, const int* nt,
                      const int* voff, const int* jobs, int njobs, int maxnt, const double* xin,
                      double* tout, const int* done, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  dim3 grid(maxnt, njobs);
  if (fp32)
    hipLaunchKernelGGL(k_trmv_lower<float>, grid, dim3(64), 0, st, (const float*)X, toff, nt,
                       voff, jobs, xin, tout, done);
  else
    hipLaunchKernelGGL(k_trmv_lower<double>, grid, dim3(64), 0, st, (const double*)X, toff, nt,
                       voff, jobs, xin, tout, done);
  return hipGetLastError();
}

hipError_t trmv_upperT(bool fp32, const void* X, const int64_t* toff, const int* nt,
                       const int* voff, const int* jobs, int njobs, int maxnt, const double* tin,
                       double* yout, const int* done, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  dim3 grid(maxnt, njobs);
  if (fp32)
    hipLaunchKernelGGL(k_trmv_upperT<float>, grid, dim3(64), 0, st, (const float*)X, toff, nt,
                       voff, jobs, tin, yout, done);
  else
    hipLaunchKernelGGL(k_trmv_upperT<double>, grid, dim3(64), 0, st, (const double*)X, toff, nt,
                       voff, jobs, tin, yout, done);
  return hipGetLastError();
}

// ------------------------------------------------ multi-RHS substitution ---
// Work split for b = 16*ncq right-hand sides: nq = 2*ncq output quadrants of
// a 32 x b tile, ns = 16/nq tile slices of the inner sum.
#define TRSM_WAVES 16
#define TRSM_MAXB 64

__device__ __forceinline__ void trsm_split(int b, int& ncq, int& nq, int& ns) {
  ncq = b / 16;
  nq = 2 * ncq;
  ns = TRSM_WAVES / nq;
  if (ns < 1) ns = 1;
}

// Reduce the per-wave partial quadrants into sacc = Rblk - sum (32 x b).
__device__ __forceinline__ void trsm_reduce(double (*spart)[256], double (*sacc)[TRSM_MAXB + 1],
                                            const double* Rblk, int b, int ncq, int nq, int ns,
                                            bool transposeless) {
  for (int t = threadIdx.x; t < TS * b; t += blockDim.x) {
    int r = t / b, cc = t % b;
    int qd = (r >> 4) * ncq + (cc >> 4);
    double s = 0.0;
    for (int sl = 0; sl < ns; ++sl) s += spart[qd + sl * nq][(r & 15) * 16 + (cc & 15)];
    sacc[r][cc] = Rblk[r * b + cc] - s;
  }
}

__global__ __launch_bounds__(1024) void k_trsm_fwd(const double* __restrict__ G,
                                                   const double* __restrict__ dinv,
                                                   const int64_t* __restrict__ toff,
                                                   const int64_t* __restrict__ doff,
                                                   const int* __restrict__ ntl,
                                                   const int* __restrict__ voff, int b,
                                                   const double* __restrict__ R,
                                                   double* __restrict__ X,
                                                   const int* __restrict__ active) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  __shared__ double spart[TRSM_WAVES][256];
  __shared__ double sacc[TS][TRSM_MAXB + 1];
  const int nt = ntl[j];
  const double* Gj = G + toff[j] * TSQ;
  const double* Dj = dinv + doff[j] * TSQ;
  const double* Rj = R + (int64_t)voff[j] * b;
  double* Xj = X + (int64_t)voff[j] * b;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int ncq, nq, ns;
  trsm_split(b, ncq, nq, ns);
  const int qd = w % nq, sl = w / nq;
  const int rq = qd / ncq, cq = qd % ncq;
  const bool worker = sl < ns;
  for (int i = 0; i < nt; ++i) {
    d4_t acc = acc_zero<double>();
    if (worker)
      for (int k = sl; k < i; k += ns)
        q_xy<double>(acc, Gj + tile_idx(i, k) * TSQ + rq * 16 * TS, TS,
                     Xj + (int64_t)k * TS * b + cq * 16, b, lane);
    if (w < TRSM_WAVES) {
#pragma unroll
      for (int v = 0; v < 4; ++v) spart[w][acc_row<double>(lane, v) * 16 + acc_col(lane)] = worker ? acc[v] : 0.0;
    }
    block_sync();
    trsm_reduce(spart, sacc, Rj + (int64_t)i * TS * b, b, ncq, nq, ns, true);
    block_sync();
    if (w < nq) {
      d4_t o = acc_zero<double>();
      q_xy<double>(o, Dj + (int64_t)i * TSQ + rq * 16 * TS, TS, &sacc[0][cq * 16],
                   TRSM_MAXB + 1, lane);
      double* out = Xj + ((int64_t)i * TS + rq * 16) * b + cq * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[acc_row<double>(lane, v) * b + acc_col(lane)] = o[v];
    }
    block_sync();
  }
}

__global__ __launch_bounds__(1024) void k_trsm_bwd(const double* __restrict__ G,
                                                   const double* __restrict__ dinv,
                                                   const int64_t* __restrict__ toff,
                                                   const int64_t* __restrict__ doff,
                                                   const int* __restrict__ ntl,
                                                   const int* __restrict__ voff, int b,
                                                   const double* __restrict__ R,
                                                   double* __restrict__ X,
                                                   const int* __restrict__ active) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  __shared__ double spart[TRSM_WAVES][256];
  __shared__ double sacc[TS][TRSM_MAXB + 1];
  const int nt = ntl[j];
  const double* Gj = G + toff[j] * TSQ;
  const double* Dj = dinv + doff[j] * TSQ;
  const double* Rj = R + (int64_t)voff[j] * b;
  double* Xj = X + (int64_t)voff[j] * b;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int ncq, nq, ns;
  trsm_split(b, ncq, nq, ns);
  const int qd = w % nq, sl = w / nq;
  const int rq = qd / ncq, cq = qd % ncq;
  const bool worker = sl < ns;
  for (int k = nt - 1; k >= 0; --k) {
    d4_t acc = acc_zero<double>();
    // sum_{i>k} G_ik^T X_i : contraction over the rows of G_ik
    if (worker)
      for (int i = k + 1 + sl; i < nt; i += ns)
        q_xTy<double>(acc, Gj + tile_idx(i, k) * TSQ + rq * 16, TS,
                      Xj + (int64_t)i * TS * b + cq * 16, b, lane);
    if (w < TRSM_WAVES) {
#pragma unroll
      for (int v = 0; v < 4; ++v) spart[w][acc_row<double>(lane, v) * 16 + acc_col(lane)] = worker ? acc[v] : 0.0;
    }
    block_sync();
    trsm_reduce(spart, sacc, Rj + (int64_t)k * TS * b, b, ncq, nq, ns, true);
    block_sync();
    if (w < nq) {
      d4_t o = acc_zero<double>();
      q_xTy<double>(o, Dj + (int64_t)k * TSQ + rq * 16, TS, &sacc[0][cq * 16], TRSM_MAXB + 1,
                    lane);
      double* out = Xj + ((int64_t)k * TS + rq * 16) * b + cq * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[acc_row<double>(lane, v) * b + acc_col(lane)] = o[v];
    }
    block_sync();
  }
}

hipError_t launch_trsm_fwd(const double* G, const double* dinv, const int64_t* toff,
                           const int64_t* doff, const int* nt, const int* voff, int nsub, int b,
                           const double* R, double* X, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_trsm_fwd, dim3(nsub), dim3(1024), 0, st, G, dinv, toff, doff, nt, voff, b,
                     R, X, active);
  return hipGetLastError();
}

hipError_t launch_trsm_bwd(const double* G, const double* dinv, const int64_t* toff,
                           const int64_t* doff, const int* nt, const int* voff, int nsub, int b,
                           const double* R, double* X, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_trsm_bwd, dim3(nsub), dim3(1024), 0, st, G, dinv, toff, doff, nt, voff, b,
                     R, X, active);
  return hipGetLastError();
}

// Y = X_j A^o_j X_j X over the padded N_j rows (zero on padding).
__global__ __launch_bounds__(256) void k_bapply(const int* __restrict__ sub_ptr,
                                                const double* __restrict__ pou,
                                                const int* __restrict__ rp,
                                                const int* __restrict__ colx,
                                                const double* __restrict__ val,
                                                const int* __restrict__ voff,
                                                const int* __restrict__ ntl, int b,
                                                const double* __restrict__ X,
                                                double* __restrict__ Y,
                                                const int* __restrict__ active) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  const int npad = ntl[j] * TS;
  const double* Xj = X + (int64_t)voff[j] * b;
  double* Yj = Y + (int64_t)voff[j] * b;
  for (int t = threadIdx.x; t < npad * b; t += blockDim.x) {
    int a = t / b, c = t % b;
    double s = 0.0;
    if (a < n) {
      double mua = pou[s0 + a];
      if (mua != 0.0) {
        for (int p = rp[s0 + a]; p < rp[s0 + a + 1]; ++p) {
          int q = colx[p];
          s += val[p] * pou[s0 + q] * Xj[(int64_t)q * b + c];
        }
        s *= mua;
      }
    }
    Yj[(int64_t)a * b + c] = s;
  }
}

hipError_t launch_bapply(const int* sub_ptr, const double* pou, const geneo_csr_batch_t* Ao,
                         const int* voff, const int* nt, int nsub, int b, const double* X,
                         double* Y, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_bapply, dim3(nsub), dim3(256), 0, st, sub_ptr, pou, Ao->rowptr, Ao->col,
                     Ao->val, voff, nt, b, X, Y, active);
  return hipGetLastError();
}

}  // namespace geneo
