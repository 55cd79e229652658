// Dense Cholesky factorisations on the matrix cores (16x16x4 MFMA).
//
//  * k_chol_batched: one workgroup (16 wavefronts) per local matrix,
//    left-looking over tile columns: update column k with the finished
//    columns to its left (quadrant MFMA products), factor the diagonal tile
//    in LDS (one wavefront), invert it, and finish the column by
//    multiplying with the inverse diagonal tile.  A failed pivot test stops
//    that matrix and records the failing row in `status`.
//  * k_trtri: X = L^{-1}, one workgroup per (matrix, tile column c): the
//    column c of X solves L X_c = E_c by blocked forward substitution.
//  * coarse_cholesky: right-looking tiled factorisation of the single coarse
//    matrix, one launch per phase (diagonal, panel, trailing update) so that
//    the trailing update spreads over the whole chip.
#include "internal.h"

namespace geneo {

// Cholesky of the TS x TS tile held in sL (lower triangle used), in place,
// plus its inverse in sI; executed by one wavefront.  Returns true when a
// pivot d fails d > pivtol.
template <typename T, int LDI>
__device__ bool diag_factor_wave(T (*sL)[TS + 1], T (*sI)[LDI], int lane, double pivtol) {
  bool fail = false;
  for (int c = 0; c < TS; ++c) {
    T d = sL[c][c];
    if (!(d > (T)pivtol)) fail = true;
    T s = sqrt(d > (T)0 ? d : (T)1);
    wave_sync();
    if (lane > c && lane < TS) sL[lane][c] /= s;
    if (lane == c) sL[c][c] = s;
    wave_sync();
    for (int e = lane; e < TSQ; e += 64) {
      int r = e / TS, q = e % TS;
      if (q > c && q <= r) sL[r][q] -= sL[r][c] * sL[q][c];
    }
    wave_sync();
  }
  // inverse: lane t < TS solves L x = e_t (column t of L^{-1}); no lane reads
  // another lane's output
  if (lane < TS) {
    const int t = lane;
    for (int r = 0; r < TS; ++r) {
      T x = (T)0;
      if (r >= t) {
        T s = (r == t) ? (T)1 : (T)0;
        for (int q = t; q < r; ++q) s -= sL[r][q] * sI[q][t];
        x = s / sL[r][r];
      }
      sI[r][t] = x;
    }
  }
  wave_sync();
  return fail;
}

// LDS row stride for 32-column tiles: 34 elements keeps the fragment reads
// of one wavefront (16 rows x 4 columns) free of bank conflicts for both
// 4- and 8-byte elements.
#define LDS_LD (TS + 2)
// Row-k tiles staged per chunk in the update phase (bytes: CH * TS * LDS_LD
// * sizeof(T)); 8 FP64 tiles = 68 KB.
#define CHOL_CH 8

template <typename T>
__global__ __launch_bounds__(1024) void k_chol_batched(T* __restrict__ tiles,
                                                       const int64_t* __restrict__ toff,
                                                       const int* __restrict__ ntl,
                                                       T* __restrict__ dinv,
                                                       const int64_t* __restrict__ doff,
                                                       int* __restrict__ status,
                                                       const int* __restrict__ jobs,
                                                       double pivtol) {
  const int j = jobs[blockIdx.x];
  const int nt = ntl[j];
  T* A = tiles + toff[j] * TSQ;
  T* Di = dinv + doff[j] * TSQ;
  __shared__ T sRow[CHOL_CH][TS][LDS_LD];
  __shared__ T sL[TS][TS + 1];
  __shared__ T sI[TS][LDS_LD];
  __shared__ int sfail;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  const int fi = lane & 15, fk = lane >> 4;  // fragment row / k-offset of this lane
  if (tid == 0) sfail = 0;
  for (int k = 0; k < nt; ++k) {
    // 1. A_ik -= sum_{jj<k} L_i,jj L_k,jj^T for i >= k.  Work item = 16-row
    //    half of an output tile (both 16-column quadrants); the row-k tiles
    //    L_k,jj are staged in LDS chunk by chunk and shared by all items.
    if (k > 0) {
      const int nit = 2 * (nt - k);
      const int rounds = (nit + nw - 1) / nw;
      for (int rd = 0; rd < rounds; ++rd) {
        const int it = rd * nw + w;
        const bool active = it < nit;
        const int i = k + (it >> 1), rq = it & 1;
        typename Mfma<T>::acc a0 = acc_zero<T>(), a1 = acc_zero<T>();
        const T* X = A + tile_idx(active ? i : k, 0) * TSQ + rq * 16 * TS;
        for (int c0 = 0; c0 < k; c0 += CHOL_CH) {
          const int cn = min(CHOL_CH, k - c0);
          block_sync();
          const T* Rsrc = A + tile_idx(k, c0) * TSQ;   // tiles (k, c0 .. c0+cn-1) are contiguous
          for (int e = tid; e < cn * TSQ; e += blockDim.x) {
            int t = e / TSQ, r = (e % TSQ) / TS, c = e % TS;
            sRow[t][r][c] = Rsrc[e];
          }
          block_sync();
          if (active) {
            for (int t = 0; t < cn; ++t) {
              const T* Xt = X + (int64_t)(c0 + t) * TSQ;
#pragma unroll
              for (int kk = 0; kk < 8; ++kk) {
                T av = Xt[fi * TS + kk * 4 + fk];
                a0 = Mfma<T>::run(av, sRow[t][fi][kk * 4 + fk], a0);
                a1 = Mfma<T>::run(av, sRow[t][16 + fi][kk * 4 + fk], a1);
              }
            }
          }
        }
        if (active) {
          T* C = A + tile_idx(i, k) * TSQ + rq * 16 * TS;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = acc_row<T>(lane, v);
            C[r * TS + acc_col(lane)] -= a0[v];
            C[r * TS + 16 + acc_col(lane)] -= a1[v];
          }
        }
      }
    }
    block_sync();
    // 2. diagonal tile: factor and invert (wavefront 0)
    if (w == 0) {
      T* D = A + tile_idx(k, k) * TSQ;
      for (int e = lane; e < TSQ; e += 64) sL[e / TS][e % TS] = D[e];
      wave_sync();
      bool fail = diag_factor_wave<T, LDS_LD>(sL, sI, lane, pivtol);
      for (int e = lane; e < TSQ; e += 64) {
        int r = e / TS, q = e % TS;
        D[e] = q <= r ? sL[r][q] : (T)0;
        Di[(int64_t)k * TSQ + e] = q <= r ? sI[r][q] : (T)0;
      }
      if (fail && lane == 0) {
        sfail = 1;
        status[j] = 1 + k * TS;
      }
    }
    block_sync();
    if (sfail) return;
    // 3. L_ik = A_ik Linv_kk^T for i > k; one wavefront owns 16 full rows
    const int nit2 = 2 * (nt - k - 1);
    for (int it = w; it < nit2; it += nw) {
      const int i = k + 1 + (it >> 1), rq = it & 1;
      T* X = A + tile_idx(i, k) * TSQ + rq * 16 * TS;
      typename Mfma<T>::acc a0 = acc_zero<T>(), a1 = acc_zero<T>();
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        T av = X[fi * TS + kk * 4 + fk];
        a0 = Mfma<T>::run(av, sI[fi][kk * 4 + fk], a0);
        a1 = Mfma<T>::run(av, sI[16 + fi][kk * 4 + fk], a1);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        X[acc_row<T>(lane, v) * TS + acc_col(lane)] = a0[v];
        X[acc_row<T>(lane, v) * TS + 16 + acc_col(lane)] = a1[v];
      }
    }
    block_sync();
  }
  if (tid == 0) status[j] = 0;
}

hipError_t launch_chol_batched(bool fp32, void* tiles, const int64_t* toff, const int* nt,
                               void* dinv, const int64_t* doff, int* status, const int* jobs,
                               int njobs, double pivtol, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_chol_batched<float>, dim3(njobs), dim3(1024), 0, st, (float*)tiles,
                       toff, nt, (float*)dinv, doff, status, jobs, pivtol);
  else
    hipLaunchKernelGGL(k_chol_batched<double>, dim3(njobs), dim3(1024), 0, st, (double*)tiles,
                       toff, nt, (double*)dinv, doff, status, jobs, pivtol);
  return hipGetLastError();
}

// X = L^{-1} for tile column c of matrix j (jobs[b] = (j, c)).
template <typename T>
__global__ __launch_bounds__(256) void k_trtri(const T* __restrict__ L, const T* __restrict__ dinv,
                                               T* __restrict__ X, const int64_t* __restrict__ toff,
                                               const int64_t* __restrict__ doff,
                                               const int* __restrict__ ntl,
                                               const int2* __restrict__ jobs) {
  const int j = jobs[blockIdx.x].x, c = jobs[blockIdx.x].y;
  const int nt = ntl[j];
  const T* Lj = L + toff[j] * TSQ;
  const T* Dj = dinv + doff[j] * TSQ;
  T* Xj = X + toff[j] * TSQ;
  __shared__ T sacc[TS][TS + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int rq = w >> 1, cq = w & 1;
  for (int e = tid; e < TSQ; e += blockDim.x) Xj[tile_idx(c, c) * TSQ + e] = Dj[(int64_t)c * TSQ + e];
  block_sync();
  for (int i = c + 1; i < nt; ++i) {
    typename Mfma<T>::acc acc = acc_zero<T>();
    for (int k = c; k < i; ++k)
      q_xy<T>(acc, Lj + tile_idx(i, k) * TSQ + rq * 16 * TS, TS,
              Xj + tile_idx(k, c) * TSQ + cq * 16, TS, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) sacc[rq * 16 + acc_row<T>(lane, v)][cq * 16 + acc_col(lane)] = -acc[v];
    block_sync();
    typename Mfma<T>::acc o = acc_zero<T>();
    q_xy<T>(o, Dj + (int64_t)i * TSQ + rq * 16 * TS, TS, &sacc[0][cq * 16], TS + 1, lane);
    T* out = Xj + tile_idx(i, c) * TSQ + rq * 16 * TS + cq * 16;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[acc_row<T>(lane, v) * TS + acc_col(lane)] = o[v];
    block_sync();
  }
}

hipError_t launch_trtri(bool fp32, const void* L, const void* dinv, void* X,
                        const int64_t* toff, const int64_t* doff, const int* nt,
                        const int2* jobs, int njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_trtri<float>, dim3(njobs), dim3(256), 0, st, (const float*)L,
                       (const float*)dinv, (float*)X, toff, doff, nt, jobs);
  else
    hipLaunchKernelGGL(k_trtri<double>, dim3(njobs), dim3(256), 0, st, (const double*)L,
                       (const double*)dinv, (double*)X, toff, doff, nt, jobs);
  return hipGetLastError();
}

// ------------------------------------------------------- coarse matrix ---
__global__ __launch_bounds__(64) void k_cpotrf(double* __restrict__ A, double* __restrict__ Di,
                                               int k, int* __restrict__ status) {
  __shared__ double sL[TS][TS + 1];
  __shared__ double sI[TS][TS + 1];
  const int lane = threadIdx.x;
  if (*status) return;
  double* D = A + tile_idx(k, k) * TSQ;
  for (int e = lane; e < TSQ; e += 64) sL[e / TS][e % TS] = D[e];
  wave_sync();
  bool fail = diag_factor_wave<double, TS + 1>(sL, sI, lane, 0.0);
  for (int e = lane; e < TSQ; e += 64) {
    int r = e / TS, q = e % TS;
    D[e] = q <= r ? sL[r][q] : 0.0;
    Di[(int64_t)k * TSQ + e] = q <= r ? sI[r][q] : 0.0;
  }
  if (fail && lane == 0) *status = 1 + k * TS;
}

// L_ik = A_ik Linv_kk^T, one workgroup per tile i > k
__global__ __launch_bounds__(256) void k_ctrsm(double* __restrict__ A,
                                               const double* __restrict__ Di, int k,
                                               const int* __restrict__ status) {
  if (*status) return;
  const int i = k + 1 + blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rq = w >> 1, cq = w & 1;
  double* X = A + tile_idx(i, k) * TSQ;
  const double* Y = Di + (int64_t)k * TSQ;
  d4_t acc = acc_zero<double>();
  q_xyT<double>(acc, X + rq * 16 * TS, TS, Y + cq * 16 * TS, TS, lane);
  block_sync();
#pragma unroll
  for (int v = 0; v < 4; ++v) X[(rq * 16 + acc_row<double>(lane, v)) * TS + cq * 16 + acc_col(lane)] = acc[v];
}

// A_ij -= L_ik L_jk^T for k < j <= i; blockIdx.x enumerates the trailing tiles
__global__ __launch_bounds__(256) void k_cupdate(double* __restrict__ A, int k, int nt,
                                                 const int* __restrict__ status) {
  if (*status) return;
  // map blockIdx.x -> (i, j) over the lower triangle of the trailing matrix
  int t = blockIdx.x;
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
  while ((int64_t)i * (i + 1) / 2 > t) --i;
  int jj = t - i * (i + 1) / 2;
  i += k + 1;
  jj += k + 1;
  if (i >= nt) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rq = w >> 1, cq = w & 1;
  if (i == jj && rq == 0 && cq == 1) return;
  d4_t acc = acc_zero<double>();
  q_xyT<double>(acc, A + tile_idx(i, k) * TSQ + rq * 16 * TS, TS,
                A + tile_idx(jj, k) * TSQ + cq * 16 * TS, TS, lane);
  double* C = A + tile_idx(i, jj) * TSQ + rq * 16 * TS + cq * 16;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[acc_row<double>(lane, v) * TS + acc_col(lane)] -= acc[v];
}

hipError_t coarse_cholesky(double* tiles, double* dinv, int nt, int* status, hipStream_t st) {
  hipError_t e = hipMemsetAsync(status, 0, sizeof(int), st);
  if (e != hipSuccess) return e;
  for (int k = 0; k < nt; ++k) {
    hipLaunchKernelGGL(k_cpotrf, dim3(1), dim3(64), 0, st, tiles, dinv, k, status);
    int rem = nt - k - 1;
    if (rem > 0) {
      hipLaunchKernelGGL(k_ctrsm, dim3(rem), dim3(256), 0, st, tiles, dinv, k, status);
      int nupd = rem * (rem + 1) / 2;
      hipLaunchKernelGGL(k_cupdate, dim3(nupd), dim3(256), 0, st, tiles, k, nt, status);
    }
  }
  return hipGetLastError();
}

}  // namespace geneo
