// Batched GenEO eigen solve, one workgroup per subdomain.
//
// The pencil A_N p = lambda B p (B = X A^o X, Sec. 4.3) is turned into the
// symmetric problem S y = nu y, S = G^{-1} B G^{-T}, C = A_N - sigma B = G G^T,
// nu = 1/(lambda - sigma), p = G^{-T} y (shift-and-invert, Sec. 4.4).  The
// largest nu are found by block subspace iteration with Rayleigh-Ritz:
//
//   W = S U;  H = U^T W;  H = Q Theta Q^T;  residuals of (U Q, Theta) from
//   W Q - U Q Theta;  U <- orth(W Q)
//
// with orth = two passes of Cholesky QR (columns first scaled to unit
// norm; a column whose pivot collapses is replaced by a fresh pseudo-random
// vector).  The small symmetric eigenproblems use cyclic Jacobi in LDS.
#include "internal.h"

namespace geneo {

#define EIG_WAVES 16
#define EIG_MAXB 64

// ---------------------------------------------------------- start block ---
__global__ void k_eig_init(double* __restrict__ U, const int* __restrict__ sub_ptr,
                           const int* __restrict__ voff, const int* __restrict__ ntl, int b,
                           uint64_t seed) {
  const int j = blockIdx.x;
  const int n = sub_ptr[j + 1] - sub_ptr[j];
  const int npad = ntl[j] * TS;
  double* Uj = U + (int64_t)voff[j] * b;
  for (int t = threadIdx.x; t < npad * b; t += blockDim.x) {
    int a = t / b, c = t % b;
    (void)n;
    Uj[t] = hash_uniform(seed, (uint64_t)j, (uint64_t)a * 977 + c);
  }
}

hipError_t launch_eig_init(double* U, const int* sub_ptr, const int* voff, const int* nt,
                           int nsub, int b, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_eig_init, dim3(nsub), dim3(256), 0, st, U, sub_ptr, voff, nt, b, seed);
  return hipGetLastError();
}

// ------------------------------------------------- small dense helpers ---
// Gram matrix sG = X^T Y (b x b) of npad-row blocks, MFMA quadrants split
// over row-chunk slices, reduced in fixed order.
__device__ void gram(const double* X, const double* Y, int npad, int b, double (*spart)[256],
                     double (*sG)[EIG_MAXB + 1]) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ncq = b / 16, nq = ncq * ncq;
  int ns = EIG_WAVES / nq;
  if (ns < 1) ns = 1;
  const int qd = w % nq, sl = w / nq;
  const int rq = qd / ncq, cq = qd % ncq;
  d4_t acc = acc_zero<double>();
  if (sl < ns && w < nq * ns) {
    const int nchunk = npad / TS;
    for (int t = sl; t < nchunk; t += ns)
      q_xTy<double>(acc, X + (int64_t)t * TS * b + rq * 16, b, Y + (int64_t)t * TS * b + cq * 16,
                    b, lane);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) spart[w][acc_row<double>(lane, v) * 16 + acc_col(lane)] = (sl < ns && w < nq * ns) ? acc[v] : 0.0;
  block_sync();
  for (int t = tid; t < b * b; t += blockDim.x) {
    int r = t / b, c = t % b;
    int q = (r >> 4) * ncq + (c >> 4);
    double s = 0.0;
    for (int k = 0; k < ns; ++k) s += spart[q + k * nq][(r & 15) * 16 + (c & 15)];
    sG[r][c] = s;
  }
  block_sync();
}

// X[rows] <- X[rows] * M (b x b, in LDS), 16-row slabs per wavefront.
__device__ void right_multiply(double* X, int npad, int b, const double (*M)[EIG_MAXB + 1]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ncq = b / 16;
  const int nslab = npad / 16;
  for (int s = w; s < nslab; s += EIG_WAVES) {
    double* Xs = X + (int64_t)s * 16 * b;
    d4_t acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = acc_zero<double>();
    const int i = lane & 15, k = lane >> 4;
    for (int kk = 0; kk < b / 4; ++kk) {
      double a = Xs[i * b + kk * 4 + k];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < ncq) acc[c] = Mfma<double>::run(a, M[kk * 4 + k][c * 16 + i], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < ncq)
#pragma unroll
        for (int v = 0; v < 4; ++v) Xs[acc_row<double>(lane, v) * b + c * 16 + acc_col(lane)] = acc[c][v];
  }
}

// Cholesky of sG (b x b, unit diagonal expected) by wavefront 0 into its
// lower triangle; returns a bitmask-free flag array bad[c] = 1 for pivots
// below `tiny`.  Then sM = L^{-T} (upper triangular).
__device__ void chol_inv_wave(double (*sG)[EIG_MAXB + 1], double (*sM)[EIG_MAXB + 1], int b,
                              int* bad, double tiny) {
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < b; ++c) {
    double d = sG[c][c];
    bool collapse = !(d > tiny);
    if (lane == 0) bad[c] = collapse ? 1 : 0;
    double s = collapse ? 1.0 : sqrt(d);
    wave_sync();
    if (lane > c && lane < b) sG[lane][c] = collapse ? 0.0 : sG[lane][c] / s;
    if (lane == c) sG[c][c] = s;
    wave_sync();
    for (int e = lane; e < b * b; e += 64) {
      int r = e / b, q = e % b;
      if (q > c && q <= r) sG[r][q] -= sG[r][c] * sG[q][c];
    }
    wave_sync();
  }
  // sM[q][t] = (L^{-1})[t][q]  i.e. L^{-T}; lane t solves L x = e_t
  if (lane < b) {
    const int t = lane;
    for (int r = 0; r < b; ++r) {
      double x = 0.0;
      if (r >= t) {
        double s = (r == t) ? 1.0 : 0.0;
        for (int q = t; q < r; ++q) s -= sG[r][q] * sM[t][q];
        x = s / sG[r][r];
      }
      sM[t][r] = x;  // row t of L^{-T} = column t of L^{-1}
    }
  }
  wave_sync();
}

// --------------------------------------------------------------- orth ---
__global__ __launch_bounds__(1024) void k_orth(double* __restrict__ U, const int* __restrict__ voff,
                                               const int* __restrict__ ntl,
                                               const int* __restrict__ sub_ptr, int b,
                                               uint64_t seed, int salt,
                                               const int* __restrict__ active) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  __shared__ double spart[EIG_WAVES][256];
  __shared__ double sG[EIG_MAXB][EIG_MAXB + 1];
  __shared__ double sM[EIG_MAXB][EIG_MAXB + 1];
  __shared__ int bad[EIG_MAXB];
  __shared__ int nbad;
  __shared__ double scl[EIG_MAXB];
  const int npad = ntl[j] * TS;
  const int n = sub_ptr[j + 1] - sub_ptr[j];
  double* Uj = U + (int64_t)voff[j] * b;
  const int tid = threadIdx.x;
  int pass = 0, refill = 0;
  while (pass < 2) {
    gram(Uj, Uj, npad, b, spart, sG);
    // scale to unit diagonal
    if (tid < b) {
      double d = sG[tid][tid];
      scl[tid] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    block_sync();
    for (int t = tid; t < b * b; t += blockDim.x) {
      int r = t / b, c = t % b;
      sG[r][c] *= scl[r] * scl[c];
    }
    block_sync();
    if (tid < 64) chol_inv_wave(sG, sM, b, bad, 1e-10);
    if (tid == 0) {
      int cnt = 0;
      for (int c = 0; c < b; ++c) cnt += bad[c] || scl[c] == 0.0;
      nbad = cnt;
    }
    block_sync();
    if (nbad > 0 && refill < 4) {
      // replace collapsed columns by fresh pseudo-random vectors and retry
      for (int t = tid; t < npad * b; t += blockDim.x) {
        int a = t / b, c = t % b;
        if (bad[c] || scl[c] == 0.0)
          Uj[t] = hash_uniform(seed + 7919ull * (salt + 1) + refill, (uint64_t)j,
                               (uint64_t)a * 977 + c);
      }
      block_sync();
      ++refill;
      pass = 0;
      continue;
    }
    // U <- U * diag(scl) * L^{-T}
    for (int t = tid; t < b * b; t += blockDim.x) {
      int r = t / b, c = t % b;
      sM[r][c] *= scl[r];
    }
    block_sync();
    right_multiply(Uj, npad, b, sM);
    block_sync();
    ++pass;
  }
}

hipError_t launch_orth(double* U, const int* voff, const int* nt, const int* sub_ptr, int nsub,
                       int b, uint64_t seed, int salt, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_orth, dim3(nsub), dim3(1024), 0, st, U, voff, nt, sub_ptr, b, seed, salt,
                     active);
  return hipGetLastError();
}

// ------------------------------------------------------- Jacobi (wave) ---
// Eigen-decomposition of the symmetric sH (b x b) by cyclic Jacobi with the
// round-robin ordering: on return diag(sH) holds the eigenvalues and sQ the
// eigenvectors (columns).
__device__ void jacobi_wave(double (*sH)[EIG_MAXB + 1], double (*sQ)[EIG_MAXB + 1], int b,
                            double* cs_c, double* cs_s, int* pp, int* pq) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < b * b; e += 64) sQ[e / b][e % b] = (e / b == e % b) ? 1.0 : 0.0;
  wave_sync();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = lane; e < b * b; e += 64) {
      int r = e / b, c = e % b;
      double v = sH[r][c];
      if (r != c) off += v * v;
      else dia += v * v;
    }
    for (int m = 32; m >= 1; m >>= 1) {
      off += __shfl_xor(off, m);
      dia += __shfl_xor(dia, m);
    }
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int round = 0; round < b - 1; ++round) {
      if (lane < b / 2) {
        int i0 = lane, i1 = b - 1 - lane;
        int p = i0 == 0 ? 0 : ((i0 - 1 + round) % (b - 1)) + 1;
        int q = ((i1 - 1 + round) % (b - 1)) + 1;
        if (p > q) { int t = p; p = q; q = t; }
        double apq = sH[p][q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          double app = sH[p][p], aqq = sH[q][q];
          double tau = (aqq - app) / (2.0 * apq);
          double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs_c[lane] = c;
        cs_s[lane] = s;
        pp[lane] = p;
        pq[lane] = q;
      }
      wave_sync();
      // rows p, q of H
      for (int e = lane; e < (b / 2) * b; e += 64) {
        int k = e / b, m = e % b;
        int p = pp[k], q = pq[k];
        double c = cs_c[k], s = cs_s[k];
        double hp = sH[p][m], hq = sH[q][m];
        sH[p][m] = c * hp - s * hq;
        sH[q][m] = s * hp + c * hq;
      }
      wave_sync();
      // columns p, q of H and of Q
      for (int e = lane; e < (b / 2) * b; e += 64) {
        int k = e / b, m = e % b;
        int p = pp[k], q = pq[k];
        double c = cs_c[k], s = cs_s[k];
        double hp = sH[m][p], hq = sH[m][q];
        sH[m][p] = c * hp - s * hq;
        sH[m][q] = s * hp + c * hq;
        double qp = sQ[m][p], qq = sQ[m][q];
        sQ[m][p] = c * qp - s * qq;
        sQ[m][q] = s * qp + c * qq;
      }
      wave_sync();
    }
  }
}

// ------------------------------------------------------- Rayleigh-Ritz ---
__global__ __launch_bounds__(1024) void k_rayleigh_ritz(
    double* __restrict__ U, const double* __restrict__ W, double* __restrict__ Y,
    double* __restrict__ theta, double* __restrict__ resid, int* __restrict__ active,
    const int* __restrict__ voff, const int* __restrict__ ntl, int b, int nev, double tau,
    int nev_max, double sigma, double tol) {
  const int j = blockIdx.x;
  if (!active[j]) return;
  __shared__ double spart[EIG_WAVES][256];
  __shared__ double sH[EIG_MAXB][EIG_MAXB + 1];
  __shared__ double sQ[EIG_MAXB][EIG_MAXB + 1];
  __shared__ double sres[EIG_WAVES][EIG_MAXB];
  __shared__ double th[EIG_MAXB];
  __shared__ double cs_c[EIG_MAXB / 2], cs_s[EIG_MAXB / 2];
  __shared__ int pp[EIG_MAXB / 2], pq[EIG_MAXB / 2], perm[EIG_MAXB];
  const int npad = ntl[j] * TS;
  double* Uj = U + (int64_t)voff[j] * b;
  const double* Wj = W + (int64_t)voff[j] * b;
  double* Yj = Y + (int64_t)voff[j] * b;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // H = U^T W, symmetrised
  gram(Uj, Wj, npad, b, spart, sH);
  for (int t = tid; t < b * b; t += blockDim.x) {
    int r = t / b, c = t % b;
    if (r < c) {
      double v = 0.5 * (sH[r][c] + sH[c][r]);
      sH[r][c] = v;
      sH[c][r] = v;
    }
  }
  block_sync();
  if (w == 0) {
    jacobi_wave(sH, sQ, b, cs_c, cs_s, pp, pq);
    if (lane == 0) {
      // stable selection sort, descending
      for (int c = 0; c < b; ++c) perm[c] = c;
      for (int c = 0; c < b; ++c) {
        int best = c;
        for (int q = c + 1; q < b; ++q)
          if (sH[perm[q]][perm[q]] > sH[perm[best]][perm[best]]) best = q;
        int t = perm[best];
        for (int q = best; q > c; --q) perm[q] = perm[q - 1];
        perm[c] = t;
      }
      for (int c = 0; c < b; ++c) th[c] = sH[perm[c]][perm[c]];
    }
    wave_sync();
  }
  block_sync();
  // Qs = Q[:, perm] into sH
  for (int t = tid; t < b * b; t += blockDim.x) {
    int r = t / b, c = t % b;
    sH[r][c] = sQ[r][perm[c]];
  }
  block_sync();
  // slabs: WQ, UQ, residual partials; Y <- UQ, U <- WQ
  for (int t = tid; t < EIG_WAVES * EIG_MAXB; t += blockDim.x) sres[t / EIG_MAXB][t % EIG_MAXB] = 0.0;
  block_sync();
  {
    const int ncq = b / 16;
    const int nslab = npad / 16;
    const int i = lane & 15, k = lane >> 4;
    for (int s = w; s < nslab; s += EIG_WAVES) {
      double* Us = Uj + (int64_t)s * 16 * b;
      const double* Ws = Wj + (int64_t)s * 16 * b;
      double* Ys = Yj + (int64_t)s * 16 * b;
      d4_t aw[4], au[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) { aw[c] = acc_zero<double>(); au[c] = acc_zero<double>(); }
      for (int kk = 0; kk < b / 4; ++kk) {
        double xw = Ws[i * b + kk * 4 + k];
        double xu = Us[i * b + kk * 4 + k];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (c >= ncq) continue;
          double q = sH[kk * 4 + k][c * 16 + i];
          aw[c] = Mfma<double>::run(xw, q, aw[c]);
          au[c] = Mfma<double>::run(xu, q, au[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c >= ncq) continue;
        const int col = c * 16 + acc_col(lane);
        double r2 = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double rv = aw[c][v] - th[col] * au[c][v];
          r2 += rv * rv;
          Ys[acc_row<double>(lane, v) * b + col] = au[c][v];
          Us[acc_row<double>(lane, v) * b + col] = aw[c][v];
        }
        r2 += __shfl_xor(r2, 16);
        r2 += __shfl_xor(r2, 32);
        if (lane < 16) sres[w][col] += r2;
      }
    }
  }
  block_sync();
  if (tid < b) {
    double s = 0.0;
    for (int q = 0; q < EIG_WAVES; ++q) s += sres[q][tid];
    sres[0][tid] = sqrt(s);
  }
  block_sync();
  if (tid == 0) {
    const double t0 = th[0];
    int nfin = 0;
    for (int c = 0; c < b; ++c) nfin += (t0 > 0.0 && th[c] > 1e-14 * t0);
    int want;
    if (tau > 0.0) {
      int below = 0;
      for (int c = 0; c < nfin; ++c) below += (sigma + 1.0 / th[c] < tau);
      want = below + 1;
      if (want > nev_max) want = nev_max;
    } else {
      want = nev;
    }
    if (want > nfin) want = nfin;
    if (want > b) want = b;
    // backward-error test: ||S y - theta y|| <= tol * ||S|| with ||S|| = theta_0
    bool ok = true;
    for (int c = 0; c < want; ++c) ok = ok && (sres[0][c] <= tol * t0);
    for (int c = 0; c < b; ++c) {
      theta[(int64_t)j * b + c] = th[c];
      resid[(int64_t)j * b + c] = t0 > 0.0 ? sres[0][c] / t0 : 0.0;
    }
    if (ok) active[j] = 0;
  }
}

hipError_t launch_rayleigh_ritz(double* U, const double* W, double* Y, double* theta,
                                double* resid, int* active, const int* voff, const int* nt,
                                const int* sub_ptr, int nsub, int b, int nev, double tau,
                                int nev_max, double sigma, double tol, hipStream_t st) {
  (void)sub_ptr;
  hipLaunchKernelGGL(k_rayleigh_ritz, dim3(nsub), dim3(1024), 0, st, U, W, Y, theta, resid,
                     active, voff, nt, b, nev, tau, nev_max, sigma, tol);
  return hipGetLastError();
}

// ----------------------------------------------------------- selection ---
// m_j and the eigenvalues lam = sigma + 1/theta (ascending), +inf where
// theta <= 1e-14 theta_max.
__global__ void k_select(const double* __restrict__ theta, int nsub, int b, int nev, double tau,
                         int nev_max, double sigma, int* __restrict__ m,
                         double* __restrict__ lam) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsub) return;
  const double* th = theta + (int64_t)j * b;
  double t0 = th[0];
  int nfin = 0, below = 0;
  for (int c = 0; c < b; ++c) {
    bool fin = t0 > 0.0 && th[c] > 1e-14 * t0;
    double l = fin ? sigma + 1.0 / th[c] : INFINITY;
    lam[(int64_t)j * b + c] = l;
    nfin += fin;
    below += fin && (l < tau);
  }
  int mj = tau > 0.0 ? (below < nev_max ? below : nev_max) : (nev < nfin ? nev : nfin);
  if (mj > nfin) mj = nfin;
  m[j] = mj;
}

hipError_t launch_select(const double* theta, int nsub, int b, int nev, double tau, int nev_max,
                         double sigma, int* m, double* lam, hipStream_t st) {
  hipLaunchKernelGGL(k_select, dim3((nsub + 127) / 128), dim3(128), 0, st, theta, nsub, b, nev,
                     tau, nev_max, sigma, m, lam);
  return hipGetLastError();
}

// ------------------------------------------------------------- basis ---
// Z_j[d][c] = X_j p_c / ||X_j p_c||_2 over D_j (row d = position in D_j),
// sign: the entry of largest magnitude (first in order) is positive.
__global__ __launch_bounds__(256) void k_basis(const double* __restrict__ P,
                                               const int* __restrict__ voff, int b,
                                               const int* __restrict__ sub_ptr,
                                               const double* __restrict__ pou,
                                               const int* __restrict__ dmap,
                                               const int* __restrict__ m,
                                               const int* __restrict__ zoff,
                                               double* __restrict__ Z) {
  const int j = blockIdx.x;
  const int mj = m[j];
  if (mj == 0) return;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  const double* Pj = P + (int64_t)voff[j] * b;
  double* Zj = Z + zoff[j];
  __shared__ double red[256];
  __shared__ int redi[256];
  const int tid = threadIdx.x;
  for (int c = 0; c < mj; ++c) {
    double s = 0.0, best = -1.0;
    int bi = 0x7fffffff;
    for (int a = tid; a < n; a += blockDim.x) {
      if (dmap[s0 + a] < 0) continue;
      double v = pou[s0 + a] * Pj[(int64_t)a * b + c];
      s += v * v;
      double av = fabs(v);
      if (av > best) { best = av; bi = a; }
    }
    red[tid] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    double nrm = sqrt(red[0]);
    __syncthreads();
    red[tid] = best;
    redi[tid] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) {
        double b2 = red[tid + o];
        int i2 = redi[tid + o];
        if (b2 > red[tid] || (b2 == red[tid] && i2 < redi[tid])) {
          red[tid] = b2;
          redi[tid] = i2;
        }
      }
      __syncthreads();
    }
    int amax = redi[0];
    double sign = (amax < n && pou[s0 + amax] * Pj[(int64_t)amax * b + c] < 0.0) ? -1.0 : 1.0;
    double scale = nrm > 0.0 ? sign / nrm : 0.0;
    __syncthreads();
    for (int a = tid; a < n; a += blockDim.x) {
      int d = dmap[s0 + a];
      if (d < 0) continue;
      Zj[(int64_t)d * mj + c] = pou[s0 + a] * Pj[(int64_t)a * b + c] * scale;
    }
    __syncthreads();
  }
}

hipError_t launch_basis(const double* P, const int* voff, int b, const int* sub_ptr,
                        const double* pou, const int* dmap, const int* m, const int* zoff,
                        const int* nd, int nsub, double* Z, hipStream_t st) {
  (void)nd;
  hipLaunchKernelGGL(k_basis, dim3(nsub), dim3(256), 0, st, P, voff, b, sub_ptr, pou, dmap, m,
                     zoff, Z);
  return hipGetLastError();
}

}  // namespace geneo
