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
    // chunks t, t + ns, ... in that order, two chunks' loads in flight
    const int nchunk = npad / TS;
    const int i = lane & 15, k = lane >> 4;
    const double* Xq = X + rq * 16 + k * b + i;
    const double* Yq = Y + cq * 16 + k * b + i;
    int t = sl;
    for (; t + ns < nchunk; t += 2 * ns) {
      double xa[8], ya[8], xb[8], yb[8];
      const int64_t oa = (int64_t)t * TS * b, ob = (int64_t)(t + ns) * TS * b;
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        xa[kk] = Xq[oa + kk * 4 * b];
        ya[kk] = Yq[oa + kk * 4 * b];
      }
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        xb[kk] = Xq[ob + kk * 4 * b];
        yb[kk] = Yq[ob + kk * 4 * b];
      }
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) acc = Mfma<double>::run(xa[kk], ya[kk], acc);
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) acc = Mfma<double>::run(xb[kk], yb[kk], acc);
    }
    if (t < nchunk)
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

// Cholesky of sG (b x b, unit diagonal expected, b <= 64) into its lower
// triangle by one wavefront (right-looking); bad[c] = 1 for pivots at or
// below `tiny` (that column of L is zeroed, its diagonal set to 1).  Then
// sM = L^{-T} (upper triangular), the inverse formed right-looking: row c of
// X = L^{-1} is finished at step c and the rows below take its rank-1
// update.  Each step's updates are spread over the 64 lanes, element by
// element; a wavefront needs no barrier between the steps.
__device__ void chol_inv_wave(double (*sG)[EIG_MAXB + 1], double (*sM)[EIG_MAXB + 1], int b,
                              int* bad, double tiny) {
  const int lane = threadIdx.x;
  wave_sync();
  for (int c = 0; c < b; ++c) {
    const double d = sG[c][c];
    const bool collapse = !(d > tiny);
    const double s = collapse ? 1.0 : sqrt(d);
    wave_sync();  // every lane has read the pivot
    if (lane == 0) bad[c] = collapse ? 1 : 0;
    if (lane > c && lane < b) sG[lane][c] = collapse ? 0.0 : sG[lane][c] / s;
    if (lane == c) sG[c][c] = s;
    wave_sync();  // column c is final
    // trailing update of the rows and columns c+1 .. b-1 (lower part)
    const int w = b - 1 - c;
    for (int e = lane; e < w * w; e += 64) {
      const int r = c + 1 + e / w, q = c + 1 + e % w;
      if (q <= r) sG[r][q] -= sG[r][c] * sG[q][c];
    }
    wave_sync();
  }
  // X = L^{-1} kept transposed in sM: sM[q][t] = X[t][q]
  for (int e = lane; e < b * b; e += 64) sM[e / b][e % b] = (e / b == e % b) ? 1.0 : 0.0;
  wave_sync();
  for (int c = 0; c < b; ++c) {
    const double dinv = 1.0 / sG[c][c];
    if (lane <= c) sM[lane][c] *= dinv;
    wave_sync();
    // X[r][q] -= L[r][c] X[c][q] for r > c, q <= c
    const int w = c + 1;
    for (int e = lane; e < (b - 1 - c) * w; e += 64) {
      const int r = c + 1 + e / w, q = e % w;
      sM[q][r] -= sG[r][c] * sM[q][c];
    }
    wave_sync();
  }
}

// ---------------------------------------------------- Jacobi (wavefront) ---
// Eigen-decomposition of the symmetric sH (B x B, B <= 64) by cyclic Jacobi
// with the round-robin ordering, by one wavefront: on return diag(sH) holds
// the eigenvalues and sQ the eigenvectors (columns).  Lanes k < B/2 compute
// the B/2 rotations (c_k, s_k) of a round into an LDS table (the pairs
// (p_k, q_k) are formed by every lane from k and the round); then every
// 2 x 2 block H({p_k, q_k}, {p_l, q_l}) takes rotation k from the left and
// rotation l from the right in one pass (the blocks partition H, so no lane
// touches another's entries), and Q its right rotations.  Rounds whose rotations are all negligible are
// skipped; sweeps stop when the off-diagonal mass is below 1e-30 of the
// diagonal's.
template <int B>
__device__ void jacobi_wave(double (*sH)[B + 1], double (*sQ)[B + 1], double* cs_c,
                            double* cs_s) {
  constexpr int P = B / 2;
  static_assert(B % 16 == 0 && B <= 64, "block width: a multiple of 16, at most 64");
  constexpr int NB = P * P / 64;  // 2 x 2 blocks of H per lane
  constexpr int NQ = B * P / 64;  // entry pairs of Q per lane
  const int lane = threadIdx.x;
  for (int e = lane; e < B * B; e += 64) sQ[e / B][e % B] = (e / B == e % B) ? 1.0 : 0.0;
  wave_sync();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = lane; e < B * B; e += 64) {
      const int r = e / B, c = e % B;
      const double v = sH[r][c];
      if (r != c) off += v * v;
      else dia += v * v;
    }
    for (int m = 32; m >= 1; m >>= 1) {
      off += __shfl_xor(off, m);
      dia += __shfl_xor(dia, m);
    }
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int round = 0; round < B - 1; ++round) {
      // pair k of the round: index 0 stays, the others turn round a circle
      auto pair = [&](int k, int& p, int& q) {
        const int u = k == 0 ? 0 : ((k - 1 + round) % (B - 1)) + 1;
        const int v = ((B - 2 - k + round) % (B - 1)) + 1;
        p = min(u, v);
        q = max(u, v);
      };
      // rotation of pair `lane`: t = tan(theta) is the smaller root of
      // t^2 + 2 tau t - 1 = 0, tau = (a_qq - a_pp) / (2 a_pq), written as
      // 2 a_pq / (d + sign r) with d = a_qq - a_pp, r = sqrt(d^2 + 4 a_pq^2)
      // (one square root and one division on the dependent chain)
      int rot = 0;
      if (lane < P) {
        int p, q;
        pair(lane, p, q);
        const double apq = sH[p][q], app = sH[p][p], aqq = sH[q][q];
        double c = 1.0, sn = 0.0;
        if (apq * apq > 1e-36 * fabs(app * aqq) && apq != 0.0) {
          const double d = aqq - app;
          const double r = sqrt(d * d + 4.0 * apq * apq);
          const double den = (d > 0.0 || (d == 0.0 && apq > 0.0)) ? d + r : d - r;
          const double t = 2.0 * apq / den;
          c = rsqrt(1.0 + t * t);
          sn = t * c;
          rot = 1;
        }
        cs_c[lane] = c;
        cs_s[lane] = sn;
      }
      if (!__any(rot)) continue;
      wave_sync();
      // every entry a lane updates is read before any is written (the
      // compiler cannot tell the reads of one block from the writes of
      // another, so a read-write-read order would serialise them)
      double hv[NB][4], rk[NB][2], rl[NB][2];
      int hp[NB][4];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int e = lane + 64 * u, k = e / P, l = e % P;
        int pk, qk, pl, ql;
        pair(k, pk, qk);
        pair(l, pl, ql);
        hp[u][0] = pk * (B + 1) + pl;
        hp[u][1] = pk * (B + 1) + ql;
        hp[u][2] = qk * (B + 1) + pl;
        hp[u][3] = qk * (B + 1) + ql;
#pragma unroll
        for (int v = 0; v < 4; ++v) hv[u][v] = (&sH[0][0])[hp[u][v]];
        rk[u][0] = cs_c[k];
        rk[u][1] = cs_s[k];
        rl[u][0] = cs_c[l];
        rl[u][1] = cs_s[l];
      }
      double qv[NQ][2], rq[NQ][2];
      int qi[NQ][2];
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const int e = lane + 64 * u, m = e / P, l = e % P;
        int pl, ql;
        pair(l, pl, ql);
        qi[u][0] = m * (B + 1) + pl;
        qi[u][1] = m * (B + 1) + ql;
        qv[u][0] = (&sQ[0][0])[qi[u][0]];
        qv[u][1] = (&sQ[0][0])[qi[u][1]];
        rq[u][0] = cs_c[l];
        rq[u][1] = cs_s[l];
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const double ck = rk[u][0], sk = rk[u][1], cl = rl[u][0], sl = rl[u][1];
        const double a = hv[u][0], bb = hv[u][1], c = hv[u][2], d = hv[u][3];
        // rows p_k, q_k
        const double a1 = ck * a - sk * c, c1 = sk * a + ck * c;
        const double b1 = ck * bb - sk * d, d1 = sk * bb + ck * d;
        // columns p_l, q_l
        (&sH[0][0])[hp[u][0]] = cl * a1 - sl * b1;
        (&sH[0][0])[hp[u][1]] = sl * a1 + cl * b1;
        (&sH[0][0])[hp[u][2]] = cl * c1 - sl * d1;
        (&sH[0][0])[hp[u][3]] = sl * c1 + cl * d1;
      }
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const double cl = rq[u][0], sl = rq[u][1], qp = qv[u][0], qq = qv[u][1];
        (&sQ[0][0])[qi[u][0]] = cl * qp - sl * qq;
        (&sQ[0][0])[qi[u][1]] = sl * qp + cl * qq;
      }
      wave_sync();
    }
  }
}

// ------------------------------------------------------ batched pieces ---
// G_j = X_j^T Y_j (b x b) for every active subdomain, one workgroup each.
__global__ __launch_bounds__(1024) void k_gram(const double* __restrict__ X,
                                               const double* __restrict__ Y,
                                               const int* __restrict__ voff,
                                               const int* __restrict__ ntl, int b,
                                               double* __restrict__ G,
                                               const int* __restrict__ active, int symm) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  __shared__ double spart[EIG_WAVES][256];
  __shared__ double sG[EIG_MAXB][EIG_MAXB + 1];
  const int npad = ntl[j] * TS;
  gram(X + (int64_t)voff[j] * b, Y + (int64_t)voff[j] * b, npad, b, spart, sG);
  double* Gj = G + (int64_t)j * b * b;
  for (int t = threadIdx.x; t < b * b; t += blockDim.x) {
    int r = t / b, c = t % b;
    Gj[t] = symm ? 0.5 * (sG[r][c] + sG[c][r]) : sG[r][c];
  }
}

// One wavefront per subdomain: Jacobi eigen-decomposition of H_j, columns
// sorted by descending eigenvalue (stable: equal values keep their index
// order; NaN after every number), into Q_j and theta_j.  Lane c places
// column c at its rank.
template <int B>
__global__ __launch_bounds__(64) void k_small_eig(const double* __restrict__ H,
                                                  double* __restrict__ Q,
                                                  double* __restrict__ theta,
                                                  const int* __restrict__ active) {
  constexpr int b = B;
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  __shared__ double sH[B][B + 1];
  __shared__ double sQ[B][B + 1];
  __shared__ double cs_c[B / 2], cs_s[B / 2];
  __shared__ int perm[B];
  const int lane = threadIdx.x;
  const double* Hj = H + (int64_t)j * b * b;
  for (int e = lane; e < b * b; e += 64) sH[e / b][e % b] = Hj[e];
  wave_sync();
  jacobi_wave<B>(sH, sQ, cs_c, cs_s);
  if (lane < b) {
    // q goes before c: larger value, or equal value and smaller index;
    // NaN ranks below every number
    const double d = sH[lane][lane];
    const bool dn = d != d;
    int rank = 0;
    for (int q = 0; q < b; ++q) {
      const double v = sH[q][q];
      const bool vn = v != v;
      const bool gt = vn ? false : (dn ? true : v > d);
      const bool eq = vn ? dn : (!dn && v == d);
      rank += (gt || (eq && q < lane)) ? 1 : 0;
    }
    perm[rank] = lane;
  }
  wave_sync();
  double* Qj = Q + (int64_t)j * b * b;
  for (int e = lane; e < b * b; e += 64) {
    const int r = e / b, c = e % b;
    Qj[e] = sQ[r][perm[c]];
  }
  if (lane < b) theta[(int64_t)j * b + lane] = sH[perm[lane]][perm[lane]];
}

// One wavefront per subdomain: Cholesky-QR factor of the Gram matrix G_j of
// the current block.  M_j = diag(s) L^{-T} with s = diag(G)^{-1/2} and
// L L^T = diag(s) G diag(s).  A column whose pivot collapses (numerically
// dependent on the previous ones) gets a zero column in M_j and its flag in
// badcol[j*b + c].
__global__ __launch_bounds__(64) void k_small_cholqr(const double* __restrict__ G, int b,
                                                             double* __restrict__ M,
                                                             int* __restrict__ badcol,
                                                             const int* __restrict__ active) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  __shared__ double sG[EIG_MAXB][EIG_MAXB + 1];
  __shared__ double sM[EIG_MAXB][EIG_MAXB + 1];
  __shared__ double scl[EIG_MAXB];
  __shared__ int sbad[EIG_MAXB];
  const int tid = threadIdx.x;
  const double* Gj = G + (int64_t)j * b * b;
  if (tid < b) {
    double d = Gj[tid * b + tid];
    scl[tid] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
  wave_sync();
  for (int e = tid; e < b * b; e += 64) {
    int r = e / b, c = e % b;
    sG[r][c] = Gj[e] * scl[r] * scl[c];
  }
  chol_inv_wave(sG, sM, b, sbad, 1e-10);
  double* Mj = M + (int64_t)j * b * b;
  for (int e = tid; e < b * b; e += 64) {
    int r = e / b, c = e % b;
    const bool badc = sbad[c] || scl[c] == 0.0;
    Mj[e] = badc ? 0.0 : sM[r][c] * scl[r];
  }
  if (tid < b) badcol[(int64_t)j * b + tid] = (sbad[tid] || scl[tid] == 0.0) ? 1 : 0;
}

// X_j <- X_j M_j for 16-row slabs; grid (slab groups, subdomains).
// With Yout != NULL also Yout_j = Xin_j M_j from a second input (used to
// form U Q and W Q in one pass together with the residual partial sums).
#define SLABS_PER_WG 8
__global__ __launch_bounds__(256) void k_right_mul(double* __restrict__ X,
                                                   const double* __restrict__ M,
                                                   const int* __restrict__ voff,
                                                   const int* __restrict__ ntl, int b,
                                                   const int* __restrict__ active) {
  const int j = blockIdx.y;
  if (active && !active[j]) return;
  const int nslab = ntl[j] * TS / 16;
  const int s0 = blockIdx.x * SLABS_PER_WG;
  if (s0 >= nslab) return;
  __shared__ double sM[EIG_MAXB][EIG_MAXB + 1];
  const double* Mj = M + (int64_t)j * b * b;
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) sM[e / b][e % b] = Mj[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ncq = b / 16;
  double* Xj = X + (int64_t)voff[j] * b;
  for (int s = s0 + w; s < min(nslab, s0 + SLABS_PER_WG); s += 4) {
    double* Xs = Xj + (int64_t)s * 16 * b;
    d4_t acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = acc_zero<double>();
    const int i = lane & 15, k = lane >> 4;
    for (int kk = 0; kk < b / 4; ++kk) {
      double a = Xs[i * b + kk * 4 + k];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < ncq) acc[c] = Mfma<double>::run(a, sM[kk * 4 + k][c * 16 + i], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < ncq)
#pragma unroll
        for (int v = 0; v < 4; ++v) Xs[acc_row<double>(lane, v) * b + c * 16 + acc_col(lane)] = acc[c][v];
  }
}

// Ritz step: Y = U Q, U <- W Q, and per-group partial sums of
// ||W Q e_c - theta_c U Q e_c||^2; grid (slab groups, subdomains).
__global__ __launch_bounds__(256) void k_ritz_update(double* __restrict__ U,
                                                     const double* __restrict__ W,
                                                     double* __restrict__ Y,
                                                     const double* __restrict__ Q,
                                                     const double* __restrict__ theta,
                                                     const int* __restrict__ voff,
                                                     const int* __restrict__ ntl, int b,
                                                     double* __restrict__ part, int ngroups,
                                                     const int* __restrict__ active) {
  const int j = blockIdx.y;
  if (active && !active[j]) return;
  const int nslab = ntl[j] * TS / 16;
  const int s0 = blockIdx.x * SLABS_PER_WG;
  __shared__ double sQ[EIG_MAXB][EIG_MAXB + 1];
  __shared__ double sres[4][EIG_MAXB];
  __shared__ double th[EIG_MAXB];
  const double* Qj = Q + (int64_t)j * b * b;
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) sQ[e / b][e % b] = Qj[e];
  for (int e = threadIdx.x; e < 4 * EIG_MAXB; e += blockDim.x) sres[e / EIG_MAXB][e % EIG_MAXB] = 0.0;
  if (threadIdx.x < b) th[threadIdx.x] = theta[(int64_t)j * b + threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ncq = b / 16;
  double* Uj = U + (int64_t)voff[j] * b;
  const double* Wj = W + (int64_t)voff[j] * b;
  double* Yj = Y + (int64_t)voff[j] * b;
  const int i = lane & 15, k = lane >> 4;
  for (int s = s0 + w; s < min(nslab, s0 + SLABS_PER_WG); s += 4) {
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
        double q = sQ[kk * 4 + k][c * 16 + i];
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
  __syncthreads();
  if (threadIdx.x < b) {
    double t = sres[0][threadIdx.x] + sres[1][threadIdx.x] + sres[2][threadIdx.x] +
               sres[3][threadIdx.x];
    part[((int64_t)j * ngroups + blockIdx.x) * b + threadIdx.x] = t;
  }
}

// Convergence test per subdomain (backward error ||r_c|| <= tol ||S||,
// ||S|| = theta_0) over the wanted pairs; clears active[j] when done.  One
// 64-thread block per subdomain: thread c reduces column c over the groups.
__global__ __launch_bounds__(64) void k_ritz_check(const double* __restrict__ part, int ngroups,
                                                   const double* __restrict__ theta,
                                                   double* __restrict__ resid,
                                                   int* __restrict__ active, int b, int nev,
                                                   double tau, const double* __restrict__ tau_sub,
                                                   int nev_max, double sigma, double tol,
                                                   EigStall stl) {
  const int j = blockIdx.x;
  if (!active[j]) return;
  if (tau_sub) tau = tau_sub[j];
  __shared__ double rr[EIG_MAXB];
  const int c = threadIdx.x;
  const double* th = theta + (int64_t)j * b;
  const double t0 = th[0];
  if (c < b) {
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += part[((int64_t)j * ngroups + g) * b + c];
    rr[c] = sqrt(s);
    resid[(int64_t)j * b + c] = t0 > 0.0 ? rr[c] / t0 : 0.0;
  }
  __syncthreads();
  if (c != 0) return;
  int nfin = 0;
  for (int q = 0; q < b; ++q) nfin += (t0 > 0.0 && th[q] > 1e-14 * t0);
  int want;
  if (tau > 0.0) {
    int below = 0;
    for (int q = 0; q < nfin; ++q) below += (sigma + 1.0 / th[q] < tau);
    want = below + 1;
    if (want > nev_max) want = nev_max;
  } else {
    want = nev;
  }
  if (want > nfin) want = nfin;
  if (want > b) want = b;
  bool ok = true;
  double rmax = 0.0;
  for (int q = 0; q < want; ++q) {
    ok = ok && (rr[q] <= tol * t0);
    rmax = fmax(rmax, t0 > 0.0 ? rr[q] / t0 : 0.0);
  }
  if (ok) {
    active[j] = 0;
    return;
  }
  // stagnation: the largest wanted residual has not halved for stl.sweeps
  // sweeps -- the iteration sits at the rounding floor of the shifted solves
  // or creeps at a ratio close to 1 (a wanted pair inside a dense part of
  // the spectrum); stop there if the residual is already acceptable
  if (stl.sweeps > 0) {
    if (rmax < 0.5 * stl.best[j]) {
      stl.best[j] = rmax;
      stl.count[j] = 0;
    } else if (++stl.count[j] >= stl.sweeps && rmax <= stl.floor) {
      active[j] = 0;
      stl.stalled[j] = 1;
    }
  }
}

// Replace the collapsed (zeroed) columns by fresh pseudo-random vectors.
__global__ void k_refill(double* __restrict__ U, const int* __restrict__ voff,
                         const int* __restrict__ ntl, int b, const int* __restrict__ badcol,
                         uint64_t seed, int salt, const int* __restrict__ active) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  const int* bj = badcol + (int64_t)j * b;
  int any = 0;
  for (int c = 0; c < b; ++c) any |= bj[c];
  if (!any) return;
  const int npad = ntl[j] * TS;
  double* Uj = U + (int64_t)voff[j] * b;
  for (int t = threadIdx.x; t < npad * b; t += blockDim.x) {
    int a = t / b, c = t % b;
    if (bj[c])
      Uj[t] = hash_uniform(seed + 7919ull * (salt + 1), (uint64_t)j, (uint64_t)a * 977 + c);
  }
}

// Orthonormalise the blocks: two passes of Cholesky QR; after the first,
// collapsed columns are replaced by pseudo-random vectors, which the second
// pass orthonormalises against the rest.
hipError_t launch_orth2(double* U, const int* voff, const int* nt, int nsub, int b,
                        uint64_t seed, int salt, const int* active, const EigWork& wk,
                        hipStream_t st) {
  dim3 grid2(wk.ngroups, nsub);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_gram, dim3(nsub), dim3(1024), 0, st, U, U, voff, nt, b, wk.G, active, 1);
    hipLaunchKernelGGL(k_small_cholqr, dim3(nsub), dim3(64), 0, st, wk.G, b, wk.M, wk.badcol,
                       active);
    hipLaunchKernelGGL(k_right_mul, grid2, dim3(256), 0, st, U, wk.M, voff, nt, b, active);
    if (pass == 0)
      hipLaunchKernelGGL(k_refill, dim3(nsub), dim3(256), 0, st, U, voff, nt, b, wk.badcol, seed,
                         salt, active);
  }
  return hipGetLastError();
}

hipError_t launch_rr2(double* U, const double* W, double* Y, double* theta, double* resid,
                      int* active, const int* voff, const int* nt, int nsub, int b, int nev,
                      double tau, const double* tau_sub, int nev_max, double sigma, double tol,
                      const EigWork& wk, const EigStall& stl, hipStream_t st) {
  hipLaunchKernelGGL(k_gram, dim3(nsub), dim3(1024), 0, st, U, W, voff, nt, b, wk.G, active, 1);
  switch (b) {
    case 16: hipLaunchKernelGGL(k_small_eig<16>, dim3(nsub), dim3(64), 0, st, wk.G, wk.M, theta, active); break;
    case 32: hipLaunchKernelGGL(k_small_eig<32>, dim3(nsub), dim3(64), 0, st, wk.G, wk.M, theta, active); break;
    case 48: hipLaunchKernelGGL(k_small_eig<48>, dim3(nsub), dim3(64), 0, st, wk.G, wk.M, theta, active); break;
    default: hipLaunchKernelGGL(k_small_eig<64>, dim3(nsub), dim3(64), 0, st, wk.G, wk.M, theta, active); break;
  }
  hipLaunchKernelGGL(k_ritz_update, dim3(wk.ngroups, nsub), dim3(256), 0, st, U, W, Y, wk.M,
                     theta, voff, nt, b, wk.part, wk.ngroups, active);
  hipLaunchKernelGGL(k_ritz_check, dim3(nsub), dim3(64), 0, st, wk.part, wk.ngroups, theta,
                     resid, active, b, nev, tau, tau_sub, nev_max, sigma, tol, stl);
  return hipGetLastError();
}

// --------------------------------------------------- Chebyshev filter ---
// One step of the Chebyshev recurrence on [0, a_j], a_j = the smallest Ritz
// value of subdomain j's block (theta sorted descending), floored at
// 1e-14 theta_0:
//   first  (Zp = Z_0):            Zn = (2/a) SZ - Zp
//   later  (Zc = Z_k, Zp = Z_k-1): Zn = (4/a) SZ - 2 Zc - Zp
// elementwise over the padded block; Zn may alias Zp or SZ.
__global__ __launch_bounds__(256) void k_cheb(double* Zn, const double* Zc, const double* SZ,
                                              const double* Zp, const double* __restrict__ theta,
                                              const int* __restrict__ voff,
                                              const int* __restrict__ ntl, int b, int first,
                                              const int* __restrict__ active) {
  const int j = blockIdx.y;
  if (active && !active[j]) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nel = (int64_t)ntl[j] * TS * b;
  if (t >= nel) return;
  const double t0 = theta[(int64_t)j * b];
  const double a = fmax(theta[(int64_t)j * b + b - 1], 1e-14 * t0);
  const int64_t e = (int64_t)voff[j] * b + t;
  if (first) Zn[e] = (2.0 / a) * SZ[e] - Zp[e];
  else Zn[e] = (4.0 / a) * SZ[e] - 2.0 * Zc[e] - Zp[e];
}

hipError_t launch_cheb(double* Zn, const double* Zc, const double* SZ, const double* Zp,
                       const double* theta, const int* voff, const int* nt, int nsub, int b,
                       int maxnt, bool first, const int* active, hipStream_t st) {
  const int64_t nel = (int64_t)maxnt * TS * b;
  hipLaunchKernelGGL(k_cheb, dim3((unsigned)((nel + 255) / 256), nsub), dim3(256), 0, st, Zn, Zc,
                     SZ, Zp, theta, voff, nt, b, first ? 1 : 0, active);
  return hipGetLastError();
}

// ----------------------------------------------------------- selection ---
// m_j and the eigenvalues lam = sigma + 1/theta (ascending), +inf where
// theta <= 1e-14 theta_max.
__global__ void k_select(const double* __restrict__ theta, int nsub, int b, int nev, double tau,
                         const double* __restrict__ tau_sub, int nev_max, double sigma,
                         int* __restrict__ m, double* __restrict__ lam) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsub) return;
  if (tau_sub) tau = tau_sub[j];
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

hipError_t launch_select(const double* theta, int nsub, int b, int nev, double tau,
                         const double* tau_sub, int nev_max, double sigma, int* m, double* lam,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_select, dim3((nsub + 127) / 128), dim3(128), 0, st, theta, nsub, b, nev,
                     tau, tau_sub, nev_max, sigma, m, lam);
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
