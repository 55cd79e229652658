// Dense Cholesky factorisations on the matrix cores (16x16x4 MFMA).
//
//  * k_potrf_*: batched blocked left-looking factorisation, one workgroup of
//    8 wavefronts per local matrix, panels of two 32-wide tile columns.
//    Bulk update of a panel with every finished column to its left: a work
//    item is the 16-row half of one tile row and produces its slab of both
//    panel tiles, so each tile L(i, jj) read from memory feeds four
//    matrix-core products per k-step.  The panel rows L(k0.., jj) that all
//    items share are read through the caches (FP32) or staged in LDS in
//    double-buffered chunks (FP64, where they are twice as large).  When
//    there are fewer items than wavefronts the jj range is split and the
//    partial sums meet in LDS in a fixed order.  Panel: for each column c
//    the diagonal tile is factored and inverted by one wavefront in
//    registers, then L(i, c) = A(i, c) Dinv(c)^T, then the other panel
//    column takes the rank-32 update from column c.  A failed pivot test
//    stops that matrix and records 1 + the failing row in `status`.
//  * k_trtri: X = L^{-1}, one workgroup per (matrix, tile column c): the
//    column c of X solves L X_c = E_c by blocked forward substitution.
//  * coarse_cholesky: right-looking tiled factorisation of the single coarse
//    matrix, one launch per phase (diagonal, panel, trailing update) so that
//    the trailing update spreads over the whole chip.
//
// The contraction index of every 32-wide product is permuted so that a lane
// reads 8 consecutive elements of one row (vector loads): lane
// (r = l % 16, g = l / 16) supplies k = 8 g + s at step s of 8.
#include "internal.h"

namespace geneo {

template <typename T> struct V8 { T v[8]; };

__device__ __forceinline__ void ld8(V8<float>& f, const float* p) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  f.v[0] = a.x; f.v[1] = a.y; f.v[2] = a.z; f.v[3] = a.w;
  f.v[4] = b.x; f.v[5] = b.y; f.v[6] = b.z; f.v[7] = b.w;
}
__device__ __forceinline__ void ld8(V8<double>& f, const double* p) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double2 a = *reinterpret_cast<const double2*>(p + 2 * u);
    f.v[2 * u] = a.x;
    f.v[2 * u + 1] = a.y;
  }
}

__device__ __forceinline__ float rdlane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double rdlane(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// LDS row stride of staged and diagonal tiles: a multiple of 16 bytes so
// that fragment reads are 128-bit, padded against bank conflicts.
template <typename T> struct DiagLd;
template <> struct DiagLd<float> { static constexpr int v = TS + 4; };
template <> struct DiagLd<double> { static constexpr int v = TS + 2; };

// Factor the TS x TS tile D = L L^T (lower triangle of D read) and invert L,
// by one wavefront, all in registers.  Lane r (mod TS) keeps row r of the
// tile; the factorisation is right-looking, with the pivot and column c
// broadcast by lane reads.  For the inverse, lane t forms column t of
// X = L^{-1} by forward substitution, reading the rows of L from the lanes
// that hold them.  Writes L (zeros above the diagonal) to Lout, X to Xout
// and, if sX is not null, to sX.  Returns 1 + the first in-tile row whose
// pivot fails d > pivtol, else 0.  Kept out of line: inlined, its unrolled
// register arrays would raise the register count of the calling kernel.
template <typename T, int LDI>
__device__ __noinline__ int diag_tile(const T* D, T* Lout, T* Xout, T (*sX)[LDI], T* sRp,
                                      int lane, double pivtol) {
  const int r = lane & (TS - 1);
  const bool writer = lane < TS;
  T a[TS];
#pragma unroll
  for (int q = 0; q < TS; q += 8) {
    V8<T> f;
    ld8(f, D + r * TS + q);
#pragma unroll
    for (int u = 0; u < 8; ++u) a[q + u] = f.v[u];
  }
  int fail = 0;
#pragma unroll
  for (int c = 0; c < TS; ++c) {
    const T d = rdlane(a[c], c);
    if (fail == 0 && !(d > (T)pivtol)) fail = c + 1;
    const T s = sqrt(d > (T)0 ? d : (T)1);
    const T inv = (T)1 / s;
    if (lane == 0) sRp[c] = inv;
    a[c] = r > c ? a[c] * inv : (r == c ? s : (T)0);
#pragma unroll
    for (int q = c + 1; q < TS; ++q) a[q] -= a[c] * rdlane(a[c], q);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (writer) {
#pragma unroll
    for (int q = 0; q < TS; ++q) Lout[r * TS + q] = q <= r ? a[q] : (T)0;
  }
  wave_sync();
  const int t = r;
  T x[TS];
#pragma unroll
  for (int rr = 0; rr < TS; ++rr) {
    T s0 = rr == t ? (T)1 : (T)0, s1 = (T)0;
#pragma unroll
    for (int q = 0; q + 1 < rr; q += 2) {
      s0 -= rdlane(a[q], rr) * x[q];
      s1 -= rdlane(a[q + 1], rr) * x[q + 1];
    }
    if (rr & 1) s0 -= rdlane(a[rr - 1], rr) * x[rr - 1];
    x[rr] = (s0 + s1) * sRp[rr];
    __builtin_amdgcn_sched_barrier(0);
  }
  if (writer) {
#pragma unroll
    for (int rr = 0; rr < TS; ++rr) {
      if (sX) sX[rr][t] = x[rr];
      Xout[rr * TS + t] = x[rr];
    }
  }
  wave_sync();
  return fail;
}

template <typename T, int NW, int KB>
struct PotrfCfg {
  static constexpr int LDI = DiagLd<T>::v;
  static constexpr int CH = sizeof(T) == 8 ? 2 : 4;  // jj per staged chunk
  // staged panel rows: [2 buffers][KB][CH][TS][LDI]
  static constexpr int YBUF = KB * CH * TS * LDI;
  static constexpr int STAGE_BYTES = 2 * YBUF * (int)sizeof(T);
  // slice partial sums: one wavefront's accumulators per slot, NW-1 slots
  static constexpr int PART = 2 * KB * 4 * 64;
  static constexpr int PART_BYTES = (NW - 1) * PART * (int)sizeof(T);
  static constexpr int SHARED_BYTES = STAGE_BYTES > PART_BYTES ? STAGE_BYTES : PART_BYTES;
  // 16-byte vectors per thread when staging one chunk
  static constexpr int VEC = 16 / (int)sizeof(T);
  static constexpr int NVEC = KB * CH * TSQ / VEC;
  static constexpr int VPT = (NVEC + NW * 64 - 1) / (NW * 64);
  static_assert(SHARED_BYTES <= 96 * 1024, "panel staging exceeds the LDS budget");
};

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 t; };
template <> struct Vec16<double> { typedef double2 t; };

// Bulk update, one item per wavefront per round, panel rows staged in LDS
// chunk by chunk (double-buffered; one barrier per chunk).  All wavefronts
// take part in staging and barriers, also those without an item.
template <typename T, int NW, int KB>
__device__ __forceinline__ void bulk_staged(T* A, int nt, int k0, int kn, int w, int tid,
                                            int lane, T* sY) {
  typedef PotrfCfg<T, NW, KB> Cfg;
  typedef typename Mfma<T>::acc Acc;
  typedef typename Vec16<T>::t VT;
  constexpr int CH = Cfg::CH, LDI = Cfg::LDI, VEC = Cfg::VEC;
  const int fi = lane & 15, fg = lane >> 4;
  const int frag = fi * TS + 8 * fg;
  const int nit = 2 * (nt - k0);
  const int nround = (nit + NW - 1) / NW;
  const int nch = (k0 + CH - 1) / CH;
  for (int rd = 0; rd < nround; ++rd) {
    const int it = rd * NW + w;
    const bool act = it < nit;
    const int i = k0 + (act ? it >> 1 : 0), rq = act ? it & 1 : 0;
    Acc acc[KB][2];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c][0] = acc[c][1] = acc_zero<T>();
    VT stg[Cfg::VPT];
    // stage chunk ch into registers: vector e -> (c, jl, row, col4)
    auto fetch = [&](int ch) {
#pragma unroll
      for (int u = 0; u < Cfg::VPT; ++u) {
        const int e = tid + u * NW * 64;
        const int c = e / (CH * TSQ / VEC), rem = e % (CH * TSQ / VEC);
        const int jl = rem / (TSQ / VEC), off = (rem % (TSQ / VEC)) * VEC;
        const int jj = ch * CH + jl;
        if (e < Cfg::NVEC && jj < k0)
          stg[u] = *reinterpret_cast<const VT*>(A + tile_idx(k0 + min(c, kn - 1), jj) * TSQ + off);
      }
    };
    auto store = [&](int ch) {
      T* buf = sY + (ch & 1) * Cfg::YBUF;
#pragma unroll
      for (int u = 0; u < Cfg::VPT; ++u) {
        const int e = tid + u * NW * 64;
        const int c = e / (CH * TSQ / VEC), rem = e % (CH * TSQ / VEC);
        const int jl = rem / (TSQ / VEC), off = (rem % (TSQ / VEC)) * VEC;
        if (e < Cfg::NVEC && ch * CH + jl < k0)
          *reinterpret_cast<VT*>(buf + ((c * CH + jl) * TS + off / TS) * LDI + off % TS) = stg[u];
      }
    };
    fetch(0);
    store(0);
    block_sync();
    const T* X = A + tile_idx(i, 0) * TSQ + rq * 16 * TS + frag;
    V8<T> x0;
    if (act) ld8(x0, X);
    for (int ch = 0; ch < nch; ++ch) {
      if (ch + 1 < nch) fetch(ch + 1);
      if (act) {
        const T* buf = sY + (ch & 1) * Cfg::YBUF;
        const int jend = min(CH, k0 - ch * CH);
        for (int jl = 0; jl < jend; ++jl) {
          const int jj = ch * CH + jl;
          V8<T> x1;
          ld8(x1, X + (int64_t)min(jj + 1, k0 - 1) * TSQ);
#pragma unroll
          for (int c = 0; c < KB; ++c)
#pragma unroll
            for (int cq = 0; cq < 2; ++cq) {
              const T* yp = buf + ((c * CH + jl) * TS + cq * 16 + fi) * LDI + 8 * fg;
              V8<T> y;
#pragma unroll
              for (int u = 0; u < 8; u += VEC) {
                const VT v = *reinterpret_cast<const VT*>(yp + u);
                if constexpr (VEC == 4) {
                  y.v[u] = v.x; y.v[u + 1] = v.y; y.v[u + 2] = v.z; y.v[u + 3] = v.w;
                } else {
                  y.v[u] = v.x; y.v[u + 1] = v.y;
                }
              }
#pragma unroll
              for (int s = 0; s < 8; ++s) acc[c][cq] = Mfma<T>::run(x0.v[s], y.v[s], acc[c][cq]);
            }
          x0 = x1;
        }
      }
      if (ch + 1 < nch) store(ch + 1);
      block_sync();
    }
    if (act) {
#pragma unroll
      for (int c = 0; c < KB; ++c) {
        if (c >= kn || k0 + c > i) continue;
        T* C = A + tile_idx(i, k0 + c) * TSQ + rq * 16 * TS;
#pragma unroll
        for (int cq = 0; cq < 2; ++cq)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            C[acc_row<T>(lane, v) * TS + cq * 16 + acc_col(lane)] -= acc[c][cq][v];
      }
    }
  }
}

// Bulk update when there are fewer items than wavefronts: the jj range of
// each item is split over ns wavefronts (jj = sl, sl + ns, ...) that read
// their operands from memory; partial sums meet in LDS in slice order.
template <typename T, int NW, int KB>
__device__ __forceinline__ void bulk_split(T* A, int nt, int k0, int kn, int w, int lane,
                                           T* sPart) {
  typedef PotrfCfg<T, NW, KB> Cfg;
  typedef typename Mfma<T>::acc Acc;
  const int fi = lane & 15, fg = lane >> 4;
  const int frag = fi * TS + 8 * fg;
  const int nit = 2 * (nt - k0);
  const int ns = min(NW / nit, k0);
  const int it = w % nit, sl = w / nit;
  const bool act = sl < ns;
  const int i = k0 + (it >> 1), rq = it & 1;
  Acc acc[KB][2];
#pragma unroll
  for (int c = 0; c < KB; ++c) acc[c][0] = acc[c][1] = acc_zero<T>();
  if (act) {
    const T* X = A + tile_idx(i, 0) * TSQ + rq * 16 * TS + frag;
    const T* Y[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) Y[c] = A + tile_idx(k0 + min(c, kn - 1), 0) * TSQ + frag;
    V8<T> x0;
    ld8(x0, X + (int64_t)sl * TSQ);
    for (int jj = sl; jj < k0; jj += ns) {
      V8<T> x1;
      ld8(x1, X + (int64_t)min(jj + ns, k0 - 1) * TSQ);
#pragma unroll
      for (int c = 0; c < KB; ++c)
#pragma unroll
        for (int cq = 0; cq < 2; ++cq) {
          V8<T> y;
          ld8(y, Y[c] + (int64_t)jj * TSQ + cq * 16 * TS);
#pragma unroll
          for (int s = 0; s < 8; ++s) acc[c][cq] = Mfma<T>::run(x0.v[s], y.v[s], acc[c][cq]);
        }
      x0 = x1;
    }
  }
  if (act && sl > 0) {
    T* P = sPart + ((sl - 1) * nit + it) * Cfg::PART;
#pragma unroll
    for (int c = 0; c < KB; ++c)
#pragma unroll
      for (int cq = 0; cq < 2; ++cq)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[((c * 2 + cq) * 4 + v) * 64 + lane] = acc[c][cq][v];
  }
  block_sync();
  if (act && sl == 0) {
    for (int s2 = 1; s2 < ns; ++s2) {
      const T* P = sPart + ((s2 - 1) * nit + it) * Cfg::PART;
#pragma unroll
      for (int c = 0; c < KB; ++c)
#pragma unroll
        for (int cq = 0; cq < 2; ++cq)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[c][cq][v] += P[((c * 2 + cq) * 4 + v) * 64 + lane];
    }
#pragma unroll
    for (int c = 0; c < KB; ++c) {
      if (c >= kn || k0 + c > i) continue;
      T* C = A + tile_idx(i, k0 + c) * TSQ + rq * 16 * TS;
#pragma unroll
      for (int cq = 0; cq < 2; ++cq)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          C[acc_row<T>(lane, v) * TS + cq * 16 + acc_col(lane)] -= acc[c][cq][v];
    }
  }
}

// Bulk update with the panel rows read through the caches; one item per
// wavefront per round, the next jj's operands prefetched into registers.
template <typename T, int NW, int KB>
__device__ __forceinline__ void bulk_direct(T* A, int nt, int k0, int kn, int w, int lane) {
  typedef typename Mfma<T>::acc Acc;
  const int fi = lane & 15, fg = lane >> 4;
  const int frag = fi * TS + 8 * fg;
  const int nit = 2 * (nt - k0);
  for (int it = w; it < nit; it += NW) {
    const int i = k0 + (it >> 1), rq = it & 1;
    Acc acc[KB][2];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c][0] = acc[c][1] = acc_zero<T>();
    const T* X = A + tile_idx(i, 0) * TSQ + rq * 16 * TS + frag;
    const T* Y[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) Y[c] = A + tile_idx(k0 + min(c, kn - 1), 0) * TSQ + frag;
    V8<T> x0, y0[KB][2];
    ld8(x0, X);
#pragma unroll
    for (int c = 0; c < KB; ++c)
#pragma unroll
      for (int cq = 0; cq < 2; ++cq) ld8(y0[c][cq], Y[c] + cq * 16 * TS);
    for (int jj = 0; jj < k0; ++jj) {
      const int jn = min(jj + 1, k0 - 1);
      V8<T> x1, y1[KB][2];
      ld8(x1, X + (int64_t)jn * TSQ);
#pragma unroll
      for (int c = 0; c < KB; ++c)
#pragma unroll
        for (int cq = 0; cq < 2; ++cq) ld8(y1[c][cq], Y[c] + (int64_t)jn * TSQ + cq * 16 * TS);
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int c = 0; c < KB; ++c)
#pragma unroll
          for (int cq = 0; cq < 2; ++cq) acc[c][cq] = Mfma<T>::run(x0.v[s], y0[c][cq].v[s], acc[c][cq]);
      x0 = x1;
#pragma unroll
      for (int c = 0; c < KB; ++c) y0[c][0] = y1[c][0], y0[c][1] = y1[c][1];
    }
#pragma unroll
    for (int c = 0; c < KB; ++c) {
      if (c >= kn || k0 + c > i) continue;
      T* C = A + tile_idx(i, k0 + c) * TSQ + rq * 16 * TS;
#pragma unroll
      for (int cq = 0; cq < 2; ++cq)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          C[acc_row<T>(lane, v) * TS + cq * 16 + acc_col(lane)] -= acc[c][cq][v];
    }
  }
}

template <typename T, int NW, int KB, bool STAGED>
__device__ __forceinline__ void potrf_body(T* __restrict__ tiles, const int64_t* __restrict__ toff,
                                           const int* __restrict__ ntl, T* __restrict__ dinv,
                                           const int64_t* __restrict__ doff,
                                           int* __restrict__ status, const int* __restrict__ jobs,
                                           double pivtol) {
  typedef PotrfCfg<T, NW, KB> Cfg;
  typedef typename Mfma<T>::acc Acc;
  constexpr int LDI = Cfg::LDI;
  const int j = jobs[blockIdx.x];
  const int nt = ntl[j];
  T* A = tiles + toff[j] * TSQ;
  T* Di = dinv + doff[j] * TSQ;
  __shared__ __align__(16) T sX[TS][LDI];
  __shared__ T sRp[TS];
  __shared__ __align__(16) unsigned char sShared[Cfg::SHARED_BYTES];
  __shared__ int sfail;
  T* sBuf = reinterpret_cast<T*>(sShared);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int fi = lane & 15, fg = lane >> 4;
  const int frag = fi * TS + 8 * fg;  // this lane's fragment offset in a 16-row slab

  for (int k0 = 0; k0 < nt; k0 += KB) {
    const int kn = min(KB, nt - k0);
    // ---- bulk update of the panel with columns 0 .. k0-1
    if (k0 > 0) {
      if (2 * (nt - k0) < NW) bulk_split<T, NW, KB>(A, nt, k0, kn, w, lane, sBuf);
      else if (STAGED) bulk_staged<T, NW, KB>(A, nt, k0, kn, w, tid, lane, sBuf);
      else bulk_direct<T, NW, KB>(A, nt, k0, kn, w, lane);
    }
    // ---- panel factorization
    for (int c = k0; c < k0 + kn; ++c) {
      if (c > k0) {
        // rank-32 update of column c with column c-1 (inside the panel)
        const int nit = 2 * (nt - c);
        for (int it = w; it < nit; it += NW) {
          const int i = c + (it >> 1), rq = it & 1;
          V8<T> x, y[2];
          ld8(x, A + tile_idx(i, c - 1) * TSQ + rq * 16 * TS + frag);
#pragma unroll
          for (int cq = 0; cq < 2; ++cq) ld8(y[cq], A + tile_idx(c, c - 1) * TSQ + cq * 16 * TS + frag);
          Acc acc[2] = {acc_zero<T>(), acc_zero<T>()};
#pragma unroll
          for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int cq = 0; cq < 2; ++cq) acc[cq] = Mfma<T>::run(x.v[s], y[cq].v[s], acc[cq]);
          T* C = A + tile_idx(i, c) * TSQ + rq * 16 * TS;
#pragma unroll
          for (int cq = 0; cq < 2; ++cq)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              C[acc_row<T>(lane, v) * TS + cq * 16 + acc_col(lane)] -= acc[cq][v];
        }
      }
      block_sync();
      if (w == 0) {
        T* D = A + tile_idx(c, c) * TSQ;
        const int f = diag_tile<T, LDI>(D, D, Di + (int64_t)c * TSQ, sX, sRp, lane, pivtol);
        if (lane == 0) {
          sfail = f;
          if (f) status[j] = c * TS + f;
        }
      }
      block_sync();
      if (sfail) return;
      // L(i, c) = A(i, c) Dinv(c)^T for i > c
      const int nit = 2 * (nt - c - 1);
      for (int it = w; it < nit; it += NW) {
        const int i = c + 1 + (it >> 1), rq = it & 1;
        T* X = A + tile_idx(i, c) * TSQ + rq * 16 * TS;
        V8<T> x, y[2];
        ld8(x, X + frag);
#pragma unroll
        for (int cq = 0; cq < 2; ++cq) {
          const T* yp = &sX[cq * 16 + fi][8 * fg];
#pragma unroll
          for (int u = 0; u < 8; ++u) y[cq].v[u] = yp[u];
        }
        Acc acc[2] = {acc_zero<T>(), acc_zero<T>()};
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int cq = 0; cq < 2; ++cq) acc[cq] = Mfma<T>::run(x.v[s], y[cq].v[s], acc[cq]);
#pragma unroll
        for (int cq = 0; cq < 2; ++cq)
#pragma unroll
          for (int v = 0; v < 4; ++v) X[acc_row<T>(lane, v) * TS + cq * 16 + acc_col(lane)] = acc[cq][v];
      }
      block_sync();
    }
  }
  if (tid == 0) status[j] = 0;
}

// One entry point per role, so that traces and profiles tell them apart:
// local Dirichlet factors (FP32, or FP64 for the subdomains that fail the
// FP32 pivot test) and the shifted Neumann factors of the eigensolver.
__global__ __launch_bounds__(512) void k_potrf_local_f32(float* tiles, const int64_t* toff,
                                                         const int* nt, float* dinv,
                                                         const int64_t* doff, int* status,
                                                         const int* jobs, double pivtol) {
  potrf_body<float, 8, 2, false>(tiles, toff, nt, dinv, doff, status, jobs, pivtol);
}
__global__ __launch_bounds__(512) void k_potrf_local_f64(double* tiles, const int64_t* toff,
                                                         const int* nt, double* dinv,
                                                         const int64_t* doff, int* status,
                                                         const int* jobs, double pivtol) {
  potrf_body<double, 8, 2, true>(tiles, toff, nt, dinv, doff, status, jobs, pivtol);
}
__global__ __launch_bounds__(512) void k_potrf_shifted_f64(double* tiles, const int64_t* toff,
                                                           const int* nt, double* dinv,
                                                           const int64_t* doff, int* status,
                                                           const int* jobs, double pivtol) {
  potrf_body<double, 8, 2, true>(tiles, toff, nt, dinv, doff, status, jobs, pivtol);
}

hipError_t launch_chol_batched(CholRole role, void* tiles, const int64_t* toff, const int* nt,
                               void* dinv, const int64_t* doff, int* status, const int* jobs,
                               int njobs, double pivtol, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  const dim3 grid(njobs), blk(512);
  switch (role) {
    case CholRole::LocalF32:
      hipLaunchKernelGGL(k_potrf_local_f32, grid, blk, 0, st, (float*)tiles, toff, nt,
                         (float*)dinv, doff, status, jobs, pivtol);
      break;
    case CholRole::LocalF64:
      hipLaunchKernelGGL(k_potrf_local_f64, grid, blk, 0, st, (double*)tiles, toff, nt,
                         (double*)dinv, doff, status, jobs, pivtol);
      break;
    case CholRole::ShiftedF64:
      hipLaunchKernelGGL(k_potrf_shifted_f64, grid, blk, 0, st, (double*)tiles, toff, nt,
                         (double*)dinv, doff, status, jobs, pivtol);
      break;
  }
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
  __shared__ double sRp[TS];
  if (*status) return;
  double* D = A + tile_idx(k, k) * TSQ;
  const int f = diag_tile<double, TS + 2>(D, D, Di + (int64_t)k * TSQ, nullptr, sRp, threadIdx.x, 0.0);
  if (f && threadIdx.x == 0) *status = k * TS + f;
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
