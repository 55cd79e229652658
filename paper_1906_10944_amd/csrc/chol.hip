// Dense Cholesky factorisations on the matrix cores (16x16x4 MFMA).
//
//  * k_potrf_*: batched blocked left-looking factorisation, one workgroup of
//    8 (local FP64), 12 (shifted FP64) or 16 (FP32) wavefronts per matrix,
//    panels of four 32-wide tile columns.
//    Bulk update of a panel with every finished column to its left: a work
//    item is the 16-row half of one tile row and produces its slab of all
//    panel tiles, so each tile L(i, jj) read from memory feeds eight
//    matrix-core chains per k-step.  The panel rows L(k0.., jj) that all
//    items share are staged in LDS in double-buffered chunks.  When there
//    are fewer items than wavefronts (FP64: than 8) the jj range is split
//    and the partial sums meet in LDS in a fixed order.  Panel: for each column c the
//    diagonal tile is factored and inverted by one wavefront in registers,
//    then L(i, c) = A(i, c) Dinv(c)^T, then the later panel columns take
//    the rank-32 update from column c.  A failed pivot test stops that
//    matrix and records 1 + the failing row in `status`.
//  * k_trtri_win: X = L^{-1}, one workgroup per (matrix, block of tile
//    columns): windowed forward substitution L X(:, C) = E_C on MFMA.
//  * k_step_potrf / k_step_trsm / k_step_update: right-looking tiled
//    factorisation of a few matrices (the coarse matrix, the FP64 refactors
//    of mixed mode) by tile-column steps, one launch per phase (diagonal,
//    panel, trailing update) over all of them, so that the trailing update
//    spreads over the whole chip.
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
// pivot fails d > pivtol, else 0.
template <typename T, int LDI>
__device__ __forceinline__ int diag_tile_body(const T* D, T* Lout, T* Xout, T (*sX)[LDI], T* sRp,
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

// Out of line for the multi-wavefront kernels (inlined, its unrolled
// register arrays would raise their register count); a kernel that runs it
// alone inlines the body.
template <typename T, int LDI>
__device__ __noinline__ int diag_tile(const T* D, T* Lout, T* Xout, T (*sX)[LDI], T* sRp,
                                      int lane, double pivtol) {
  return diag_tile_body<T, LDI>(D, Lout, Xout, sX, sRp, lane, pivtol);
}

template <typename T, int NW, int KB>
struct PotrfCfg {
  static constexpr int LDI = DiagLd<T>::v;
  // jj per staged chunk: 4 (FP64) or 8 (FP32) panel tiles per buffer
  static constexpr int CH = (sizeof(T) == 8 ? 4 : 8) / KB > 0 ? (sizeof(T) == 8 ? 4 : 8) / KB : 1;
  // staged panel rows: [2 buffers][KB][CH][TS][LDI]
  static constexpr int YBUF = KB * CH * TS * LDI;
  static constexpr int STAGE_BYTES = 2 * YBUF * (int)sizeof(T);
  // split updates use at most NWS wavefronts (FP64: 8, to keep the partial
  // sums within LDS); one wavefront's accumulators per slot, NWS-1 slots
  static constexpr int NWS = (sizeof(T) == 8 && NW > 8) ? 8 : NW;
  static constexpr int PART = 2 * KB * 4 * 64;
  static constexpr int PART_BYTES = (NWS - 1) * PART * (int)sizeof(T);
  static constexpr int SHARED_BYTES = STAGE_BYTES > PART_BYTES ? STAGE_BYTES : PART_BYTES;
  // 16-byte vectors per thread when staging one chunk
  static constexpr int VEC = 16 / (int)sizeof(T);
  static constexpr int NVEC = KB * CH * TSQ / VEC;
  static constexpr int VPT = (NVEC + NW * 64 - 1) / (NW * 64);
  static_assert(SHARED_BYTES <= 128 * 1024, "panel staging exceeds the LDS budget");
};

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 t; };
template <> struct Vec16<double> { typedef double2 t; };

// Bulk update, one item per wavefront per round, panel rows staged in LDS
// chunk by chunk (double-buffered; one barrier per chunk).  All wavefronts
// take part in staging and barriers, also those without an item.
// Envelope (Ej: first nonzero tile column per tile row, NULL = dense;
// rlast: the last tile row with a nonzero tile in the panel): only rows
// k0 .. rlast are updated, row i from tile column Ej[i] on, and the panel
// rows are staged from column Ej[k0] on (the smallest start of any item).
template <typename T, int NW, int KB>
__device__ __forceinline__ void bulk_staged(T* A, int nt, int k0, int kn, int w, int tid,
                                            int lane, T* sY, const int* Ej, int rlast) {
  typedef PotrfCfg<T, NW, KB> Cfg;
  typedef typename Mfma<T>::acc Acc;
  typedef typename Vec16<T>::t VT;
  constexpr int CH = Cfg::CH, LDI = Cfg::LDI, VEC = Cfg::VEC;
  const int fi = lane & 15, fg = lane >> 4;
  const int frag = fi * TS + 8 * fg;
  const int nit = 2 * (rlast - k0 + 1);
  const int nround = (nit + NW - 1) / NW;
  const int jbeg = Ej ? min(Ej[k0], k0) : 0;
  const int nch = (k0 - jbeg + CH - 1) / CH;
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
        const int jj = jbeg + ch * CH + jl;
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
        if (e < Cfg::NVEC && jbeg + ch * CH + jl < k0)
          *reinterpret_cast<VT*>(buf + ((c * CH + jl) * TS + off / TS) * LDI + off % TS) = stg[u];
      }
    };
    fetch(0);
    store(0);
    block_sync();
    const T* X = A + tile_idx(i, 0) * TSQ + rq * 16 * TS + frag;
    // the item's first nonzero tile (tiles left of it are zero: their
    // products would add nothing)
    const int js = Ej ? max(jbeg, min(Ej[i], k0)) : 0;
    V8<T> x0;
    if (act && js < k0) ld8(x0, X + (int64_t)js * TSQ);
    for (int ch = 0; ch < nch; ++ch) {
      if (ch + 1 < nch) fetch(ch + 1);
      if (act) {
        const T* buf = sY + (ch & 1) * Cfg::YBUF;
        const int jend = min(CH, k0 - jbeg - ch * CH);
        for (int jl = 0; jl < jend; ++jl) {
          const int jj = jbeg + ch * CH + jl;
          if (jj < js) continue;
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
                                           T* sPart, const int* Ej) {
  typedef PotrfCfg<T, NW, KB> Cfg;
  typedef typename Mfma<T>::acc Acc;
  const int fi = lane & 15, fg = lane >> 4;
  const int frag = fi * TS + 8 * fg;
  const int nit = 2 * (nt - k0);
  const int ns = min(Cfg::NWS / nit, k0);
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
    // slice sl takes jj = sl, sl + ns, ... (as in the dense order), from
    // the first of them at or right of the row's first nonzero tile
    const int e = Ej ? Ej[i] : 0;
    const int j0 = e > sl ? sl + (e - sl + ns - 1) / ns * ns : sl;
    V8<T> x0;
    if (j0 < k0) ld8(x0, X + (int64_t)j0 * TSQ);
    for (int jj = j0; jj < k0; jj += ns) {
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
__device__ __forceinline__ void bulk_direct(T* A, int nt, int k0, int kn, int w, int lane,
                                            const int* Ej, int rlast) {
  typedef typename Mfma<T>::acc Acc;
  const int fi = lane & 15, fg = lane >> 4;
  const int frag = fi * TS + 8 * fg;
  const int nit = 2 * (rlast - k0 + 1);
  for (int it = w; it < nit; it += NW) {
    const int i = k0 + (it >> 1), rq = it & 1;
    Acc acc[KB][2];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c][0] = acc[c][1] = acc_zero<T>();
    const T* X = A + tile_idx(i, 0) * TSQ + rq * 16 * TS + frag;
    const T* Y[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) Y[c] = A + tile_idx(k0 + min(c, kn - 1), 0) * TSQ + frag;
    const int js = Ej ? min(Ej[i], k0) : 0;
    V8<T> x0, y0[KB][2];
    if (js < k0) {
      ld8(x0, X + (int64_t)js * TSQ);
#pragma unroll
      for (int c = 0; c < KB; ++c)
#pragma unroll
        for (int cq = 0; cq < 2; ++cq) ld8(y0[c][cq], Y[c] + (int64_t)js * TSQ + cq * 16 * TS);
    }
    for (int jj = js; jj < k0; ++jj) {
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
                                           double pivtol, const int* __restrict__ envE,
                                           const int* __restrict__ envR) {
  typedef PotrfCfg<T, NW, KB> Cfg;
  typedef typename Mfma<T>::acc Acc;
  constexpr int LDI = Cfg::LDI;
  const int j = jobs[blockIdx.x];
  const int nt = ntl[j];
  T* A = tiles + toff[j] * TSQ;
  T* Di = dinv + doff[j] * TSQ;
  // envelope: rows i take tiles from column Ej[i] on; column k has
  // nonzero tiles down to row last(k)
  const int* Ej = envE ? envE + doff[j] : nullptr;
  const int* Rj = envR ? envR + doff[j] : nullptr;
  auto last = [&](int k) { return Rj ? min(max(Rj[k], k), nt - 1) : nt - 1; };
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
      // split only while every item gets at least one of the NWS slices
      const int rl = last(k0 + kn - 1);
      if (2 * (nt - k0) < Cfg::NWS) bulk_split<T, NW, KB>(A, nt, k0, kn, w, lane, sBuf, Ej);
      else if (STAGED) bulk_staged<T, NW, KB>(A, nt, k0, kn, w, tid, lane, sBuf, Ej, rl);
      else bulk_direct<T, NW, KB>(A, nt, k0, kn, w, lane, Ej, rl);
    }
    // ---- panel factorization
    for (int c = k0; c < k0 + kn; ++c) {
      if (c > k0) {
        // rank-32 update of the panel columns c' >= c with column c-1:
        // A(i, c') -= L(i, c-1) L(c', c-1)^T for i >= c'
        // (rows below last(pc) have a zero tile in column pc)
        const int pc = c - 1, rl = last(pc);
        int nit = 0;
        for (int cc = c; cc < k0 + kn; ++cc) nit += 2 * max(0, rl + 1 - cc);
        for (int it = w; it < nit; it += NW) {
          int cc = c, rem = it;
          while (rem >= 2 * max(0, rl + 1 - cc)) rem -= 2 * max(0, rl + 1 - cc++);
          const int i = cc + (rem >> 1), rq = rem & 1;
          V8<T> x, y[2];
          ld8(x, A + tile_idx(i, pc) * TSQ + rq * 16 * TS + frag);
#pragma unroll
          for (int cq = 0; cq < 2; ++cq) ld8(y[cq], A + tile_idx(cc, pc) * TSQ + cq * 16 * TS + frag);
          Acc acc[2] = {acc_zero<T>(), acc_zero<T>()};
#pragma unroll
          for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int cq = 0; cq < 2; ++cq) acc[cq] = Mfma<T>::run(x.v[s], y[cq].v[s], acc[cq]);
          T* C = A + tile_idx(i, cc) * TSQ + rq * 16 * TS;
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
      // L(i, c) = A(i, c) Dinv(c)^T for c < i <= last(c)
      const int nit = 2 * (last(c) - c);
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

// Wavefronts of the FP32 local factorisation: its registers (128) and LDS
// (one workgroup per CU) allow 16, which gives the bulk updates twice the
// items in flight of the FP64 kernels (whose registers allow 8).
#define POTRF32_NW 16

// One entry point per role, so that traces and profiles tell them apart:
// local Dirichlet factors (FP32, or FP64 for the subdomains that fail the
// FP32 pivot test) and the shifted Neumann factors of the eigensolver.
__global__ __launch_bounds__(POTRF32_NW * 64) void k_potrf_local_f32(
    float* tiles, const int64_t* toff, const int* nt, float* dinv, const int64_t* doff,
    int* status, const int* jobs, double pivtol, const int* envE, const int* envR) {
  potrf_body<float, POTRF32_NW, 4, true>(tiles, toff, nt, dinv, doff, status, jobs, pivtol, envE,
                                         envR);
}
__global__ __launch_bounds__(512) void k_potrf_local_f64(
    double* tiles, const int64_t* toff, const int* nt, double* dinv, const int64_t* doff,
    int* status, const int* jobs, double pivtol, const int* envE, const int* envR) {
  potrf_body<double, 8, 4, true>(tiles, toff, nt, dinv, doff, status, jobs, pivtol, envE, envR);
}
#define POTRF64S_NW 12
__global__ __launch_bounds__(POTRF64S_NW * 64) void k_potrf_shifted_f64(
    double* tiles, const int64_t* toff, const int* nt, double* dinv, const int64_t* doff,
    int* status, const int* jobs, double pivtol, const int* envE, const int* envR) {
  potrf_body<double, POTRF64S_NW, 4, true>(tiles, toff, nt, dinv, doff, status, jobs, pivtol,
                                           envE, envR);
}

hipError_t launch_chol_batched(CholRole role, void* tiles, const int64_t* toff, const int* nt,
                               void* dinv, const int64_t* doff, int* status, const int* jobs,
                               int njobs, double pivtol, const int* envE, const int* envR,
                               hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  if (!envE != !envR) return hipErrorInvalidValue;
  const dim3 grid(njobs), blk(512);
  switch (role) {
    case CholRole::LocalF32:
      hipLaunchKernelGGL(k_potrf_local_f32, grid, dim3(POTRF32_NW * 64), 0, st, (float*)tiles, toff, nt,
                         (float*)dinv, doff, status, jobs, pivtol, envE, envR);
      break;
    case CholRole::LocalF64:
      hipLaunchKernelGGL(k_potrf_local_f64, grid, blk, 0, st, (double*)tiles, toff, nt,
                         (double*)dinv, doff, status, jobs, pivtol, envE, envR);
      break;
    case CholRole::ShiftedF64:
      hipLaunchKernelGGL(k_potrf_shifted_f64, grid, dim3(POTRF64S_NW * 64), 0, st, (double*)tiles, toff, nt,
                         (double*)dinv, doff, status, jobs, pivtol, envE, envR);
      break;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------
// k_trtri_win: X = L^{-1}, one workgroup per (matrix, block of NCT tile
// columns C = c0 .. c0+NCT-1): forward substitution L X(:, C) = E_C over the
// rows c0 .. nt-1 (b = 32 NCT right-hand sides).  The rows are taken in
// windows of 16 tile rows held in registers (FP32: 16 wavefronts, one
// window row each; FP64: 8 wavefronts, wavefront w owns rows w and w + 8).
// Each window first takes its update from the finished rows (left-looking;
// the tiles L(k, jj) are streamed with the next one prefetched), then is
// solved right-looking: the owner of row i forms
// X(i, C) = Dinv(i) acc_i and publishes it, transposed, in LDS; after one
// barrier every wavefront subtracts L(k, i) X(i, C) from its later rows.
// Tiles above the diagonal (column tile > row) are zero: never read or
// written.  Two tile columns per workgroup (FP32) halve the reads of L.
// The tiles of X are stored transposed (tile (i, k) holds X(i, k)^T), the
// layout in which k_lauum reads them.
// wavefronts per workgroup and window rows per wavefront: FP32 16 x 1 (its
// 112 registers allow 4 wavefronts per SIMD), FP64 8 x 2
template <typename T> struct TwCfg {
  static constexpr int NW = sizeof(T) == 4 ? 16 : 8;
  static constexpr int MR = sizeof(T) == 4 ? 1 : 2;
};

template <typename T, int NCT>
__global__ __launch_bounds__(TwCfg<T>::NW * 64) void k_trtri_win(const T* __restrict__ L,
                                                          const T* __restrict__ dinv,
                                                          T* __restrict__ X,
                                                          const int64_t* __restrict__ toff,
                                                          const int64_t* __restrict__ doff,
                                                          const int* __restrict__ ntl,
                                                          const int2* __restrict__ jobs,
                                                          const int* __restrict__ envE) {
  typedef typename Mfma<T>::acc Acc;
  constexpr int NCQ = 2 * NCT, b = 32 * NCT, LDI = DiagLd<T>::v;
  constexpr int TW_NW = TwCfg<T>::NW, TW_MR = TwCfg<T>::MR, TW_W = TW_NW * TW_MR;
  const int j = jobs[blockIdx.x].x, c0 = jobs[blockIdx.x].y;
  const int nt = ntl[j];
  if (c0 >= nt) return;
  // envelope of L (NULL: dense): row k of L is zero left of tile column
  // E(k), so its products there are skipped (X itself is dense)
  const int* Ej = envE ? envE + doff[j] : nullptr;
  auto first = [&](int k) { return Ej ? Ej[k] : 0; };
  const T* Lj = L + toff[j] * TSQ;
  const T* Dj = dinv + doff[j] * TSQ;
  T* Xj = X + toff[j] * TSQ;
  __shared__ __align__(16) T sTmp[b * LDI];
  __shared__ __align__(16) T sX[2][b * LDI];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int fi = lane & 15, fg = lane >> 4;
  auto mma = [&](Acc (&acc)[2][NCQ], const V8<T> (&a)[2], const V8<T>& bf, int cq) {
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int rq = 0; rq < 2; ++rq) acc[rq][cq] = Mfma<T>::run(a[rq].v[s], bf.v[s], acc[rq][cq]);
  };
  // B fragment of X(jj, C) from memory: column cq*16 + fi of the block,
  // rows 8 fg .. 8 fg + 7 of tile (jj, c0 + cq / 2), i.e. 8 consecutive
  // entries of a row of the stored (transposed) tile; zero above the diagonal
  // X(jj, tc) is zero for tc > jj: the load is issued anyway (from a tile
  // in range) and the values replaced, so the number of loads in flight is
  // the same on every path
  auto bfrag_mem = [&](V8<T>& f, int jj, int cq) {
    const int tc = c0 + (cq >> 1);
    ld8(f, Xj + tile_idx(jj, min(tc, jj)) * TSQ + ((cq & 1) * 16 + fi) * TS + 8 * fg);
    if (tc > jj) {
#pragma unroll
      for (int s = 0; s < 8; ++s) f.v[s] = (T)0;
    }
  };
  auto bfrag_lds = [&](V8<T>& f, const T* sT, int cq) {
    const T* p = sT + (cq * 16 + fi) * LDI + 8 * fg;
#pragma unroll
    for (int s = 0; s < 8; ++s) f.v[s] = p[s];
  };
  auto afrag = [&](V8<T> (&a)[2], const T* t) {
#pragma unroll
    for (int rq = 0; rq < 2; ++rq) ld8(a[rq], t + (rq * 16 + fi) * TS + 8 * fg);
  };
  for (int p0 = c0; p0 < nt; p0 += TW_W) {
    const int p1 = min(nt, p0 + TW_W);
    Acc acc[TW_MR][2][NCQ];
    int krow[TW_MR];
#pragma unroll
    for (int m = 0; m < TW_MR; ++m) {
      krow[m] = p0 + w + TW_NW * m;
#pragma unroll
      for (int rq = 0; rq < 2; ++rq)
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = rq * 16 + acc_row<T>(lane, v), col = cq * 16 + acc_col(lane);
            acc[m][rq][cq][v] = (krow[m] == c0 + (col >> 5) && r == (col & 31)) ? (T)-1 : (T)0;
          }
    }
    // acc holds -E + the products so far (negation is exact: bitwise the
    // negated E - products), negated again where the owner reads it
    // ---- update from the finished rows c0 .. p0-1
#pragma unroll
    for (int m = 0; m < TW_MR; ++m) {
      const int k = krow[m];
      if (k >= p1 || p0 == c0) continue;
      const int jlo = max(c0, first(k));
      if (jlo >= p0) continue;
      // X(jj, .) loaded before the next factor tile, two tile buffers
      // alternating: the wait for X leaves the next tile in flight
      auto step = [&](const V8<T> (&cur)[2], V8<T> (&nxt)[2], int jj) {
        V8<T> bf[NCQ];
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq) bfrag_mem(bf[cq], jj, cq);
        afrag(nxt, Lj + tile_idx(k, min(jj + 1, p0 - 1)) * TSQ);
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq) mma(acc[m], cur, bf[cq], cq);
      };
      V8<T> a0[2], a1[2];
      afrag(a0, Lj + tile_idx(k, jlo) * TSQ);
      int jj = jlo;
      for (; jj + 1 < p0; jj += 2) {
        step(a0, a1, jj);
        step(a1, a0, jj + 1);
      }
      if (jj < p0) step(a0, a1, jj);
    }
    // ---- right-looking solve inside the window
    for (int st = 0; st < p1 - p0; ++st) {
      const int i = p0 + st, ow = st % TW_NW, om = st / TW_NW;
      T* sXo = sX[st & 1];
      if (w == ow) {
#pragma unroll
        for (int m = 0; m < TW_MR; ++m) {
          if (m != om) continue;
#pragma unroll
          for (int rq = 0; rq < 2; ++rq)
#pragma unroll
            for (int cq = 0; cq < NCQ; ++cq)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                sTmp[(cq * 16 + acc_col(lane)) * LDI + rq * 16 + acc_row<T>(lane, v)] = -acc[m][rq][cq][v];
          wave_sync();
          V8<T> a[2];
#pragma unroll
          for (int rq = 0; rq < 2; ++rq) ld8(a[rq], Dj + (int64_t)i * TSQ + (rq * 16 + fi) * TS + 8 * fg);
          Acc o[2][NCQ];
#pragma unroll
          for (int rq = 0; rq < 2; ++rq)
#pragma unroll
            for (int cq = 0; cq < NCQ; ++cq) o[rq][cq] = acc_zero<T>();
#pragma unroll
          for (int cq = 0; cq < NCQ; ++cq) {
            V8<T> bf;
            bfrag_lds(bf, sTmp, cq);
            mma(o, a, bf, cq);
          }
#pragma unroll
          for (int rq = 0; rq < 2; ++rq)
#pragma unroll
            for (int cq = 0; cq < NCQ; ++cq) {
              const int tc = c0 + (cq >> 1);
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int r = rq * 16 + acc_row<T>(lane, v), col = cq * 16 + acc_col(lane);
                sXo[col * LDI + r] = o[rq][cq][v];
              }
              if (tc > i) continue;
              // stored transposed: row (col & 31) of the tile holds column col of X
              T* dst = Xj + tile_idx(i, tc) * TSQ + ((cq & 1) * 16 + acc_col(lane)) * TS + rq * 16;
              if constexpr (sizeof(T) == 4) {
                *reinterpret_cast<float4*>(dst + 4 * (lane >> 4)) =
                    make_float4(o[rq][cq][0], o[rq][cq][1], o[rq][cq][2], o[rq][cq][3]);
              } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) dst[acc_row<T>(lane, v)] = o[rq][cq][v];
              }
            }
        }
      }
      block_sync();
#pragma unroll
      for (int m = 0; m < TW_MR; ++m) {
        const int k = krow[m];
        if (k >= p1 || k <= i || first(k) > i) continue;
        V8<T> a[2];
        afrag(a, Lj + tile_idx(k, i) * TSQ);
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq) {
          V8<T> bf;
          bfrag_lds(bf, sXo, cq);
          mma(acc[m], a, bf, cq);
        }
      }
    }
    block_sync();
  }
}

int trtri_cols_per_job(bool fp32) { return fp32 ? 2 : 1; }

hipError_t launch_trtri(bool fp32, const void* L, const void* dinv, void* X,
                        const int64_t* toff, const int64_t* doff, const int* nt,
                        const int2* jobs, int njobs, const int* envE, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL((k_trtri_win<float, 2>), dim3(njobs), dim3(TwCfg<float>::NW * 64), 0, st,
                       (const float*)L, (const float*)dinv, (float*)X, toff, doff, nt, jobs,
                       envE);
  else
    hipLaunchKernelGGL((k_trtri_win<double, 1>), dim3(njobs), dim3(TwCfg<double>::NW * 64), 0, st,
                       (const double*)L, (const double*)dinv, (double*)X, toff, doff, nt, jobs,
                       envE);
  return hipGetLastError();
}

// k_lauum: the symmetric inverse S = X^T X = A^{-1} from the inverse factor
// X = L^{-1} (transposed tiles, as k_trtri_win leaves them): S(I, J) =
// sum_{K >= I} X(K, I)^T X(K, J) for J <= I, written row-major in the packed
// format, the diagonal tiles in full.  One wavefront per two output tiles
// (J, J + 1) of a tile row, which share the fragments of X(K, I); the
// LA_NW wavefronts of a workgroup take consecutive pairs of one tile row,
// so they also read the same X(K, I) (served from L1).  With the transposed
// tiles both operands of every product are rows of stored tiles: each lane
// reads 8 consecutive entries (two vector loads) per fragment, the next
// K's fragments loaded while the current ones are multiplied.  Jobs come
// matrix by matrix; blocks are handed to the 8 XCDs in contiguous slices of
// the job list (block b runs on XCD b % 8), so each XCD works on its own
// matrices and keeps their factors in its L2.
#define LA_NW 4
#define LA_TW 2  // output tiles per wavefront

template <typename T>
__global__ __launch_bounds__(LA_NW * 64) void k_lauum(const T* __restrict__ XT, T* __restrict__ S,
                                                      const int64_t* __restrict__ toff,
                                                      const int* __restrict__ ntl,
                                                      const int2* __restrict__ jobs, int njobs,
                                                      int per_xcd) {
  typedef typename Mfma<T>::acc Acc;
  const int q = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (q >= njobs) return;
  const int2 jb = jobs[q];
  // wavefront w takes the output tiles J and J + 1 of row I: both use the
  // fragments of X(K, I), loaded once per K for the two
  const int j = jb.x, I = jb.y >> 16, J = (jb.y & 0xffff) + LA_TW * (threadIdx.x >> 6);
  if (J > I) return;  // no barriers below: a wavefront may leave early
  const bool two = J + 1 <= I;
  const int J1 = two ? J + 1 : J;  // a second copy of tile J when J + 1 > I (not stored)
  const int nt = ntl[j];
  const int lane = threadIdx.x & 63, fi = lane & 15, fg = lane >> 4;
  const T* Xj = XT + toff[j] * TSQ + fi * TS + 8 * fg;
  Acc acc[2][2][2];
#pragma unroll
  for (int o = 0; o < 2; ++o)
#pragma unroll
    for (int rq = 0; rq < 2; ++rq)
#pragma unroll
      for (int cq = 0; cq < 2; ++cq) acc[o][rq][cq] = acc_zero<T>();
  struct Ops {
    V8<T> a[2], b[2][2];
  };
  auto load = [&](Ops& f, int K) {
    const T* ta = Xj + tile_idx(K, I) * TSQ;
    const T* tb0 = Xj + tile_idx(K, J) * TSQ;
    const T* tb1 = Xj + tile_idx(K, J1) * TSQ;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      ld8(f.a[h], ta + h * 16 * TS);
      ld8(f.b[0][h], tb0 + h * 16 * TS);
      ld8(f.b[1][h], tb1 + h * 16 * TS);
    }
  };
  // two operand sets alternate (K unrolled by two): a register copy of a
  // load in flight would wait for it, so K + 1's loads are issued into the
  // other set and stay in flight during K's products; each tile's products
  // are added in K order, as with one tile per wavefront
  auto step = [&](const Ops& c, Ops& n, int K) {
    load(n, K + 1 < nt ? K + 1 : K);
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int rq = 0; rq < 2; ++rq)
#pragma unroll
          for (int cq = 0; cq < 2; ++cq)
            acc[o][rq][cq] = Mfma<T>::run(c.a[rq].v[s], c.b[o][cq].v[s], acc[o][rq][cq]);
  };
  Ops f0, f1;
  load(f0, I);
  int K = I;
  for (; K + 1 < nt; K += 2) {
    step(f0, f1, K);
    step(f1, f0, K + 1);
  }
  if (K < nt) step(f0, f1, K);
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    if (o == 1 && !two) break;
    T* Sj = S + (toff[j] + tile_idx(I, J + o)) * TSQ;
#pragma unroll
    for (int rq = 0; rq < 2; ++rq)
#pragma unroll
      for (int cq = 0; cq < 2; ++cq)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          Sj[(rq * 16 + acc_row<T>(lane, v)) * TS + cq * 16 + acc_col(lane)] = acc[o][rq][cq][v];
  }
}

int lauum_tiles_per_job() { return LA_NW * LA_TW; }

hipError_t launch_lauum(bool fp32, const void* XT, void* S, const int64_t* toff, const int* nt,
                        const int2* jobs, int njobs, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  const int per = (njobs + 7) / 8;
  if (fp32)
    hipLaunchKernelGGL(k_lauum<float>, dim3(8 * per), dim3(LA_NW * 64), 0, st,
                       (const float*)XT, (float*)S, toff, nt, jobs, njobs, per);
  else
    hipLaunchKernelGGL(k_lauum<double>, dim3(8 * per), dim3(LA_NW * 64), 0, st,
                       (const double*)XT, (double*)S, toff, nt, jobs, njobs, per);
  return hipGetLastError();
}

// ------------------------------------------------------- coarse matrix ---
// Right-looking Cholesky by tile-column steps, batched over matrices
// jobs[blockIdx.y] (tiles at toff, inverted diagonal tiles at doff): step k
// factors and inverts the diagonal tile (one wavefront), forms the column
// panel L_ik = A_ik Linv_kk^T (one workgroup per tile) and updates the
// trailing matrix A_ij -= L_ik L_jk^T (one workgroup per tile).  For a few
// matrices (the coarse matrix, the FP64 refactors of mixed mode) this uses
// many short workgroups instead of holding one CU per matrix for the whole
// factorisation.  status[j] = 0, or TS k + f at the first failed pivot
// (set by step 0, later steps then skip the matrix).
__global__ __launch_bounds__(64) void k_step_potrf(double* __restrict__ A, double* __restrict__ Di,
                                                   const int64_t* __restrict__ toff,
                                                   const int64_t* __restrict__ doff,
                                                   const int* __restrict__ ntl,
                                                   const int* __restrict__ jobs, int k,
                                                   int* __restrict__ status,
                                                   const double* __restrict__ pivtol) {
  __shared__ double sRp[TS];
  const int j = jobs[blockIdx.x];
  if (k >= ntl[j] || (k > 0 && status[j])) return;
  double* D = A + (toff[j] + tile_idx(k, k)) * TSQ;
  const int f = diag_tile_body<double, TS + 2>(D, D, Di + (doff[j] + k) * TSQ, nullptr, sRp,
                                               threadIdx.x, pivtol ? *pivtol : 0.0);
  if (threadIdx.x == 0 && (f || k == 0)) status[j] = f ? k * TS + f : 0;
}

// L_ik = A_ik Linv_kk^T, one workgroup per tile i > k (down to the last
// nonzero tile R(k) of column k when the envelope envR is given)
__global__ __launch_bounds__(256) void k_step_trsm(double* __restrict__ A,
                                                   const double* __restrict__ Di,
                                                   const int64_t* __restrict__ toff,
                                                   const int64_t* __restrict__ doff,
                                                   const int* __restrict__ ntl,
                                                   const int* __restrict__ jobs, int k,
                                                   const int* __restrict__ status,
                                                   const int* __restrict__ envR) {
  const int j = jobs[blockIdx.y];
  const int i = k + 1 + blockIdx.x;
  if (i >= ntl[j] || status[j]) return;
  if (envR && i > envR[doff[j] + k]) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rq = w >> 1, cq = w & 1;
  double* X = A + (toff[j] + tile_idx(i, k)) * TSQ;
  const double* Y = Di + (doff[j] + k) * TSQ;
  d4_t acc = acc_zero<double>();
  q_xyT<double>(acc, X + rq * 16 * TS, TS, Y + cq * 16 * TS, TS, lane);
  block_sync();
#pragma unroll
  for (int v = 0; v < 4; ++v) X[(rq * 16 + acc_row<double>(lane, v)) * TS + cq * 16 + acc_col(lane)] = acc[v];
}

// A_ij -= L_ik L_jk^T for k < j <= i (<= R(k) with the envelope: below it
// L_ik is zero); blockIdx.x enumerates the trailing tiles
__global__ __launch_bounds__(256) void k_step_update(double* __restrict__ A,
                                                     const int64_t* __restrict__ toff,
                                                     const int64_t* __restrict__ doff,
                                                     const int* __restrict__ ntl,
                                                     const int* __restrict__ jobs, int k,
                                                     const int* __restrict__ status,
                                                     const int* __restrict__ envR) {
  const int j = jobs[blockIdx.y];
  const int nt = ntl[j];
  if (status[j]) return;
  // map blockIdx.x -> (i, jj) over the lower triangle of the trailing matrix
  int t = blockIdx.x;
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
  while ((int64_t)i * (i + 1) / 2 > t) --i;
  int jj = t - i * (i + 1) / 2;
  i += k + 1;
  jj += k + 1;
  if (i >= nt) return;
  if (envR && i > envR[doff[j] + k]) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rq = w >> 1, cq = w & 1;
  if (i == jj && rq == 0 && cq == 1) return;
  const double* Aj = A + toff[j] * TSQ;
  d4_t acc = acc_zero<double>();
  q_xyT<double>(acc, Aj + tile_idx(i, k) * TSQ + rq * 16 * TS, TS,
                Aj + tile_idx(jj, k) * TSQ + cq * 16 * TS, TS, lane);
  double* C = A + (toff[j] + tile_idx(i, jj)) * TSQ + rq * 16 * TS + cq * 16;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[acc_row<double>(lane, v) * TS + acc_col(lane)] -= acc[v];
}

hipError_t launch_chol_steps(double* tiles, double* dinv, const int64_t* toff,
                             const int64_t* doff, const int* nt, const int* jobs, int njobs,
                             int maxnt, int* status, hipStream_t st, const double* pivtol,
                             const int* envR, const int* rlast) {
  if (njobs <= 0) return hipSuccess;
  for (int k = 0; k < maxnt; ++k) {
    hipLaunchKernelGGL(k_step_potrf, dim3(njobs), dim3(64), 0, st, tiles, dinv, toff, doff, nt,
                       jobs, k, status, pivtol);
    // tile rows below the diagonal that the step reaches
    const int rem = (rlast ? std::min(rlast[k], maxnt - 1) : maxnt - 1) - k;
    if (rem > 0) {
      hipLaunchKernelGGL(k_step_trsm, dim3(rem, njobs), dim3(256), 0, st, tiles, dinv, toff,
                         doff, nt, jobs, k, status, envR);
      hipLaunchKernelGGL(k_step_update, dim3(rem * (rem + 1) / 2, njobs), dim3(256), 0, st,
                         tiles, toff, doff, nt, jobs, k, status, envR);
    }
  }
  return hipGetLastError();
}

}  // namespace geneo
