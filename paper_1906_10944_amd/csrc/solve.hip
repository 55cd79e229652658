// Local solves, triangular solves with the packed tile factors, and products
// with packed symmetric inverses.
//
//  * k_local_solve_f32 / _f64: the local Dirichlet solves of the apply in
//    the triangular form, y = L^{-T} L^{-1} x with each subdomain's banded
//    Cholesky factor (FP32 or FP64), one workgroup per subdomain, inside
//    the factor's tile envelope.  Bound by two reads of the envelope and by
//    the latency of the row-by-row substitution.
//  * k_symv_rows / k_symv_cols: y = S x for the symmetric inverses S =
//    A^{-1} of the local Dirichlet matrices (in the inverse form) and of
//    the coarse matrix, all in one launch each.  The first reads every
//    stored tile once (one wavefront per chunk of up to 8 tiles of a tile
//    row) and leaves partial sums: its chunk's share of the row sums and
//    the transposed products of the off-diagonal tiles; the second adds
//    those in a fixed order.  HBM-bound on the one read of S.
//  * k_trsm_win: X = G^{-1} R and X = G^{-T} R with b <= 32 right-hand sides
//    for the shift-and-invert eigen sweeps (FP64, one workgroup per
//    subdomain): windows of 16 tile rows held in registers, a left-looking
//    update from the finished rows, then right-looking substitution inside
//    the window with the inverted diagonal tiles.
//  * k_trsm_w1: the same with one tile row per wavefront (windows of 8)
//    and deeper load pipelines (b <= 48).  Both kernels also run on 16-
//    column blocks of the right-hand sides, b / 16 workgroups per subdomain,
//    for sweeps with fewer active subdomains than compute units.
//  * k_trsm_fwd / k_trsm_bwd: the same solves row by row for b = 64
//    (inner sums split over tile slices, reduced in LDS).
//  * k_bapply: Y = X_j A^o_j X_j X (the B-matrix of the GenEO eigenproblem),
//    from a compact copy of B_j built once per setup (k_bcompact), on the
//    rows of B_j that hold entries only.
#include "internal.h"

namespace geneo {

// Tiles of a tile row per row partial of the symmetric product (a wavefront
// takes one or more such groups).
#define SYMV_CHUNK 8

// Four consecutive entries of a tile row as stored (raw, converted to FP64
// only where they are used, so a prefetched tile costs 16 / 32 VGPRs).  The
// inverses are streamed once per apply with nontemporal loads, which keeps
// them from displacing the vectors and partial sums in the caches (those
// are then read back by k_symv_cols without going to HBM).
template <typename T> struct Piece;
template <> struct Piece<float> {
  float4 v;
  __device__ __forceinline__ void load(const float* p) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v t = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    v = make_float4(t[0], t[1], t[2], t[3]);
  }
  __device__ __forceinline__ double at(int q) const {
    return (double)(q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w);
  }
};
template <> struct Piece<double> {
  double2 u, w;
  __device__ __forceinline__ void load(const double* p) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v a = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
    const d2v b = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p) + 1);
    u = make_double2(a[0], a[1]);
    w = make_double2(b[0], b[1]);
  }
  __device__ __forceinline__ double at(int q) const {
    return q == 0 ? u.x : q == 1 ? u.y : q == 2 ? w.x : w.y;
  }
};

// Tiles k0 .. k1-1 of row i of y = S x for a symmetric inverse S (packed
// lower tiles, the diagonal tiles in full), in groups of SYMV_CHUNK tiles
// (k0 a multiple of it).  A group's share of y_i = sum_{k<=i} S_ik x_k goes
// to its row partial (32 sums at R + TS g for group g), and for k < i the
// transposed product S_ik^T x_i of each tile to W(i, k) (32 sums): every
// tile is read once, both partials are added in a fixed order by
// k_symv_cols.  Lane (column group l%8, row l/8) loads the
// 4-column pieces of rows l/8 + 8m (m < 4) of a tile with vector loads,
// with the 4 entries of x_k they multiply; NB tiles are loaded at a time
// (NB = 4 for FP32 tiles, 2 for FP64: 16 KB in flight per wavefront) and
// nothing stays in flight from one batch to the next.  The row sums stay
// in the lane until the end; the column sums are reduced over the 8 lanes
// of a column group per tile, the 4 sums of a lane spread over the group as
// they are reduced (4 exchanges instead of 12).  FP64 arithmetic.
template <typename T, int NB = (sizeof(T) == 4 ? 4 : 2)>
__device__ __forceinline__ void symv_chunk(const T* __restrict__ Srow, int i, int k0, int k1,
                                           const double* __restrict__ xv, double* __restrict__ R,
                                           T* __restrict__ Wrow, int lane) {
  const int cg = lane & 7, r0 = lane >> 3;
  const bool h3 = lane & 8, h4 = lane & 16;
  const T* Sr = Srow + r0 * TS + cg * 4;
  const double* xg = xv + cg * 4;
  double xi[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) xi[m] = xv[i * TS + r0 + 8 * m];
  double s[4];
  int kend = k1;  // end of the current group of tiles
  struct Buf {
    Piece<T> a[4];
    double2 x01, x23;
  };
  auto load = [&](Buf& b, int k) {
    const int kk = min(k, kend - 1);
    const T* t = Sr + (int64_t)kk * TSQ;
#pragma unroll
    for (int m = 0; m < 4; ++m) b.a[m].load(t + 8 * m * TS);
    b.x01 = *reinterpret_cast<const double2*>(xg + kk * TS);
    b.x23 = *reinterpret_cast<const double2*>(xg + kk * TS + 2);
  };
  // tile k (in cur) into the row sums; for k < i returns this lane's share
  // of the transposed product
  auto use = [&](const Buf& cur, bool offdiag) -> double {
    const Piece<T>(&a)[4] = cur.a;
    const double2 x01 = cur.x01, x23 = cur.x23;
#pragma unroll
    for (int m = 0; m < 4; ++m)
      s[m] += a[m].at(0) * x01.x + a[m].at(1) * x01.y + a[m].at(2) * x23.x + a[m].at(3) * x23.y;
    if (!offdiag) return 0.0;
    double c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      c[q] = a[0].at(q) * xi[0] + a[1].at(q) * xi[1] + a[2].at(q) * xi[2] + a[3].at(q) * xi[3];
    // bit 3: keep columns 2h3, 2h3+1, pass the other two; bit 4: keep
    // column 2h3+h4; bit 5: plain sum.  Lanes 0..31 then hold the 32 sums.
    double e0 = h3 ? c[2] : c[0], e1 = h3 ? c[3] : c[1];
    const double o0 = h3 ? c[0] : c[2], o1 = h3 ? c[1] : c[3];
    e0 += __shfl_xor(o0, 8);
    e1 += __shfl_xor(o1, 8);
    double e = h4 ? e1 : e0;
    const double f = h4 ? e0 : e1;
    e += __shfl_xor(f, 16);
    e += __shfl_xor(e, 32);
    return e;
  };
  // groups of SYMV_CHUNK tiles, each with its own row partial: the sums do
  // not depend on how many groups one wavefront takes
  for (int g0 = k0, gi = 0; g0 < k1; g0 += SYMV_CHUNK, ++gi) {
    kend = min(g0 + SYMV_CHUNK, k1);
#pragma unroll
    for (int m = 0; m < 4; ++m) s[m] = 0.0;
    for (int k = g0; k < kend; k += NB) {
      Buf b[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) load(b[u], k + u);
      // keep the loads ahead of the arithmetic
      __builtin_amdgcn_sched_barrier(0);
      double e[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) e[u] = k + u < kend ? use(b[u], k + u < i) : 0.0;
      if (lane < 32) {
#pragma unroll
        for (int u = 0; u < NB; ++u)
          if (k + u < kend && k + u < i) Wrow[(k + u) * TS + cg * 4 + 2 * h3 + h4] = (T)e[u];
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      s[m] += __shfl_xor(s[m], 1);
      s[m] += __shfl_xor(s[m], 2);
      s[m] += __shfl_xor(s[m], 4);
    }
    if (cg == 0) {
#pragma unroll
      for (int m = 0; m < 4; ++m) R[gi * TS + r0 + 8 * m] = s[m];
    }
  }
}

int symv_chunk_tiles() { return SYMV_CHUNK; }

// The task lists of the symmetric products, one workgroup per job, one
// thread per tile row: row i has ceil((i + 1) / SYMV_CHUNK) chunks, taken
// g at a time; its tasks follow those of rows 0 .. i-1 (a closed form), at
// the job's offsets in the forward and the reverse list.
__global__ __launch_bounds__(256) void k_symv_tasks(const SymvJob* __restrict__ jobs, int g,
                                                    int nchunk, SymvTask* __restrict__ fwd,
                                                    SymvTask* __restrict__ rev) {
  const int q = blockIdx.x;
  const SymvJob jb = jobs[q];
  const int G = g * SYMV_CHUNK;
  for (int i = threadIdx.x; i < jb.nt; i += blockDim.x) {
    const int64_t p0 = symv_tasks_before(i, G);
    const int c0 = (int)symv_tasks_before(i, SYMV_CHUNK);  // first chunk of row i
    const int ntk = (i + G) / G;
    for (int u = 0; u < ntk; ++u) {
      SymvTask k;
      k.s_row = (jb.toff + tile_idx(i, 0)) * TSQ;
      k.w_row = (jb.toff + tile_idx(i, 0)) * TS;
      k.xoff = jb.xoff;
      k.r_off = (q * nchunk + c0 + u * g) * TS;
      k.i = (short)i;
      k.k0 = (short)(u * G);
      k.k1 = (short)min(u * G + G, i + 1);
      k.kind = (short)jb.kind;
      fwd[jb.off_f + p0 + u] = k;
      if (rev) rev[jb.off_r + p0 + u] = k;
    }
  }
}

hipError_t symv_make_tasks(const SymvJob* jobs, int njobs, int g, int nchunk, SymvTask* fwd,
                           SymvTask* rev, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_symv_tasks, dim3(njobs), dim3(256), 0, st, jobs, g, nchunk, fwd, rev);
  return hipGetLastError();
}

// One launch for all subdomains and the coarse problem, one wavefront per
// task (a chunk of up to SYMV_CHUNK tiles of a tile row), whose
// descriptor is the wavefront's only dependent load before it streams
// tiles.  The tasks of a job are consecutive; the host passes the tasks in
// one of two walk orders over the jobs, alternating between applies, so
// each apply starts on the matrices the previous one read last, which are
// still in the Infinity Cache.
__global__ __launch_bounds__(64) void k_symv_rows(SymvArgs A, const int* __restrict__ done) {
  if (done && *done) return;
  const SymvTask tk = A.tasks[blockIdx.x];
  const int lane = threadIdx.x;
  double* R = A.R + tk.r_off;
  if (tk.kind == 2)
    symv_chunk<double>(A.SH + tk.s_row, tk.i, tk.k0, tk.k1, A.xH, R, A.WH + tk.w_row, lane);
  else if (tk.kind == 1)
    symv_chunk<double>(A.S64 + tk.s_row, tk.i, tk.k0, tk.k1, A.x + tk.xoff, R, A.W64 + tk.w_row,
                       lane);
  else
    symv_chunk<float>(A.S32 + tk.s_row, tk.i, tk.k0, tk.k1, A.x + tk.xoff, R, A.W32 + tk.w_row,
                      lane);
}

// y_k = sum of the row partials of row k (chunks in order) + sum_{i>k}
// W(i, k) (i ascending): thread (tile column blockIdx.x * 8 + tid / 32,
// entry tid % 32) of job blockIdx.y.
template <typename T>
__device__ __forceinline__ void symv_col(const T* __restrict__ Wj, const double* __restrict__ Rq,
                                         const int* __restrict__ cstart, int k, int nt, int c,
                                         double* __restrict__ yv) {
  double acc = 0.0;
  for (int t = cstart[k]; t < cstart[k + 1]; ++t) acc += Rq[t * TS + c];
  int i = k + 1;
  // eight loads in flight, added in order
  for (; i + 8 <= nt; i += 8) {
    T w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = Wj[tile_idx(i + u, k) * TS + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (double)w[u];
  }
  for (; i < nt; ++i) acc += (double)Wj[tile_idx(i, k) * TS + c];
  yv[k * TS + c] = acc;
}

__global__ __launch_bounds__(256) void k_symv_cols(SymvArgs A, const int* __restrict__ done) {
  if (done && *done) return;
  const int q = blockIdx.y;
  const int2 jb = A.jobs[q];
  const int k = blockIdx.x * 8 + (threadIdx.x >> 5), c = threadIdx.x & 31;
  const double* Rq = A.R + (int64_t)q * A.nchunk * TS;
  if (jb.y == 2) {
    if (k < A.ntc) symv_col<double>(A.WH, Rq, A.cstart, k, A.ntc, c, A.yH);
    return;
  }
  const int j = jb.x, nt = A.nt[j];
  if (k >= nt) return;
  double* yv = A.y + A.voff[j];
  if (jb.y) symv_col<double>(A.W64 + A.toff64[j] * TS, Rq, A.cstart, k, nt, c, yv);
  else symv_col<float>(A.W32 + A.toff32[j] * TS, Rq, A.cstart, k, nt, c, yv);
}

hipError_t symv_rows(const SymvArgs& a, const int* done, hipStream_t st) {
  if (a.ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_symv_rows, dim3(a.ntasks), dim3(64), 0, st, a, done);
  return hipGetLastError();
}

hipError_t symv_cols(const SymvArgs& a, const int* done, hipStream_t st) {
  if (a.njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_symv_cols, dim3((a.maxnt + 7) / 8, a.njobs), dim3(256), 0, st, a, done);
  return hipGetLastError();
}

// ------------------------------------------------------ local solves ---
// y = L^{-T} L^{-1} x for one subdomain's banded Cholesky factor, one
// workgroup of NW wavefronts per subdomain, all of its vector in LDS
// (FP64).  Forward, tile row i: s_i = x_i - sum_{E(i) <= k < i} L_ik y_k,
// y_i = Dinv_i s_i; backward, in place: t_i = y_i - sum_{i < k <= R(i)}
// L_ki^T z_k, z_i = Dinv_i^T t_i.  The off-diagonal tiles of a row are
// dealt to the wavefronts by their distance from the diagonal (wavefront w
// takes distances w + 1, w + 1 + NW, ...); each leaves its 32 partial
// sums in LDS, and after one barrier every wavefront adds them in the same
// fixed order and applies the inverted diagonal tile itself (the same
// arithmetic everywhere, so the copies of y_i the wavefronts write to LDS
// are equal, and each reads back only its own writes: one barrier per tile
// row).  The off-diagonal tiles of row i + 2 (MT per wavefront) and the
// diagonal tile and x of row i + 1 are loaded while row i is completed.  Lane (r, h) takes entry r of the
// row (backward: column) and half h of the 32 entries it is summed over,
// FP32 tiles converted to FP64 as used.
// FP32 factors: 4 wavefronts of 2 tiles per row, band tiles two rows ahead
// (168 registers, three workgroups per CU); FP64 factors, whose tiles take
// twice the registers: 4 wavefronts of 2 tiles, band tiles one row ahead,
// so that two workgroups fit on a CU.
#define LS32_NW 4
#define LS32_MT 2
#define LS64_NW 4
#define LS64_MT 2
#define LS_NW_MAX 8

template <typename T> struct Frag16 { T v[16]; };
// entries [r][16h .. 16h+15] of a tile
template <typename T>
__device__ __forceinline__ void frag_row(Frag16<T>& f, const T* t, int r, int h) {
  const T* p = t + r * TS + 16 * h;
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float4 a = reinterpret_cast<const float4*>(p)[u];
      f.v[4 * u] = a.x;
      f.v[4 * u + 1] = a.y;
      f.v[4 * u + 2] = a.z;
      f.v[4 * u + 3] = a.w;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double2 a = reinterpret_cast<const double2*>(p)[u];
      f.v[2 * u] = a.x;
      f.v[2 * u + 1] = a.y;
    }
  }
}
// entries [16h .. 16h+15][c] of a tile
template <typename T>
__device__ __forceinline__ void frag_col(Frag16<T>& f, const T* t, int c, int h) {
#pragma unroll
  for (int q = 0; q < 16; ++q) f.v[q] = t[(16 * h + q) * TS + c];
}
// sum_q f_q v_q over 16 consecutive LDS entries, in order
template <typename T>
__device__ __forceinline__ double dot16(const Frag16<T>& f, const double* v) {
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const double2 b = reinterpret_cast<const double2*>(v)[u];
    s += (double)f.v[2 * u] * b.x;
    s += (double)f.v[2 * u + 1] * b.y;
  }
  return s;
}

template <typename T, int NW, int MT, int PD>
__device__ void local_solve_job(const T* __restrict__ Lj, const T* __restrict__ Dj,
                                const int* __restrict__ Ej, const int* __restrict__ Rj, int nt,
                                const double* __restrict__ xj, double* __restrict__ yj,
                                double* ys, double (*part)[NW][TS], double (*sv)[TS],
                                int* sE, int* sR) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 31, h = lane >> 5;
  // the envelope in LDS (dense: E = 0, R = nt - 1)
  for (int e = threadIdx.x; e < nt; e += blockDim.x) {
    sE[e] = Ej ? Ej[e] : 0;
    sR[e] = Rj ? Rj[e] : nt - 1;
  }
  block_sync();
  auto first = [&](int i) { return sE[i]; };
  auto last = [&](int k) { return sR[k]; };
  // row sum of entry r from the partials (fixed order), then this lane's
  // 16 entries of the sums through the wavefront's own LDS row
  auto gather = [&](double(*pp)[TS], double base, double (&o)[16]) {
    double t = pp[0][r];
#pragma unroll
    for (int ww = 1; ww < NW; ++ww) t += pp[ww][r];
    if (lane < TS) sv[w][r] = base - t;
    wave_sync();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double2 b = reinterpret_cast<const double2*>(sv[w] + 16 * h)[u];
      o[2 * u] = b.x;
      o[2 * u + 1] = b.y;
    }
  };
  // The off-diagonal tiles of row i + 1 are loaded into the registers of
  // row i's right after their last use, so they arrive during the barrier,
  // the reduction and the diagonal product.  The diagonal tiles (and x)
  // alternate between two sets, rows unrolled by two: no register holding
  // a load in flight is ever copied (that would wait for the load).  Every
  // prefetch is issued (row and tile indices clamped into the matrix, the
  // products of tiles outside the envelope skipped where they are used), so
  // the number of loads in flight is the same on every path and the waits
  // for the older ones can be partial.
  Frag16<T> a0[MT], a1[MT], d0, d1;
  // PD = 2: two band buffers by row parity; PD = 1: one buffer, the next
  // row's tiles loaded into it (fewer registers)
  Frag16<T>(&b1)[MT] = PD == 2 ? a1 : a0;
  double x0 = 0.0, x1 = 0.0;
  // ---- forward: ys = L^{-1} x
  // The off-diagonal tiles of row i + 2 are loaded into the buffer of row
  // i right after its last use (two buffers, by row parity), the diagonal
  // tile and x of row i + 1 just before them: each load has two rows (one
  // for the diagonal) to arrive, and the waits for the older loads leave
  // the newer ones in flight.
  auto fetch_band_f = [&](Frag16<T> (&ab)[MT], int i) {
    const int e = first(i);
#pragma unroll
    for (int m = 0; m < MT; ++m)
      frag_row(ab[m], Lj + tile_idx(i, max(i - 1 - w - NW * m, e)) * TSQ, r, h);
  };
  auto fetch_diag_f = [&](Frag16<T>& fd, double& fx, int i) {
    frag_row(fd, Dj + (int64_t)i * TSQ, r, h);
    fx = xj[i * TS + r];
  };
  auto fwd_row = [&](int i, Frag16<T> (&ab)[MT], const Frag16<T>& cd, double cx,
                     Frag16<T>& nd, double& nx) {
    const int e = first(i);
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int k = i - 1 - w - NW * m;
      if (k >= e) s += dot16(ab[m], ys + k * TS + 16 * h);
    }
    for (int k = i - 1 - w - NW * MT; k >= e; k -= NW) {
      Frag16<T> t;
      frag_row(t, Lj + tile_idx(i, k) * TSQ, r, h);
      s += dot16(t, ys + k * TS + 16 * h);
    }
    fetch_diag_f(nd, nx, min(i + 1, nt - 1));
    fetch_band_f(ab, min(i + PD, nt - 1));
    s += __shfl_xor(s, 32);
    double(*pp)[TS] = part[i & 1];
    if (lane < TS) pp[w][r] = s;
    block_sync();
    double sc[16];
    gather(pp, cx, sc);
    double y = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) y += (double)cd.v[q] * sc[q];
    y += __shfl_xor(y, 32);
    if (lane < TS) ys[i * TS + r] = y;
    wave_sync();
  };
  fetch_band_f(a0, 0);
  fetch_diag_f(d0, x0, 0);
  if (PD == 2) fetch_band_f(a1, min(1, nt - 1));
  int i = 0;
  for (; i + 1 < nt; i += 2) {
    fwd_row(i, a0, d0, x0, d1, x1);
    fwd_row(i + 1, b1, d1, x1, d0, x0);
  }
  if (i < nt) fwd_row(i, a0, d0, x0, d1, x1);
  // the last forward row's partials are read before the backward rows
  // rewrite either buffer
  block_sync();
  // ---- backward, in place: ys = L^{-T} ys (the same load pipeline)
  auto fetch_band_b = [&](Frag16<T> (&ab)[MT], int i) {
    const int rl = last(i);
#pragma unroll
    for (int m = 0; m < MT; ++m)
      frag_col(ab[m], Lj + tile_idx(min(i + 1 + w + NW * m, rl), i) * TSQ, r, h);
  };
  auto bwd_row = [&](int i, Frag16<T> (&ab)[MT], const Frag16<T>& cd, Frag16<T>& nd) {
    const int rl = last(i);
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int k = i + 1 + w + NW * m;
      if (k <= rl) s += dot16(ab[m], ys + k * TS + 16 * h);
    }
    for (int k = i + 1 + w + NW * MT; k <= rl; k += NW) {
      Frag16<T> t;
      frag_col(t, Lj + tile_idx(k, i) * TSQ, r, h);
      s += dot16(t, ys + k * TS + 16 * h);
    }
    frag_col(nd, Dj + (int64_t)max(i - 1, 0) * TSQ, r, h);
    fetch_band_b(ab, max(i - PD, 0));
    s += __shfl_xor(s, 32);
    // y_i[r], read by every wavefront before the barrier after which z_i
    // overwrites it
    const double yr = ys[i * TS + r];
    double(*pp)[TS] = part[i & 1];
    if (lane < TS) pp[w][r] = s;
    block_sync();
    double tc[16];
    gather(pp, yr, tc);
    double z = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) z += (double)cd.v[q] * tc[q];
    z += __shfl_xor(z, 32);
    if (lane < TS) ys[i * TS + r] = z;
    wave_sync();
  };
  fetch_band_b(a0, nt - 1);
  frag_col(d0, Dj + (int64_t)(nt - 1) * TSQ, r, h);
  if (PD == 2) fetch_band_b(a1, max(nt - 2, 0));
  i = nt - 1;
  for (; i >= 1; i -= 2) {
    bwd_row(i, a0, d0, d1);
    bwd_row(i - 1, b1, d1, d0);
  }
  if (i == 0) bwd_row(0, a0, d0, d1);
  block_sync();
  for (int e = threadIdx.x; e < nt * TS; e += blockDim.x) yj[e] = ys[e];
}

// one launch per factor precision (its registers set the occupancy: three
// workgroups per CU with FP32 factors, two with FP64)
template <typename T, int NW, int MT, int PD>
__device__ __forceinline__ void local_solve_block(const LocalSolveArgs& A, int j) {
  extern __shared__ double lsmem[];
  double(*part)[NW][TS] = reinterpret_cast<double(*)[NW][TS]>(lsmem);
  double(*sv)[TS] = reinterpret_cast<double(*)[TS]>(lsmem + 2 * NW * TS);
  double* ys = lsmem + 3 * NW * TS;
  int* sE = reinterpret_cast<int*>(ys + A.maxnt * TS);
  int* sR = sE + A.maxnt;
  constexpr bool f64 = sizeof(T) == 8;
  const int nt = A.nt[j];
  const int64_t to = f64 ? A.toff64[j] : A.toff32[j], dof = f64 ? A.doff64[j] : A.doff32[j];
  const T* L = f64 ? (const T*)A.L64 : (const T*)A.L32;
  const T* D = f64 ? (const T*)A.D64 : (const T*)A.D32;
  const int* E = f64 ? A.E64 : A.E32;
  const int* R = f64 ? A.R64 : A.R32;
  local_solve_job<T, NW, MT, PD>(L + to * TSQ, D + dof * TSQ, E ? E + dof : nullptr, R ? R + dof : nullptr,
                     nt, A.x + A.voff[j], A.y + A.voff[j], ys, part, sv, sE, sR);
}
__global__ __launch_bounds__(LS32_NW * 64) void k_local_solve_f32(LocalSolveArgs A,
                                                                   const int* __restrict__ done) {
  if (done && *done) return;
  local_solve_block<float, LS32_NW, LS32_MT, 2>(A, A.jobs32[blockIdx.x]);
}
__global__ __launch_bounds__(LS64_NW * 64) void k_local_solve_f64(LocalSolveArgs A,
                                                                const int* __restrict__ done) {
  if (done && *done) return;
  local_solve_block<double, LS64_NW, LS64_MT, 1>(A, A.jobs64[blockIdx.x]);
}

static size_t local_solve_lds(int maxnt) {
  return (size_t)(3 * LS_NW_MAX + maxnt) * TS * sizeof(double) + 2 * (size_t)maxnt * sizeof(int);
}

hipError_t local_solve_check(int maxnt) {
  const size_t lds = local_solve_lds(maxnt);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds <= 64 * 1024) return hipSuccess;
  // above the default limit of dynamic LDS (set once, thread-safe)
  static const hipError_t e = [] {
    hipError_t r = hipFuncSetAttribute((const void*)k_local_solve_f32,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (r == hipSuccess)
      r = hipFuncSetAttribute((const void*)k_local_solve_f64,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    return r;
  }();
  return e;
}

hipError_t local_solve(const LocalSolveArgs& a, const int* done, hipStream_t st) {
  const size_t lds = local_solve_lds(a.maxnt);
  if (a.njobs32 > 0)
    hipLaunchKernelGGL(k_local_solve_f32, dim3(a.njobs32), dim3(LS32_NW * 64), lds, st, a, done);
  if (a.njobs64 > 0)
    hipLaunchKernelGGL(k_local_solve_f64, dim3(a.njobs64), dim3(LS64_NW * 64), lds, st, a, done);
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
                                                   const int* __restrict__ active,
                                                   const int* __restrict__ envE,
                                                   const int* __restrict__ envR) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  const int* Ej = envE ? envE + doff[j] : nullptr;
  const int* Rl = envR ? envR + doff[j] : nullptr;
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
    // slice sl takes k = sl, sl + ns, ...; tiles left of E(i) are zero
    const int e = Ej ? Ej[i] : 0;
    if (worker)
      for (int k = e > sl ? sl + (e - sl + ns - 1) / ns * ns : sl; k < i; k += ns)
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
                                                   const int* __restrict__ active,
                                                   const int* __restrict__ envE,
                                                   const int* __restrict__ envR) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  const int* Ej = envE ? envE + doff[j] : nullptr;
  const int* Rl = envR ? envR + doff[j] : nullptr;
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
    // (tiles below R(k) are zero)
    const int iend = Rl ? min(nt, Rl[k] + 1) : nt;
    if (worker)
      for (int i = k + 1 + sl; i < iend; i += ns)
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

// ----------------------------------------- windowed multi-RHS substitution ---
// Forward G X = R and backward G^T X = R for the eigen sweeps, one
// workgroup of NW (8 or 4) wavefronts per subdomain.  The tile rows are
// taken in windows of 2 NW; the 32 x b blocks of the current window stay in
// registers as matrix-core accumulators (wavefront w owns window rows
// w and w + NW).  Each window first takes its update from all finished rows
// (left-looking; factor tiles streamed with the next one in flight, no
// barriers), then is solved right-looking: the owner of row i forms
// X_i = Dinv_i acc_i (or Dinv_i^T acc_i) and publishes it, transposed, in
// LDS; after one barrier every wavefront subtracts G_ki X_i (G_ik^T X_i)
// from its later rows.  b = 16 * NCQ right-hand sides, b <= 32 (wider
// blocks take the row-by-row kernels above: their accumulators would not
// fit in registers).
#define TRW_MR 2

struct F8 { double v[8]; };

// A-operand fragment of rows r0..r0+15 of a tile: lane (fi, fg) takes
// row r0 + fi, columns 8 fg .. 8 fg + 7 (plain), or the transposed tile
// (column r0 + fi, rows 8 fg ..) (tr).
__device__ __forceinline__ void afrag(F8& f, const double* t, int r0, int fi, int fg) {
  const double2* p = reinterpret_cast<const double2*>(t + (r0 + fi) * TS + 8 * fg);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double2 a = p[u];
    f.v[2 * u] = a.x;
    f.v[2 * u + 1] = a.y;
  }
}
__device__ __forceinline__ void afrag_tr(F8& f, const double* t, int r0, int fi, int fg) {
#pragma unroll
  for (int s = 0; s < 8; ++s) f.v[s] = t[(8 * fg + s) * TS + r0 + fi];
}
// B-operand fragment of a 32 x b block stored row-major with stride b in
// memory: lane (fi, fg) takes column c0 + fi, rows 8 fg .. 8 fg + 7.
__device__ __forceinline__ void bfrag_g(F8& f, const double* x, int b, int c0, int fi, int fg) {
#pragma unroll
  for (int s = 0; s < 8; ++s) f.v[s] = x[(8 * fg + s) * b + c0 + fi];
}
// ... and from the transposed LDS copy sT[col][row] (row stride TRW_LD).
#define TRW_LD (TS + 2)
__device__ __forceinline__ void bfrag_s(F8& f, const double* sT, int c0, int fi, int fg) {
  const double2* p = reinterpret_cast<const double2*>(sT + (c0 + fi) * TRW_LD + 8 * fg);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double2 a = p[u];
    f.v[2 * u] = a.x;
    f.v[2 * u + 1] = a.y;
  }
}

// acc[.][cq] += A B_cq for one column quadrant cq.
template <int NCQ>
__device__ __forceinline__ void trw_mma(d4_t (&acc)[2][NCQ], const F8 (&a)[2], const F8& bf, int cq) {
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int rq = 0; rq < 2; ++rq)
      acc[rq][cq] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rq].v[s], bf.v[s], acc[rq][cq], 0, 0, 0);
}

// Owner step: X_i = D acc_i, D = Dinv_i (BWD: Dinv_i^T); acc_i goes through
// LDS (transposed) to become the B operand; X_i is written to global memory
// and, transposed, to sXo.
// NEG: the accumulator holds the negated right-hand side (-acc_i is used).
template <int NCQ, bool BWD, bool NEG = false>
__device__ __forceinline__ void trw_finish(const d4_t (&acc)[2][NCQ], const double* Dt, double* sTmp,
                                           double* sXo, double* Xi, int b, int lane) {
  const int fi = lane & 15, fg = lane >> 4;
#pragma unroll
  for (int rq = 0; rq < 2; ++rq)
#pragma unroll
    for (int cq = 0; cq < NCQ; ++cq)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        sTmp[(cq * 16 + acc_col(lane)) * TRW_LD + rq * 16 + acc_row<double>(lane, v)] =
            NEG ? -acc[rq][cq][v] : acc[rq][cq][v];
  wave_sync();
  F8 a[2];
#pragma unroll
  for (int rq = 0; rq < 2; ++rq) {
    if (BWD) afrag_tr(a[rq], Dt, rq * 16, fi, fg);
    else afrag(a[rq], Dt, rq * 16, fi, fg);
  }
  d4_t o[2][NCQ];
#pragma unroll
  for (int rq = 0; rq < 2; ++rq)
#pragma unroll
    for (int cq = 0; cq < NCQ; ++cq) o[rq][cq] = acc_zero<double>();
#pragma unroll
  for (int cq = 0; cq < NCQ; ++cq) {
    F8 bf;
    bfrag_s(bf, sTmp, cq * 16, fi, fg);
    trw_mma<NCQ>(o, a, bf, cq);
  }
#pragma unroll
  for (int rq = 0; rq < 2; ++rq)
#pragma unroll
    for (int cq = 0; cq < NCQ; ++cq)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rq * 16 + acc_row<double>(lane, v), c = cq * 16 + acc_col(lane);
        sXo[c * TRW_LD + r] = o[rq][cq][v];
        Xi[r * b + c] = o[rq][cq][v];
      }
}

// Workgroup -> (subdomain slot, column block).  With SPLIT column blocks
// per subdomain (LDB = SPLIT * b columns in the blocks R and X), the
// workgroups of one subdomain get ids 8 apart: the dispatcher deals ids
// round-robin to the 8 XCDs, so they run on one XCD and share its L2 for
// the factor tiles.  The columns of a triangular solve are independent, and
// each column block is computed with the same products in the same order
// as in the unsplit kernel: the result is bitwise the same.
template <int SPLIT>
__device__ __forceinline__ int trsm_slot(int bid, int& part) {
  if (SPLIT == 1) {
    part = 0;
    return bid;
  }
  part = (bid >> 3) % SPLIT;
  return (bid & 7) + 8 * (bid / (8 * SPLIT));
}

template <int NCQ, bool BWD, int LDB, int NW>
__global__ __launch_bounds__(NW * 64, 2) void k_trsm_win(const double* __restrict__ G,
                                                         const double* __restrict__ dinv,
                                                         const int64_t* __restrict__ toff,
                                                         const int64_t* __restrict__ doff,
                                                         const int* __restrict__ ntl,
                                                         const int* __restrict__ voff,
                                                         const double* __restrict__ R,
                                                         double* __restrict__ X,
                                                         const int* __restrict__ active,
                                                         const int* __restrict__ order,
                                                         int nsub, const int* __restrict__ envE,
                                                         const int* __restrict__ envR) {
  constexpr int b = 16 * NCQ;  // columns solved by this workgroup
  static_assert(LDB % b == 0, "column blocks");
  int part;
  const int slot = trsm_slot<LDB / b>(blockIdx.x, part);
  if (slot >= nsub) return;
  const int j = order ? order[slot] : slot;
  if (active && !active[j]) return;
  __shared__ __align__(16) double sTmp[b * TRW_LD];
  __shared__ __align__(16) double sX[2][b * TRW_LD];
  const int nt = ntl[j];
  const double* Gj = G + toff[j] * TSQ;
  const double* Dj = dinv + doff[j] * TSQ;
  const double* Rj = R + (int64_t)voff[j] * LDB + part * b;
  double* Xj = X + (int64_t)voff[j] * LDB + part * b;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int fi = lane & 15, fg = lane >> 4;
  const int nwin = (nt + NW * TRW_MR - 1) / (NW * TRW_MR);
  // envelope: row k has nonzero tiles from column E(k), column k down to
  // row R(k) (all others are zero: their products are skipped)
  const int* Ej = envE ? envE + doff[j] : nullptr;
  const int* Rl = envR ? envR + doff[j] : nullptr;
  auto first = [&](int k) { return Ej ? Ej[k] : 0; };
  auto last = [&](int k) { return Rl ? Rl[k] : nt - 1; };
  for (int wi = 0; wi < nwin; ++wi) {
    // window rows [p0, p1); BWD windows run from the bottom
    const int p0 = BWD ? max(0, nt - (wi + 1) * NW * TRW_MR) : wi * NW * TRW_MR;
    const int p1 = BWD ? nt - wi * NW * TRW_MR : min(nt, p0 + NW * TRW_MR);
    // acc holds -R_k + the products so far (negation is exact, so this is
    // bitwise the negated R_k - products); the owner negates at the end
    d4_t acc[TRW_MR][2][NCQ];
    int krow[TRW_MR];
#pragma unroll
    for (int m = 0; m < TRW_MR; ++m) {
      krow[m] = p0 + w + NW * m;
      const bool own = krow[m] < p1;
      const int kr = min(krow[m], nt - 1);   // every load issued, in range
#pragma unroll
      for (int rq = 0; rq < 2; ++rq)
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double r = Rj[((int64_t)kr * TS + rq * 16 + acc_row<double>(lane, v)) * LDB +
                                cq * 16 + acc_col(lane)];
            acc[m][rq][cq][v] = own ? -r : 0.0;
          }
    }
    auto load_a = [&](const double* t, F8 (&aa)[2]) {
#pragma unroll
      for (int rq = 0; rq < 2; ++rq) {
        if (BWD) afrag_tr(aa[rq], t, rq * 16, fi, fg);
        else afrag(aa[rq], t, rq * 16, fi, fg);
      }
    };
    // ---- left-looking update from the finished rows
    // FWD: acc_k += sum_{jj < p0} G_k,jj X_jj      BWD: acc_k += sum_{jj >= p1} G_jj,k^T X_jj
    // Each step first issues the loads of X_jj, then those of the next
    // factor tile, then the products: the wait for X_jj and the current
    // tile leaves the next tile in flight.  Two tile buffers alternate
    // (no register copy of a load in flight, which would wait for it).
#pragma unroll
    for (int m = 0; m < TRW_MR; ++m) {
      const int k = krow[m];
      if (k >= p1) continue;
      const int jlo = BWD ? p1 : first(k), jhi = BWD ? min(nt, last(k) + 1) : p0;
      if (jlo >= jhi) continue;
      auto tile = [&](int jj) {
        return BWD ? Gj + tile_idx(jj, k) * TSQ : Gj + tile_idx(k, jj) * TSQ;
      };
      auto step = [&](const F8 (&cur)[2], F8 (&nxt)[2], int jj) {
        F8 bf[NCQ];
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq)
          bfrag_g(bf[cq], Xj + (int64_t)jj * TS * LDB, LDB, cq * 16, fi, fg);
        load_a(tile(min(jj + 1, jhi - 1)), nxt);
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq) trw_mma<NCQ>(acc[m], cur, bf[cq], cq);
        __builtin_amdgcn_sched_barrier(0);
      };
      F8 a0[2], a1[2];
      load_a(tile(jlo), a0);
      int jj = jlo;
      for (; jj + 1 < jhi; jj += 2) {
        step(a0, a1, jj);
        step(a1, a0, jj + 1);
      }
      if (jj < jhi) step(a0, a1, jj);
    }
    // ---- right-looking solve inside the window
    for (int st = 0; st < p1 - p0; ++st) {
      const int i = BWD ? p1 - 1 - st : p0 + st;
      const int li = i - p0, ow = li % NW, om = li / NW;
      double* sXo = sX[st & 1];
      if (w == ow) {
#pragma unroll
        for (int m = 0; m < TRW_MR; ++m)
          if (m == om)
            trw_finish<NCQ, BWD, true>(acc[m], Dj + (int64_t)i * TSQ, sTmp, sXo,
                                       Xj + (int64_t)i * TS * LDB, LDB, lane);
      }
      // the factor tile of the first row's update does not depend on X_i:
      // its loads are in flight while the wavefront waits at the barrier
      // (the second row's load then overlaps the first row's products;
      // loading both before the barrier would hold 64 more registers
      // through the owner's product)
      auto tile_i = [&](int k) {
        return BWD ? Gj + tile_idx(i, k) * TSQ : Gj + tile_idx(k, i) * TSQ;
      };
      auto wants = [&](int k) {
        return k < p1 && (BWD ? k < i && i <= last(k) : k > i && first(k) <= i);
      };
      F8 a0[2];
      if (wants(krow[0])) load_a(tile_i(krow[0]), a0);
      block_sync();
#pragma unroll
      for (int m = 0; m < TRW_MR; ++m) {
        const int k = krow[m];
        if (!wants(k)) continue;
        F8 a[2];
        if (m == 0) {
          a[0] = a0[0];
          a[1] = a0[1];
        } else {
          load_a(tile_i(k), a);
        }
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq) {
          F8 bf;
          bfrag_s(bf, sXo, cq * 16, fi, fg);
          trw_mma<NCQ>(acc[m], a, bf, cq);
        }
      }
    }
    block_sync();
  }
}

// Windowed substitution with deeper load pipelines.  One workgroup of
// NW (8 or 4) wavefronts per subdomain; windows of NW tile rows, wavefront w
// owning window row p0 + w (its 32 x b block as matrix-core accumulators,
// holding -R + the products so far).  The left-looking update streams the
// row's factor tiles with AD tiles in flight beyond the one in use and,
// with BP, loads the right-hand block X_jj of the next step one step ahead,
// so that neither the HBM latency of the factor nor the L2 latency of X
// stalls the matrix cores (an FP64 tile product with b = 32 right-hand
// sides is 32 MFMAs, about one HBM round trip).  AD and BP are chosen per
// block width so that the pipelines fit in 256 VGPRs without spills.  The
// substitution inside the window is the right-looking one of k_trsm_win.

template <int NCQ, bool BWD, int AD, bool BP, int LDB, int NW>
__global__ __launch_bounds__(NW * 64, 2) void k_trsm_w1(const double* __restrict__ G,
                                                        const double* __restrict__ dinv,
                                                        const int64_t* __restrict__ toff,
                                                        const int64_t* __restrict__ doff,
                                                        const int* __restrict__ ntl,
                                                        const int* __restrict__ voff,
                                                        const double* __restrict__ R,
                                                        double* __restrict__ X,
                                                        const int* __restrict__ active,
                                                        const int* __restrict__ order,
                                                        int nsub, const int* __restrict__ envE,
                                                        const int* __restrict__ envR) {
  static_assert(AD == 1 || AD == 2, "factor tiles in flight");
  constexpr int b = 16 * NCQ;  // columns solved by this workgroup
  static_assert(LDB % b == 0, "column blocks");
  int part;
  const int slot = trsm_slot<LDB / b>(blockIdx.x, part);
  if (slot >= nsub) return;
  const int j = order ? order[slot] : slot;
  if (active && !active[j]) return;
  __shared__ __align__(16) double sTmp[b * TRW_LD];
  __shared__ __align__(16) double sX[2][b * TRW_LD];
  const int nt = ntl[j];
  const double* Gj = G + toff[j] * TSQ;
  const double* Dj = dinv + doff[j] * TSQ;
  const double* Rj = R + (int64_t)voff[j] * LDB + part * b;
  double* Xj = X + (int64_t)voff[j] * LDB + part * b;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int fi = lane & 15, fg = lane >> 4;
  const int nwin = (nt + NW - 1) / NW;
  // envelope (as in k_trsm_win)
  const int* Ej = envE ? envE + doff[j] : nullptr;
  const int* Rl = envR ? envR + doff[j] : nullptr;
  auto first = [&](int k) { return Ej ? Ej[k] : 0; };
  auto last = [&](int k) { return Rl ? Rl[k] : nt - 1; };
  // factor tile (k, jj) (FWD) or (jj, k) read transposed (BWD)
  auto loadA = [&](F8 (&aa)[2], int k, int jj) {
    const double* t = BWD ? Gj + tile_idx(jj, k) * TSQ : Gj + tile_idx(k, jj) * TSQ;
#pragma unroll
    for (int rq = 0; rq < 2; ++rq) {
      if (BWD) afrag_tr(aa[rq], t, rq * 16, fi, fg);
      else afrag(aa[rq], t, rq * 16, fi, fg);
    }
  };
  auto loadB = [&](F8& bb, int jj, int cq) { bfrag_g(bb, Xj + (int64_t)jj * TS * LDB, LDB, cq * 16, fi, fg); };
  for (int wi = 0; wi < nwin; ++wi) {
    // window rows [p0, p1); BWD windows run from the bottom
    const int p0 = BWD ? max(0, nt - (wi + 1) * NW) : wi * NW;
    const int p1 = BWD ? nt - wi * NW : min(nt, p0 + NW);
    const int k = p0 + w;
    const bool own = k < p1;
    d4_t acc[2][NCQ];
#pragma unroll
    for (int rq = 0; rq < 2; ++rq)
#pragma unroll
      for (int cq = 0; cq < NCQ; ++cq)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[rq][cq][v] = own ? -Rj[((int64_t)k * TS + rq * 16 + acc_row<double>(lane, v)) * LDB +
                                     cq * 16 + acc_col(lane)]
                               : 0.0;
    // ---- left-looking update from the finished rows
    // FWD: acc_k += sum_{jj < p0} G_k,jj X_jj      BWD: acc_k += sum_{jj >= p1} G_jj,k^T X_jj
    const int jlo = BWD ? p1 : (own ? first(k) : 0);
    const int jhi = BWD ? (own ? min(nt, last(k) + 1) : nt) : p0;
    if (own && jlo < jhi && BP) {
      // whole next right-hand block in flight during this step's products
      F8 a0[2], a1[2], a2[2];
      F8 bc[NCQ], bn[NCQ];
      loadA(a0, k, jlo);
      if (jlo + 1 < jhi) loadA(a1, k, jlo + 1);
#pragma unroll
      for (int cq = 0; cq < NCQ; ++cq) loadB(bc[cq], jlo, cq);
      for (int jj = jlo; jj < jhi; ++jj) {
        // the loads of the steps ahead go out before this step's products
        if (AD == 2 && jj + 2 < jhi) loadA(a2, k, jj + 2);
        if (jj + 1 < jhi) {
#pragma unroll
          for (int cq = 0; cq < NCQ; ++cq) loadB(bn[cq], jj + 1, cq);
        }
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq) trw_mma<NCQ>(acc, a0, bc[cq], cq);
#pragma unroll
        for (int rq = 0; rq < 2; ++rq) {
          a0[rq] = a1[rq];
          if (AD == 2) a1[rq] = a2[rq];
        }
        if (AD == 1 && jj + 2 < jhi) loadA(a1, k, jj + 2);
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq) bc[cq] = bn[cq];
      }
    } else if (own && jlo < jhi) {
      // one column group of the right-hand block in flight: group q + 1 is
      // loaded during the products with group q, group 0 of the next step
      // during the last group of this one
      F8 a0[2], a1[2];
      F8 bcur, bnxt;
      loadA(a0, k, jlo);
      if (jlo + 1 < jhi) loadA(a1, k, jlo + 1);
      loadB(bcur, jlo, 0);
      for (int jj = jlo; jj < jhi; ++jj) {
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq) {
          if (cq + 1 < NCQ) loadB(bnxt, jj, cq + 1);
          else if (jj + 1 < jhi) loadB(bnxt, jj + 1, 0);
          trw_mma<NCQ>(acc, a0, bcur, cq);
          bcur = bnxt;
        }
#pragma unroll
        for (int rq = 0; rq < 2; ++rq) a0[rq] = a1[rq];
        if (jj + 2 < jhi) loadA(a1, k, jj + 2);
      }
    }
    // ---- right-looking solve inside the window
    for (int st = 0; st < p1 - p0; ++st) {
      const int i = BWD ? p1 - 1 - st : p0 + st;
      double* sXo = sX[st & 1];
      if (w == i - p0)
        trw_finish<NCQ, BWD, true>(acc, Dj + (int64_t)i * TSQ, sTmp, sXo,
                                   Xj + (int64_t)i * TS * LDB, LDB, lane);
      const bool want = own && (BWD ? k < i && i <= last(k) : k > i && first(k) <= i);
      F8 a[2];
      if (want) loadA(a, k, i);
      block_sync();
      if (want) {
#pragma unroll
        for (int cq = 0; cq < NCQ; ++cq) {
          F8 bf;
          bfrag_s(bf, sXo, cq * 16, fi, fg);
          trw_mma<NCQ>(acc, a, bf, cq);
        }
      }
    }
    block_sync();
  }
}

// Grid of a solve: one workgroup per subdomain, or SPLIT per subdomain
// (slots rounded up to a multiple of 8, see trsm_slot).
static dim3 trsm_grid(int nsub, int split) {
  return split == 1 ? dim3(nsub) : dim3(split * ((nsub + 7) / 8 * 8));
}

#define TRSM_ARGS G, dinv, toff, doff, nt, voff, R, X, active, order, nsub, envE, envR

template <bool BWD, int NW>
static hipError_t launch_trsm_w1(const double* G, const double* dinv, const int64_t* toff,
                                 const int64_t* doff, const int* nt, const int* voff, int nsub,
                                 int b, int split, const double* R, double* X, const int* active,
                                 const int* order, const int* envE, const int* envR,
                                 hipStream_t st) {
  const dim3 grid = trsm_grid(nsub, split), blk(NW * 64);
  switch (split == 1 ? b : -b) {
    case 16: hipLaunchKernelGGL((k_trsm_w1<1, BWD, 2, true, 16, NW>), grid, blk, 0, st, TRSM_ARGS); break;
    case 32: hipLaunchKernelGGL((k_trsm_w1<2, BWD, 1, true, 32, NW>), grid, blk, 0, st, TRSM_ARGS); break;
    case 48: hipLaunchKernelGGL((k_trsm_w1<3, BWD, 1, false, 48, NW>), grid, blk, 0, st, TRSM_ARGS); break;
    case -32: hipLaunchKernelGGL((k_trsm_w1<1, BWD, 2, true, 32, NW>), grid, blk, 0, st, TRSM_ARGS); break;
    case -48: hipLaunchKernelGGL((k_trsm_w1<1, BWD, 2, true, 48, NW>), grid, blk, 0, st, TRSM_ARGS); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool BWD, int NW>
static hipError_t launch_trsm_win(const double* G, const double* dinv, const int64_t* toff,
                                  const int64_t* doff, const int* nt, const int* voff, int nsub,
                                  int b, int split, const double* R, double* X, const int* active,
                                  const int* order, const int* envE, const int* envR,
                                  hipStream_t st) {
  const dim3 grid = trsm_grid(nsub, split), blk(NW * 64);
  switch (split == 1 ? b : -b) {
    case 16: hipLaunchKernelGGL((k_trsm_win<1, BWD, 16, NW>), grid, blk, 0, st, TRSM_ARGS); break;
    case 32: hipLaunchKernelGGL((k_trsm_win<2, BWD, 32, NW>), grid, blk, 0, st, TRSM_ARGS); break;
    case -32: hipLaunchKernelGGL((k_trsm_win<1, BWD, 32, NW>), grid, blk, 0, st, TRSM_ARGS); break;
    case -48: hipLaunchKernelGGL((k_trsm_win<1, BWD, 48, NW>), grid, blk, 0, st, TRSM_ARGS); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#undef TRSM_ARGS

int trsm_max_split(int b) { return b <= 48 ? b / 16 : 1; }

int trsm_variants() { return 4; }

// b <= 48: variant 0 two rows per wavefront, 8 wavefronts (windows of 16
// rows; b <= 32 unsplit), variant 1 one row per wavefront with deeper load
// pipelines, 8 wavefronts (windows of 8), variants 2 and 3 the same with 4
// wavefronts (half the window; two workgroups fit a CU, so two subdomains'
// substitution chains interleave).  split = b / 16: the same kernels on
// 16-column blocks, b / 16 workgroups per subdomain.  Every choice forms
// each row's sum over the columns in ascending order, whatever the window:
// bitwise the same X.  b = 64: row by row.
template <bool BWD>
static hipError_t launch_trsm(const double* G, const double* dinv, const int64_t* toff,
                              const int64_t* doff, const int* nt, const int* voff, int nsub,
                              int b, const double* R, double* X, const int* active,
                              const int* order, const int* envE, const int* envR, int variant,
                              int split, hipStream_t st) {
  if (split != 1 && (b > 48 || split != b / 16)) return hipErrorInvalidValue;
  if (!envE != !envR || variant < 0 || variant > 3) return hipErrorInvalidValue;
  // b = 48 unsplit has no two-rows kernel (its accumulators would spill)
  if (b == 48 && split == 1 && (variant & 1) == 0) variant += 1;
  if (b <= 48) {
    switch (variant) {
      case 0: return launch_trsm_win<BWD, 8>(G, dinv, toff, doff, nt, voff, nsub, b, split, R, X,
                                             active, order, envE, envR, st);
      case 1: return launch_trsm_w1<BWD, 8>(G, dinv, toff, doff, nt, voff, nsub, b, split, R, X,
                                            active, order, envE, envR, st);
      case 2: return launch_trsm_win<BWD, 4>(G, dinv, toff, doff, nt, voff, nsub, b, split, R, X,
                                             active, order, envE, envR, st);
      default: return launch_trsm_w1<BWD, 4>(G, dinv, toff, doff, nt, voff, nsub, b, split, R, X,
                                             active, order, envE, envR, st);
    }
  }
  if (BWD)
    hipLaunchKernelGGL(k_trsm_bwd, dim3(nsub), dim3(1024), 0, st, G, dinv, toff, doff, nt, voff,
                       b, R, X, active, envE, envR);
  else
    hipLaunchKernelGGL(k_trsm_fwd, dim3(nsub), dim3(1024), 0, st, G, dinv, toff, doff, nt, voff,
                       b, R, X, active, envE, envR);
  return hipGetLastError();
}

hipError_t launch_trsm_fwd(const double* G, const double* dinv, const int64_t* toff,
                           const int64_t* doff, const int* nt, const int* voff, int nsub, int b,
                           const double* R, double* X, const int* active, const int* order,
                           const int* envE, const int* envR, int variant, int split,
                           hipStream_t st) {
  return launch_trsm<false>(G, dinv, toff, doff, nt, voff, nsub, b, R, X, active, order, envE,
                            envR, variant, split, st);
}

hipError_t launch_trsm_bwd(const double* G, const double* dinv, const int64_t* toff,
                           const int64_t* doff, const int* nt, const int* voff, int nsub, int b,
                           const double* R, double* X, const int* active, const int* order,
                           const int* envE, const int* envR, int variant, int split,
                           hipStream_t st) {
  return launch_trsm<true>(G, dinv, toff, doff, nt, voff, nsub, b, R, X, active, order, envE,
                           envR, variant, split, st);
}

// B_j = X_j A^o_j X_j (the B-matrix of the GenEO eigenproblem) in compact
// CSR over the local rows: only the entries that are nonzero in B_j (the
// overlap matrix shares the Neumann matrix's pattern and is zero away from
// the overlap zone), scaled by mu_a mu_q.  Built once per setup: a count
// pass, an exclusive scan, a fill pass (thread per local row, 2D grid over
// (row chunk, subdomain)).
template <bool FILL>
__global__ __launch_bounds__(256) void k_bcompact(const int* __restrict__ sub_ptr,
                                                  const double* __restrict__ pou,
                                                  const int* __restrict__ rp,
                                                  const int* __restrict__ colx,
                                                  const double* __restrict__ val,
                                                  int* __restrict__ cnt,
                                                  const int* __restrict__ brp,
                                                  int* __restrict__ bcol,
                                                  double* __restrict__ bval) {
  const int j = blockIdx.y;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const double mua = pou[s0 + a];
  int k = 0;
  const int o = FILL ? brp[s0 + a] : 0;
  if (mua != 0.0) {
    // entries in batches of 8: the index and value loads, then the
    // partition-of-unity gathers, all in flight before the first entry is
    // kept or dropped (in entry order)
    const int p1 = rp[s0 + a + 1];
    for (int p0 = rp[s0 + a]; p0 < p1; p0 += 8) {
      int qq[8];
      double vv[8], mq[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int p = min(p0 + u, p1 - 1);  // in range; extra entries unused
        qq[u] = colx[p];
        vv[u] = val[p];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) mq[u] = pou[s0 + qq[u]];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        // every value is used (no early exit), so the loads stay batched
        const double w = mua * vv[u] * mq[u];
        const bool keep = p0 + u < p1 && w != 0.0;
        if (FILL && keep) {
          bcol[o + k] = qq[u];
          bval[o + k] = w;
        }
        k += keep ? 1 : 0;
      }
    }
  }
  if (!FILL) cnt[s0 + a] = k;
}

// Rows of the compact B with at least one entry, as (subdomain, local row):
// flag pass (into cnt, after its counts are scanned), exclusive scan into
// rpos (rpos[nloc] = the number of such rows), fill pass.
__global__ __launch_bounds__(256) void k_brows(const int* __restrict__ sub_ptr, int* __restrict__ cnt,
                                               const int* __restrict__ rpos,
                                               int2* __restrict__ rows, int fill) {
  const int j = blockIdx.y;
  const int s0 = sub_ptr[j], n = sub_ptr[j + 1] - s0;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  if (!fill) cnt[s0 + a] = cnt[s0 + a] > 0 ? 1 : 0;
  else if (cnt[s0 + a]) rows[rpos[s0 + a]] = make_int2(j, a);
}

hipError_t launch_bcompact(const int* sub_ptr, const double* pou, const geneo_csr_batch_t* Ao,
                           int nsub, int64_t nloc, int maxrows, int* cnt, int* brp, int* bcol,
                           double* bval, int* rpos, int2* rows, hipStream_t st) {
  const dim3 grid((maxrows + 255) / 256, nsub);
  hipLaunchKernelGGL(k_bcompact<false>, grid, dim3(256), 0, st, sub_ptr, pou, Ao->rowptr, Ao->col,
                     Ao->val, cnt, nullptr, nullptr, nullptr);
  hipError_t e = scan_exclusive_i32(cnt, brp, nloc, nullptr, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bcompact<true>, grid, dim3(256), 0, st, sub_ptr, pou, Ao->rowptr, Ao->col,
                     Ao->val, nullptr, brp, bcol, bval);
  hipLaunchKernelGGL(k_brows, grid, dim3(256), 0, st, sub_ptr, cnt, nullptr, nullptr, 0);
  e = scan_exclusive_i32(cnt, rpos, nloc, nullptr, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_brows, grid, dim3(256), 0, st, sub_ptr, cnt, rpos, rows, 1);
  return hipGetLastError();
}

// Y = B_j X on the rows of B_j that hold entries (the listed rows); the
// other rows of Y are zero and stay so (the caller clears Y once), so a
// product writes only the overlap zone.  One thread per (listed row,
// column).
__global__ __launch_bounds__(256) void k_bapply(const int* __restrict__ sub_ptr,
                                               const int* __restrict__ brp,
                                               const int* __restrict__ bcol,
                                               const double* __restrict__ bval,
                                               const int2* __restrict__ rows, int nrows,
                                               const int* __restrict__ voff, int b,
                                               const double* __restrict__ X,
                                               double* __restrict__ Y,
                                               const int* __restrict__ active) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int r = (int)(t / b), c = (int)(t % b);
  if (r >= nrows) return;
  const int2 ja = rows[r];
  const int j = ja.x, a = ja.y;
  if (active && !active[j]) return;
  const int g = sub_ptr[j] + a;
  const double* Xj = X + (int64_t)voff[j] * b;
  double s = 0.0;
  // entries in batches of 8: all index and value loads, then all the
  // gathers of X, are in flight together; the sum keeps the entry order
  const int p0 = brp[g], p1 = brp[g + 1];
  for (int p = p0; p < p1; p += 8) {
    int cc[8];
    double vv[8], xx[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      cc[u] = p + u < p1 ? bcol[p + u] : 0;
      vv[u] = p + u < p1 ? bval[p + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) xx[u] = p + u < p1 ? Xj[(int64_t)cc[u] * b + c] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (p + u < p1) s += vv[u] * xx[u];
  }
  Y[((int64_t)voff[j] + a) * b + c] = s;
}

hipError_t launch_bapply(const int* sub_ptr, const int* brp, const int* bcol, const double* bval,
                         const int2* rows, int nrows, const int* voff, int b, const double* X,
                         double* Y, const int* active, hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  const int64_t nel = (int64_t)nrows * b;
  hipLaunchKernelGGL(k_bapply, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, st, sub_ptr,
                     brp, bcol, bval, rows, nrows, voff, b, X, Y, active);
  return hipGetLastError();
}

}  // namespace geneo
