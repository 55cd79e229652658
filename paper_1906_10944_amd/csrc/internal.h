// Internal declarations of libgeneo (host launchers of the device kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "common.h"
#include "geneo.h"

namespace geneo {

// Per-subdomain layout of the dense local factors and padded vectors.
struct LocalLayout {
  int n = 0;                          // subdomains
  std::vector<int> nrow;              // matrix order per subdomain
  std::vector<int> nt;                // tile rows = ceil(nrow / TS) (at least 1)
  std::vector<int64_t> toff;          // tile offset (units of TSQ elements)
  std::vector<int64_t> doff;          // diagonal-tile offset = sum of nt
  std::vector<int> voff;              // padded-vector offset = sum of nt*TS
  int64_t ntiles = 0, ndiag = 0;
  int64_t nvec = 0;
  int maxnt = 0;
  void build(const std::vector<int>& rows);
};

// ---------------------------------------------------------------- util.hip
hipError_t scan_exclusive_i32(const int* in, int* out, int64_t n, int* total_dev,
                              hipStream_t st);  // out[n] also written
hipError_t launch_dmap(const int* sub_ptr, const uint8_t* flags, int nsub, int* dmap,
                       int* nd, hipStream_t st);
hipError_t launch_dvec(const int* sub_ptr, const int* sub_idx, const int* dmap,
                       const int* voff, const int* nt, int nsub, const geneo_csr_t* A,
                       int* dglob, int* didx, double* dscale, hipStream_t st);
hipError_t launch_owners(const int* sub_ptr, const int* sub_idx, int nsub, int64_t nloc,
                         int ndof, int* optr, int* ocount, int2* olist, hipStream_t st);
hipError_t launch_adjacency(const int* optr, const int2* olist, int ndof, int nsub,
                            uint8_t* adj, hipStream_t st);
hipError_t launch_pairs(const uint8_t* adj, int nsub, int* cnt, int* off, int2* pairs,
                        int* npairs_dev, hipStream_t st, bool count_only);

// ------------------------------------------------------------- dense.hip
// Tile envelopes (per matrix, one int per tile row at the matrix's diagonal
// tile offset doff): E(i) = first tile column of tile row i that may hold a
// nonzero (nondecreasing), R(k) = last tile row with E(i) <= k.  The fills
// lower E from env_init's E(i) = i (when env is not NULL); env_finish makes
// E nondecreasing and forms R.  Both over the matrices jobs[0 .. njobs)
// (jobs NULL: 0 .. njobs-1).
hipError_t launch_env_init(int* env, const int64_t* doff, const int* nt, const int* jobs,
                           int njobs, hipStream_t st);
hipError_t launch_env_finish(int* envE, int* envR, const int64_t* doff, const int* nt,
                             const int* jobs, int njobs, hipStream_t st);
hipError_t launch_densify_dirichlet(bool fp32, void* tiles, const int64_t* toff,
                                    const int* nt, const int* voff, const int* jobs,
                                    int njobs, const int* sub_ptr, const int* sub_idx,
                                    const int* dmap, const int* dglob, const double* dscale,
                                    const geneo_csr_t* A, int ntmax /* max tile count */,
                                    int* env, const int64_t* doff, hipStream_t st);
hipError_t launch_densify_shifted(double* tiles, const int64_t* toff, const int* nt,
                                  int nsub, const int* sub_ptr, const double* pou,
                                  const geneo_csr_batch_t* An, const geneo_csr_batch_t* Ao,
                                  double sigma, int* env, const int64_t* doff, hipStream_t st);
// The shifted matrices' envelope from the patterns of A_N,j and A^o_j
// (lowers E from env_init's values; env_finish follows), and the zeroing of
// each matrix's envelope tiles (ntmax = largest tile count).
hipError_t launch_env_shifted(const int* nt, int nsub, int ntmax, const int* sub_ptr,
                              const geneo_csr_batch_t* An, const geneo_csr_batch_t* Ao, int* env,
                              const int64_t* doff, hipStream_t st);
hipError_t launch_env_clear(double* tiles, const int64_t* toff, const int* nt, int nsub,
                            int ntmax, const int* envE, const int64_t* doff, hipStream_t st);

// -------------------------------------------------------------- chol.hip
// envE / envR: the matrices' tile envelopes (NULL: dense).  Tiles outside
// the envelope are zero and are neither read nor written: the factors are
// bitwise those of the dense factorisation.
enum class CholRole { LocalF32, LocalF64, ShiftedF64 };
hipError_t launch_chol_batched(CholRole role, void* tiles, const int64_t* toff, const int* nt,
                               void* dinv, const int64_t* doff, int* status, const int* jobs,
                               int njobs, double pivtol, const int* envE, const int* envR,
                               hipStream_t st);
// jobs[] = (matrix, first tile column c0) with c0 a multiple of
// trtri_cols_per_job(fp32); tile columns c0 .. c0 + that - 1 are done.
// envE: the envelope of L (NULL: dense); X = L^{-1} is written in full.
int trtri_cols_per_job(bool fp32);
hipError_t launch_trtri(bool fp32, const void* L, const void* dinv, void* X,
                        const int64_t* toff, const int64_t* doff, const int* nt,
                        const int2* jobs, int njobs, const int* envE, hipStream_t st);
// S = X^T X (= A^{-1} for X = L^{-1}) from the transposed tiles k_trtri_win
// writes; jobs[] = (matrix, I << 16 | J0) for the output tiles (I, J0 ..
// J0 + lauum_tiles_per_job() - 1), J <= I, in the packed layout of toff.
int lauum_tiles_per_job();
hipError_t launch_lauum(bool fp32, const void* XT, void* S, const int64_t* toff, const int* nt,
                        const int2* jobs, int njobs, hipStream_t st);
// FP64 Cholesky of matrices jobs[0 .. njobs-1] (tiles at toff, inverted
// diagonal tiles to doff) by right-looking tile-column steps, 3 launches per
// step over all of them (maxnt = largest tile order): for a few matrices,
// where one workgroup per matrix would hold CUs for the whole
// factorisation.  status[j] = 0 or TS k + f at the first failed pivot: a
// pivot d fails unless d > *pivtol (pivtol: device, NULL = 0).  envR
// (device, at doff; NULL = dense): the last nonzero tile row of each tile
// column, below which the steps skip the zero tiles; rlast (host [maxnt],
// NULL = dense): its largest value over the matrices, which sizes the grids.
hipError_t launch_chol_steps(double* tiles, double* dinv, const int64_t* toff,
                             const int64_t* doff, const int* nt, const int* jobs, int njobs,
                             int maxnt, int* status, hipStream_t st,
                             const double* pivtol = nullptr, const int* envR = nullptr,
                             const int* rlast = nullptr);

// ------------------------------------------------------------- solve.hip
// `done` (device flag, may be NULL): skip the work once PCG has converged.
// Local solves of the apply, y_j = L_j^{-T} L_j^{-1} x_j with the Cholesky
// factor L_j of each subdomain's scaled Dirichlet matrix (packed tiles at
// toff, inverted diagonal tiles at doff, tile envelopes E / R at doff or
// NULL for dense): the subdomains jobs32[0 .. njobs32-1] with FP32
// factors, then jobs64[0 .. njobs64-1] with FP64 ones (two launches).
// Vectors at voff[j] (nt[j] * TS entries) in x and y.
struct LocalSolveArgs {
  const float *L32 = nullptr, *D32 = nullptr;
  const double *L64 = nullptr, *D64 = nullptr;
  const int64_t *toff32 = nullptr, *doff32 = nullptr, *toff64 = nullptr, *doff64 = nullptr;
  const int *E32 = nullptr, *R32 = nullptr, *E64 = nullptr, *R64 = nullptr;
  const int *nt = nullptr, *voff = nullptr;
  const int *jobs32 = nullptr, *jobs64 = nullptr;
  int njobs32 = 0, njobs64 = 0, maxnt = 0;
  const double* x = nullptr;
  double* y = nullptr;
};
hipError_t local_solve(const LocalSolveArgs& a, const int* done, hipStream_t st);
// hipSuccess if matrices of maxnt tile rows fit the local solves' LDS (and
// raises the kernel's LDS limit where they need more than the default)
hipError_t local_solve_check(int maxnt);
// y = S x for the symmetric inverses (packed lower tiles, diagonal tiles in
// full) of all subdomains and the coarse matrix: symv_rows forms the
// partial sums R and W, symv_cols then adds them into y (stream order).
// jobs[] = (subdomain, 1 if its inverse is FP64 in S64 (tiles at toff64)
// else FP32 in S32 (tiles at toff32)), or (., 2) for the coarse inverse SH
// with vectors xH -> yH.  W32 / W64 / WH hold TS partials per tile of S32 /
// S64 / SH, at the same tile offsets.
// One wavefront's work in symv_rows: tiles k0 .. k1-1 of tile row i of one
// matrix, kind 0 / 1 / 2 = FP32 subdomain (S32, W32), FP64 subdomain (S64,
// W64), coarse (SH, WH, vectors xH / yH).  Built on the host, one load per
// wavefront.
struct SymvTask {
  int64_t s_row;  // element offset of tile (i, 0) in S32 / S64 / SH
  int64_t w_row;  // element offset of W(i, 0) in W32 / W64 / WH
  int xoff;       // offset of the matrix's vectors in x / y (0 for the coarse)
  int r_off;      // element offset of this chunk's row partial in R
  short i, k0, k1, kind;
};
struct SymvArgs {
  const float* S32;
  const double* S64;
  const int64_t* toff32;
  const int64_t* toff64;
  const int* nt;
  const int* voff;
  const int2* jobs;
  int njobs, maxnt;  // maxnt covers ntc
  const double* SH;
  int ntc;
  float* W32;
  double* W64;
  double* WH;
  const double* x;
  double* y;
  const double* xH;
  double* yH;
  // symv_rows: one task per wavefront (ntasks), jobs in walk order
  const SymvTask* tasks;
  int ntasks;
  // chunks of the tile rows of the largest matrix (maxnt rows), rows in
  // order, symv_chunk_tiles() tiles each: cstart[i] = first chunk of row i
  // (maxnt + 1 entries); R holds njobs * nchunk row partials of TS sums,
  // job q's chunk t at (q * nchunk + t) * TS
  const int* cstart;
  int nchunk;
  double* R;
};
int symv_chunk_tiles();
// One matrix of the symmetric products, for the task generator: its tiles
// at toff (S32 / S64 / SH by kind), its vectors at xoff, nt tile rows, and
// the first index of its tasks in the forward and the reverse lists.
struct SymvJob {
  int64_t toff;
  int xoff, nt, kind, off_f, off_r, pad;
};
// Tasks of row i of a matrix with g chunk groups per task: ceil((i+1) / G),
// G = g * symv_chunk_tiles(); tasks of rows 0 .. i-1 (and chunks of rows
// 0 .. i-1 with G = symv_chunk_tiles()):
__host__ __device__ inline int64_t symv_tasks_before(int i, int G) {
  const int64_t f = i / G, r = i % G;
  return G * f * (f + 1) / 2 + r * (f + 1);
}
// Writes the tasks of every job q (g groups of symv_chunk_tiles() tiles per
// task, row partials at (q * nchunk + chunk) * TS) into fwd and rev.
hipError_t symv_make_tasks(const SymvJob* jobs, int njobs, int g, int nchunk, SymvTask* fwd,
                           SymvTask* rev, hipStream_t st);
hipError_t symv_rows(const SymvArgs& a, const int* done, hipStream_t st);
hipError_t symv_cols(const SymvArgs& a, const int* done, hipStream_t st);
// Triangular solves with the shifted factors, one workgroup per subdomain
// (split = 1) or b / 16 per subdomain, each on 16 of the b columns
// (split = trsm_max_split(b) > 1), for the first nsub entries of `order`
// (may be NULL = by index); `variant` (0 .. trsm_variants() - 1) picks the
// kernel (0 and 2 are not available unsplit for b = 48: 1 and 3 run).  envE / envR: the factors' tile envelopes
// (NULL: dense); the zero tiles outside them are skipped.  Every variant
// and split gives bitwise the same X, and so does the envelope.
int trsm_max_split(int b);
int trsm_variants();
hipError_t launch_trsm_fwd(const double* G, const double* dinv, const int64_t* toff,
                           const int64_t* doff, const int* nt, const int* voff, int nsub,
                           int b, const double* R, double* X, const int* active,
                           const int* order, const int* envE, const int* envR, int variant,
                           int split, hipStream_t st);
hipError_t launch_trsm_bwd(const double* G, const double* dinv, const int64_t* toff,
                           const int64_t* doff, const int* nt, const int* voff, int nsub,
                           int b, const double* R, double* X, const int* active,
                           const int* order, const int* envE, const int* envR, int variant,
                           int split, hipStream_t st);
// B_j = X_j A^o_j X_j in compact CSR over the nloc local rows: brp [nloc+1]
// (cnt [nloc] scratch), bcol / bval sized by the nonzeros of the A^o batch;
// maxrows bounds |N_j|.
// rpos (nloc + 1) / rows (up to nloc): the rows of B that hold entries,
// rpos[nloc] their number
hipError_t launch_bcompact(const int* sub_ptr, const double* pou, const geneo_csr_batch_t* Ao,
                           int nsub, int64_t nloc, int maxrows, int* cnt, int* brp, int* bcol,
                           double* bval, int* rpos, int2* rows, hipStream_t st);
hipError_t launch_bapply(const int* sub_ptr, const int* brp, const int* bcol, const double* bval,
                         const int2* rows, int nrows, const int* voff, int b, const double* X,
                         double* Y, const int* active, hipStream_t st);

// ------------------------------------------------------------- eigen.hip
hipError_t launch_eig_init(double* U, const int* sub_ptr, const int* voff, const int* nt,
                           int nsub, int b, uint64_t seed, hipStream_t st);
struct EigWork {
  double* G;     // nsub * b * b  Gram / Rayleigh quotient matrices
  double* M;     // nsub * b * b  small factors / Ritz rotations
  double* part;  // nsub * ngroups * b residual partial sums
  int* badcol;   // nsub * b collapsed-column flags
  int ngroups;   // slab groups per subdomain
};
hipError_t launch_orth2(double* U, const int* voff, const int* nt, int nsub, int b,
                        uint64_t seed, int salt, const int* active, const EigWork& wk,
                        hipStream_t st);
// Per-subdomain stagnation state of the eigen sweeps (see geneo_opts_t).
struct EigStall {
  double* best;  // nsub: smallest largest-wanted-residual so far
  int* count;    // nsub: sweeps since the last new minimum
  int* stalled;  // nsub: 1 once stopped at the floor
  int sweeps;    // 0 disables
  double floor;
};
// tau_sub (device, may be NULL): per-subdomain thresholds replacing tau
hipError_t launch_rr2(double* U, const double* W, double* Y, double* theta, double* resid,
                      int* active, const int* voff, const int* nt, int nsub, int b, int nev,
                      double tau, const double* tau_sub, int nev_max, double sigma, double tol,
                      const EigWork& wk, const EigStall& stl, hipStream_t st);
// Chebyshev filter step (see k_cheb): first ? Zn = (2/a) SZ - Zp
//                                          : Zn = (4/a) SZ - 2 Zc - Zp.
hipError_t launch_cheb(double* Zn, const double* Zc, const double* SZ, const double* Zp,
                       const double* theta, const int* voff, const int* nt, int nsub, int b,
                       int maxnt, bool first, const int* active, hipStream_t st);
hipError_t launch_select(const double* theta, int nsub, int b, int nev, double tau,
                         const double* tau_sub, int nev_max, double sigma, int* m, double* lam,
                         hipStream_t st);
hipError_t launch_basis(const double* P, const int* voff, int b, const int* sub_ptr,
                        const double* pou, const int* dmap, const int* m, const int* zoff,
                        const int* nd, int nsub, double* Z, hipStream_t st);

// ------------------------------------------------------------ coarse.hip
hipError_t launch_galerkin_w(const geneo_csr_batch_t* An, const int* sub_ptr, const int* dmap,
                             const double* Z, const int* zoff, const int* m,
                             const int* woff, int nsub, int64_t maxwork /* max_j |N_j| m_j */, double* W, hipStream_t st);
hipError_t launch_coarse_blocks(const int2* pairs, int npairs, const int* sub_ptr,
                                const int* sub_idx, const int* didx, const int* dvoff,
                                const int* nd, const double* Z, const int* zoff,
                                const double* W, const int* woff, const int* m,
                                const int* coff, double* AHt, hipStream_t st);
hipError_t launch_coarse_init(double* AHt, int ntc, int nc, hipStream_t st);
// *tol = nc * eps * max_k (A_H)_kk: the coarse factor's pivot threshold
hipError_t launch_coarse_pivtol(const double* AHt, int nc, double* tol, hipStream_t st);
hipError_t launch_coarse_to_dense(const double* AHt, int ntc, int nc, double* out,
                                  hipStream_t st);

// --------------------------------------------------------------- pcg.hip
struct PcgScalars;
hipError_t launch_spmv(const geneo_csr_t* A, const double* x, double* y, int lpr,
                       hipStream_t st);
hipError_t launch_gather_local(const double* r, const int* dglob, const double* dscale,
                               int64_t nvec, double* xl, hipStream_t st);
}  // namespace geneo
