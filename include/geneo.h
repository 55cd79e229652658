/*
 * geneo.h -- C ABI of libgeneo: GenEO two-level overlapping additive Schwarz
 * preconditioner inside preconditioned conjugate gradients, on one AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Seelinger, Reinarz, Scheichl, "A High-Performance Implementation of
 * a Robust Preconditioner for Heterogeneous Problems" (arXiv:1906.10944).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Pointers documented as "device" are HIP device pointers owned by the
 *    caller; pointers documented as "host" are ordinary host memory.
 *  - Indices are 0-based int32; every count must stay below 2^31.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *    stream).  Work is enqueued on it; an entry point returns once its
 *    results are complete on that stream unless stated otherwise.
 *  - Every entry point returns GENEO_OK (0) or one of the GENEO_ERR_* codes
 *    below; no C++ exception crosses the ABI.  geneo_strerror() maps a code
 *    to a message and geneo_last_error() gives the detail of the most recent
 *    failure in the calling thread.
 *  - Floating point is IEEE binary64 unless stated otherwise.
 */
#ifndef GENEO_H
#define GENEO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
enum {
  GENEO_OK = 0,
  GENEO_ERR_ARG = 1,            /* invalid argument or inconsistent sizes */
  GENEO_ERR_OOM = 2,            /* device allocation failed */
  GENEO_ERR_LOCAL_NOT_SPD = 3,  /* a local Dirichlet matrix failed its FP64 Cholesky */
  GENEO_ERR_EIGEN_NOCONV = 4,   /* eigen sweeps hit eig_maxit before eig_tol
                                   (or a stagnation above eig_floor) */
  GENEO_ERR_COARSE_NOT_SPD = 5, /* the coarse matrix A_H failed its Cholesky:
                                   a pivot at or below nc * eps * max_k (A_H)_kk
                                   (numerically singular, e.g. a repeated
                                   basis vector) */
  GENEO_ERR_MAXIT = 6,          /* PCG stopped at maxit; x and info are filled */
  GENEO_ERR_HIP = 7,            /* a HIP runtime call failed */
  GENEO_ERR_SHIFT_NOT_SPD = 8   /* A_N,j - sigma*B_j failed its Cholesky */
};

const char* geneo_strerror(int code);
const char* geneo_last_error(void);

/* Library version string, e.g. "geneo 0.1 gfx950". */
const char* geneo_version(void);

/* ------------------------------------------------ structured Q1 problems */
/*
 * A structured box grid of Q1 elements (Sec. 2: the Darcy form of eq. (2)
 * with ncomp = 1, the linear-elasticity form of eq. (3) without traction
 * with ncomp = 3) and its box partition into overlapping subdomains (Sec. 3).
 *
 *   elements  e = ix + ne[0]*(iy + ne[1]*iz)
 *   nodes     k = ix + (ne[0]+1)*(iy + (ne[1]+1)*iz)
 *   dofs      k*ncomp + c
 *   dirichlet bit (2*axis + side): homogeneous Dirichlet on that face
 *             (side 0 = coordinate 0, side 1 = far face)
 *   parts     subdomains per axis; the first ne % parts parts get one extra
 *             element; subdomain j = px + parts[0]*(py + parts[1]*pz);
 *             each part is widened by `ovl` element layers per side,
 *             clipped to the grid (ovl >= 1).
 * In 2D set ne[2] = parts[2] = 1 and h[2] = 1.
 */
typedef struct {
  int dim;            /* 2 or 3 */
  int ncomp;          /* 1 (Darcy) or 3 (elasticity, dim = 3 only) */
  int ne[3];          /* elements per axis */
  double h[3];        /* element edge lengths */
  int parts[3];       /* subdomains per axis */
  int ovl;            /* overlap in element layers, >= 1 */
  int dirichlet;      /* face bitmask */
  double load[3];     /* constant body load per component */
  int pou;            /* partition of unity: GENEO_POU_CONSTANT or
                         GENEO_POU_SARKIS (see geneo_assemble_q1) */
  int element;        /* GENEO_ELEM_Q1, or GENEO_ELEM_S20: 20-node
                         serendipity bricks (the element of the paper's
                         composite experiments, Sec. 5.3; 3D elasticity,
                         piecewise-constant partition of unity).  Nodes: the
                         points of the half-step lattice (coordinates 0 ..
                         2 ne per axis) with at most one odd coordinate,
                         numbered lexicographically (x fastest) over those;
                         element integrals by the 3-point Gauss rule. */
} geneo_grid_t;

enum { GENEO_POU_CONSTANT = 0, GENEO_POU_SARKIS = 1 };
enum { GENEO_ELEM_Q1 = 0, GENEO_ELEM_S20 = 1 };

/* Sizes of the arrays geneo_assemble_q1 writes. */
typedef struct {
  int64_t ndof;       /* global dofs N */
  int64_t nnz;        /* nonzeros of the global CSR matrix */
  int64_t nsub;       /* subdomains */
  int64_t nloc;       /* sum_j |N_j| (entries of the subdomain index lists) */
  int64_t nnz_loc;    /* nonzeros of the batched local (Neumann/overlap) CSR */
  int64_t nmax;       /* max_j |N_j| */
} geneo_q1_sizes_t;

/* Host-only size computation; no device work.  Returns GENEO_ERR_ARG for an
 * invalid grid. */
int geneo_q1_sizes(const geneo_grid_t* grid, geneo_q1_sizes_t* sizes);

/* The eigenvalue threshold of Thm. 1 for every subdomain of the box
 * partition: tau[j] = delta_j / H_j (host array [nsub]), with H_j the
 * diameter of Omega_j (the diagonal of its element box) and delta_j the
 * width of its overlap zone Omega_j^o, 2 * ovl * min_a h_a (the strips on
 * both sides of a neighbour's core boundary).  Host only; GENEO_ERR_ARG
 * for an invalid grid. */
int geneo_q1_thm1_tau(const geneo_grid_t* grid, double* tau);

/*
 * Device assembly of a structured Q1 problem (Sec. 2 eqs. (2)-(3); Sec. 3
 * for the subdomains; Sec. 4.3 for the local matrices and the partition of
 * unity).  All outputs are caller-allocated device arrays sized by
 * geneo_q1_sizes:
 *
 *  coeff      [nelem] kappa per element (ncomp = 1), or [nelem*21] the upper
 *             triangle of the 6x6 Voigt stiffness (order 11,22,33,23,13,12,
 *             engineering shear), row major (ncomp = 3).  Device, input.
 *  A_rowptr   [ndof+1], A_col [nnz], A_val [nnz]: global stiffness matrix
 *             (2^d-point Gauss), columns ascending, homogeneous Dirichlet
 *             conditions imposed by symmetric elimination (zero row and
 *             column, unit diagonal).
 *  b          [ndof]: load vector, zero at Dirichlet dofs.
 *  sub_ptr    [nsub+1], sub_idx [nloc]: N_j as ascending global dofs.
 *  sub_flags  [nloc]: bit0 = dof in D_j (not on the artificial boundary of
 *             Omega_j and not Dirichlet), bit1 = Dirichlet dof.
 *  pou        [nloc]: partition of unity (Def. 3), 0 outside D_j.
 *             GENEO_POU_CONSTANT: the piecewise-constant one of Fig. 1
 *             (left), 1/c_k on D_j (c_k = number of subdomains having k off
 *             their artificial boundary).  GENEO_POU_SARKIS: the smooth one
 *             of Fig. 1 (right), d_j(x_k) / sum_i d_i(x_k) on D_j, where
 *             d_i(x) is the distance (physical units) of node x from the
 *             faces of box Omega_i that lie inside Omega (0 when x is not
 *             in Omega_i; 1 for a box without such faces).
 *  loc_rowptr [nloc+1], loc_col [nnz_loc]: shared pattern of the batched
 *             local matrices; row r of subdomain j is global row
 *             sub_ptr[j] + r, columns are LOCAL indices into N_j.
 *  an_val     [nnz_loc]: Neumann matrices A_N,j (all elements of Omega_j,
 *             Dirichlet elimination on physical Dirichlet dofs only).
 *  ao_val     [nnz_loc]: overlap matrices A^o_j (elements of Omega_j lying
 *             in at least one other subdomain), same boundary treatment.
 */
int geneo_assemble_q1(const geneo_grid_t* grid, const double* coeff,
                      int* A_rowptr, int* A_col, double* A_val, double* b,
                      int* sub_ptr, int* sub_idx, uint8_t* sub_flags,
                      double* pou, int* loc_rowptr, int* loc_col,
                      double* an_val, double* ao_val, void* stream);

/* ----------------------------------------------------- general operators */

/* Global sparse SPD matrix A in CSR form (device arrays). */
typedef struct {
  int n;              /* rows = columns */
  int64_t nnz;
  const int* rowptr;  /* [n+1] */
  const int* col;     /* [nnz] */
  const double* val;  /* [nnz] */
} geneo_csr_t;

/*
 * Overlapping subdomains (Sec. 3) as index lists (device arrays):
 *  sub_ptr [nsub+1]  offsets into sub_idx
 *  sub_idx [nloc]    N_j: global dofs of subdomain j, strictly ascending
 *  sub_flags [nloc]  bit0: dof belongs to D_j, the dofs of the local
 *                    Dirichlet problem A_j = R_j A R_j^T
 *  pou [nloc]        partition-of-unity weights mu_{j,k} (Def. 3); they
 *                    must vanish outside D_j
 */
typedef struct {
  int nsub;
  int64_t nloc;
  const int* sub_ptr;
  const int* sub_idx;
  const uint8_t* sub_flags;
  const double* pou;
} geneo_subdomains_t;

/*
 * Block-diagonal batch of local matrices, one |N_j| x |N_j| block per
 * subdomain, in CSR form with LOCAL column indices (device arrays):
 * rows sub_ptr[j] .. sub_ptr[j+1]-1 belong to subdomain j.
 */
typedef struct {
  const int* rowptr;  /* [nloc+1] */
  const int* col;     /* local column indices */
  const double* val;
} geneo_csr_batch_t;

enum { GENEO_PREC_FP64 = 0, GENEO_PREC_MIXED = 1 };
/* Forms of the local solves A_j^{-1} r_j of the apply (Def. 2), option
 * local_solve: forward and backward substitution with the banded Cholesky
 * factor, or one product with the symmetric inverse formed in the setup. */
enum { GENEO_LOCAL_AUTO = 0, GENEO_LOCAL_TRIANGULAR = 1, GENEO_LOCAL_INVERSE = 2 };

typedef struct {
  int nev;            /* eigenvectors per subdomain when tau <= 0 */
  double tau;         /* > 0: take eigenvalues < tau ... */
  int nev_max;        /* ... at most nev_max of them */
  double sigma;       /* shift of the spectral transform, < 0 (Sec. 4.4) */
  int precision;      /* GENEO_PREC_FP64 or GENEO_PREC_MIXED: FP32 local
                         Dirichlet factors (diagonally scaled) with a per-
                         subdomain FP64 refactor when the pivot test fails */
  double pivot_tol;   /* FP32 pivot test: a scaled Schur pivot below this
                         fails the subdomain over to FP64 */
  double eig_tol;     /* Ritz residual ||S y - nu y|| <= eig_tol * ||S||,
                         S = G^{-1} B G^{-T}, ||S|| = nu_max */
  int eig_maxit;      /* maximum subspace sweeps */
  int eig_block;      /* block size (multiple of 16, <= 64); 0 = automatic */
  uint64_t seed;      /* seed of the start block of the subspace iteration */
  int coarse;         /* 1: two-level method (Def. 2); 0: one level only */
  int eig_stall;      /* > 0: a subdomain whose largest wanted residual has
                         not halved for eig_stall sweeps (rounding floor of
                         its shifted solves, or a ratio close to 1) stops if
                         that residual is <= eig_floor * ||S|| (and counts in
                         geneo_setup_info_t.eig_stalled).  0 disables. */
  double eig_floor;   /* largest residual accepted at such a stagnation */
  int eig_cheb;       /* >= 2: from the third sweep on, the Ritz block is
                         filtered by the Chebyshev polynomial of this degree
                         on [0, a] (a = smallest Ritz value of the block)
                         before it is orthonormalised: eig_cheb - 1 extra
                         shifted solves per sweep, faster convergence of the
                         wanted pairs.  0 or 1: plain subspace iteration.
                         At most 6 (GENEO_ERR_ARG above): the filter grows
                         like x^degree, and a floating subdomain's kernel
                         modes (Ritz values near 1/|sigma|) would outgrow the
                         smallest wanted ones by more than 1/u and erase
                         them (degree 8 stalls every floating subdomain of
                         the 96^3 layers). */
  int symv_tiles;     /* tiles per wavefront in the products with the local
                         inverses: 8, 16 or 32, or 0 = the fastest of these,
                         timed on the device at the first setup of each
                         problem shape and kept for that device and shape
                         (results are bitwise the same for every value) */
  int refine;         /* iterative-refinement steps after each PCG solve
                         (0..8): r = b - A x with every row summed in
                         double-double, A d = r by PCG to refine_rtol |r|,
                         x += d.  0 = the plain method. */
  double refine_rtol; /* tolerance of the correction solves */
  int eig_solve;      /* kernel of the eigen sweeps' triangular solves
                         (b <= 48): 1 = two tile rows per wavefront (b <= 32,
                         or 16-column blocks), 2 = one row per wavefront with
                         deeper load pipelines, both with 8 wavefronts per
                         subdomain; 3, 4 = the same with 4 (two subdomains
                         per CU); 0 = the fastest, timed on the device at the
                         first setup of each problem shape */
  int eig_split;      /* 16-column blocks on b / 16 workgroups per
                         subdomain (b = 32, 48) in the sweeps that start
                         with at most this many subdomains active (as far
                         as the host knows): -1 = never, 0 = a limit timed
                         at the first setup of the shape.  Every eig_solve
                         / eig_split choice gives bitwise the same result. */
  int envelope;       /* 1 = the local factorisations and the eigen solves
                         skip the tiles outside each matrix's envelope
                         (left of the first entry of each row: zero in the
                         Cholesky factor, as no fill reaches them), and the
                         shifted matrices clear only their envelope tiles;
                         0 = dense.  Both give bitwise the same result.
                         2 = as 1, with the shifted matrices' tiles outside
                         the envelope filled with NaN (a check that nothing
                         reads them). */
  int shifted_steps;  /* the shifted factorisations A_N,j - sigma B_j by
                         tile-column steps, each step one launch over all
                         subdomains with a workgroup per trailing tile (for
                         few large subdomains, where one workgroup per
                         matrix would leave most compute units idle):
                         1 = always, -1 = never (one workgroup per matrix),
                         0 = when there are at most 32 subdomains.  The
                         two differ in rounding order only. */
  int local_solve;    /* form of the apply's local solves:
                         GENEO_LOCAL_TRIANGULAR (two substitutions with the
                         Cholesky factor, inside its envelope: two reads of
                         the band per apply, row-by-row latency),
                         GENEO_LOCAL_INVERSE (one fully parallel product
                         with A_j^{-1} = L^{-T} L^{-1}, formed in the setup:
                         one read of the dense packed inverse), or
                         GENEO_LOCAL_AUTO (0): the one with the smaller
                         estimated time per iteration for the problem's
                         sizes (large banded 3D subdomains: triangular;
                         small or few subdomains: inverse).  The two agree
                         up to rounding. */
  const double* tau_sub; /* host [nsub], or NULL: per-subdomain thresholds
                         tau_j > 0 replacing tau (take the eigenvalues
                         < tau_j, at most nev_max of them), e.g. the
                         delta_j / H_j of Thm. 1 (geneo_q1_thm1_tau).  Read
                         during geneo_setup only. */
} geneo_opts_t;

/* Fills the defaults: nev 8, tau 0 (fixed count), nev_max 16,
 * sigma -1e-3, FP64, pivot_tol 1e-3, eig_tol 1e-8, eig_maxit 300,
 * eig_block 0, seed 0, coarse 1, eig_stall 10, eig_floor 1e-6, eig_cheb 4,
 * symv_tiles 0, refine 0, refine_rtol 1e-6, eig_solve 0, eig_split 0,
 * envelope 1, shifted_steps 0, local_solve 0, tau_sub NULL. */
void geneo_default_opts(geneo_opts_t* opts);

typedef struct geneo_handle_s* geneo_handle_t;

/*
 * Setup of the two-level additive Schwarz preconditioner
 *   M^{-1} = R_H^T A_H^{-1} R_H + sum_j R_j^T A_j^{-1} R_j      (Def. 2)
 * with the GenEO coarse space (Def. 4): for each subdomain the m_j smallest
 * eigenpairs of A_N,j p = lambda X_j A^o_j X_j p (Sec. 4.3, discrete eq. (4)),
 * solved with the shift-and-invert transform (Sec. 4.4); coarse basis
 * vectors X_j p / ||X_j p||_2; A_H = Z^T A Z (Def. 2, Sec. 4.5).
 *
 *  A      global matrix (device); A_j = A[D_j, D_j] is read from it.
 *  subs   subdomain lists and partition of unity (device).
 *  An     batched Neumann matrices A_N,j (device); needed when coarse = 1.
 *  Ao     batched overlap matrices A^o_j (device); needed when coarse = 1.
 *  opts   host; NULL = defaults.
 *  out    receives the handle.
 * The handle copies or derives everything it keeps: inputs may be freed
 * once the call returns.  Errors: GENEO_ERR_ARG, GENEO_ERR_OOM,
 * GENEO_ERR_LOCAL_NOT_SPD, GENEO_ERR_SHIFT_NOT_SPD, GENEO_ERR_EIGEN_NOCONV,
 * GENEO_ERR_COARSE_NOT_SPD, GENEO_ERR_HIP; on error *out is NULL.
 */
int geneo_setup(const geneo_csr_t* A, const geneo_subdomains_t* subs,
                const geneo_csr_batch_t* An, const geneo_csr_batch_t* Ao,
                const geneo_opts_t* opts, void* stream, geneo_handle_t* out);

/* z = M^{-1} r (Def. 2).  r, z: device [n]; may not alias.  Asynchronous:
 * returns after enqueueing on `stream`. */
int geneo_apply(geneo_handle_t h, const double* r, double* z, void* stream);

/* Releases every device buffer of the handle (synchronises the device
 * first).  NULL is ignored.  The library keeps released device blocks, up
 * to 64 GiB per device, for reuse by later setups; geneo_trim() returns
 * them to the driver. */
void geneo_destroy(geneo_handle_t h);

/* Returns the device blocks the library keeps for reuse (released by
 * destroyed handles and finished setups) to the driver, for the current
 * device.  Synchronises the device.  GENEO_OK or GENEO_ERR_HIP. */
int geneo_trim(void);

typedef struct {
  int nsub;
  int nc;                 /* dim V_H = sum_j m_j */
  int fallback_fp64;      /* subdomains refactored in FP64 (mixed mode) */
  int eig_sweeps;         /* subspace sweeps used */
  int eig_block;          /* block size used */
  double eig_max_resid;   /* largest relative Ritz residual of a kept pair */
  double t_setup_ms;      /* wall time of geneo_setup */
  double t_phase_ms[8];   /* 0 index lists, 1 local factors, 2 shifted
                             factors, 3 eigen sweeps, 4 basis + Galerkin,
                             5 coarse factor, 6-7 reserved */
  int64_t bytes_local_factors;  /* bytes of what the apply keeps for the
                                   local solves: the Cholesky factors with
                                   their inverted diagonal tiles, or the
                                   symmetric inverses */
  int eig_stalled;        /* subdomains stopped at their rounding floor */
  int symv_tiles;         /* tiles per wavefront of the local products */
  int eig_solve;          /* triangular-solve kernel of the eigen sweeps'
                             unsplit solves (1 .. 4, see geneo_opts_t) */
  int eig_split;          /* the sweeps' solves are split into 16-column
                             blocks while at most this many subdomains are
                             active (0 = never) */
  int local_solve;        /* GENEO_LOCAL_TRIANGULAR or GENEO_LOCAL_INVERSE:
                             the form the apply uses */
  int eig_solve_split;    /* kernel of the split (16-column) solves, 1 .. 4
                             as eig_solve */
} geneo_setup_info_t;

int geneo_get_setup_info(geneo_handle_t h, geneo_setup_info_t* info);

/* Host copies of the selected eigen data: m [nsub] counts and
 * lam [nsub*ldl] eigenvalues (ascending, first m_j valid, the rest of each
 * row filled with the further computed Ritz values or +inf). */
int geneo_get_eigenvalues(geneo_handle_t h, int* m, double* lam, int ldl);

/* Host copy of the precision of each local solve with A_j (Sec. 3): fp64
 * [nsub] receives 1 where the Cholesky factor of A_j is kept in FP64 (FP64
 * mode, or in mixed mode a subdomain whose FP32 factor failed the pivot
 * test) and 0 where it is FP32. */
int geneo_get_local_precision(geneo_handle_t h, int* fp64);

/* Host copies of the coarse basis (Def. 4) as dense columns over N_j:
 * zoff [nsub+1] (host) receives the VALUE offsets of the blocks,
 * zoff[j] = sum_{i<j} |N_i| m_i, so zoff[nsub] is the length z needs (the
 * column offsets sum_{i<j} m_i follow from geneo_get_eigenvalues' counts).
 * `z` (optional, host) receives, for each subdomain j, the |N_j| x m_j
 * block row major at offset zoff[j]; zsize is its length, at least
 * zoff[nsub], else GENEO_ERR_ARG.  `ah` (optional, host, may be NULL)
 * receives A_H = Z^T A Z (Def. 2) as nc x nc row major. */
int geneo_get_coarse(geneo_handle_t h, int64_t* zoff, double* z, int64_t zsize,
                     double* ah);

/* -------------------------------------------------------------- the solve */
typedef struct {
  int iters;            /* products with A */
  int converged;        /* ||b - A x||_2 <= rtol ||b||_2 on the recurrence */
  double relres;        /* final recurrence residual / ||b|| */
  double kappa_est;     /* CG-Lanczos condition number estimate */
  double t_solve_ms;    /* wall time of the solve (refinement included) */
  int refine_iters;     /* PCG iterations of the refinement steps */
  double true_relres;   /* |b - A x| / |b| of the returned x, the residual
                           summed in double-double */
} geneo_pcg_info_t;

/*
 * Preconditioned CG (x0 = 0 is NOT assumed: x holds the start vector) for
 * A x = b with the two-level preconditioner M, stopped as soon as the
 * recurrence residual satisfies ||r_k||_2 <= rtol ||b||_2 (the residual
 * reduction used in Sec. 5), iteration count = products with A.  A zero b,
 * or a start vector already within the tolerance, returns 0 iterations
 * with x unchanged.
 *  A     device CSR; b, x device [n] (x in: start vector, out: solution);
 *  nrhs  right-hand sides stored one after the other (b, x of size n*nrhs),
 *        solved independently; info (host) has nrhs entries.
 * The iterations run on M's own stream, ordered after the work already
 * enqueued on `stream`, and `stream` is ordered after them; the call
 * returns once the solve is complete.  Solves on one handle must not
 * overlap (they share its work vectors); different handles may solve
 * from different threads at once.
 * Returns GENEO_ERR_MAXIT if any right-hand side did not converge.
 */
int pcg_solve(const geneo_csr_t* A, geneo_handle_t M, const double* b,
              double* x, int nrhs, double rtol, int maxit,
              geneo_pcg_info_t* info, void* stream);

/*
 * pcg_solve without any allocation, for callers that cannot allocate device
 * memory during the solve (tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, semantics and results as pcg_solve (the
 * same kernels in the same order), with these differences:
 *  - the PCG vectors, the refinement correction and residual, partial
 *    sums, scalars and coefficient records live in one fixed device array
 *    of the library (56.1 MiB per GPU, held from the first call on that GPU
 *    until the process ends) instead of buffers the handle allocates; no
 *    hipMalloc, hipFree, pinned allocation, event or graph is created;
 *  - limits: n <= 1048576 and maxit <= 4096, else GENEO_ERR_ARG;
 *  - the iterations run directly on `stream`, without graph capture, and
 *    the host reads the done flag every 8 iterations, so the call is not
 *    capturable itself;
 *  - every call on one GPU shares that array, and it keeps the last call's
 *    contents: calls that overlap on one GPU (any handles, any streams)
 *    race and must be serialised by the caller.
 */
int pcg_solve_noalloc(const geneo_csr_t* A, geneo_handle_t M, const double* b,
                      double* x, int nrhs, double rtol, int maxit,
                      geneo_pcg_info_t* info, void* stream);

/* y = A x with the library's CSR kernel (device arrays). */
int geneo_spmv(const geneo_csr_t* A, const double* x, double* y, void* stream);

/* ----------------------------------------------------- kernel timing --- */
/*
 * Benchmark instrumentation.  geneo_prof_enable(1) clears earlier records
 * and makes the library record a HIP event pair, on the launch stream,
 * around each launch of its main kernels (launches inside graph capture
 * are not recorded); geneo_prof_enable(0) stops recording.  Each record
 * carries the algorithmic bytes and flops of that launch.
 * geneo_prof_query sums the records of one kernel name (host pointers):
 * total_ms (event time), launches, bytes and flops (either may be NULL).
 * Names: "densify_dirichlet", "chol_dirichlet_f32", "chol_dirichlet_f64",
 * "densify_shifted", "chol_shifted_f64", "trsm_bwd", "trsm_fwd",
 * "trsm_bwd_split", "trsm_fwd_split" (the eigen solves on 16-column
 * blocks), "bapply", "rayleigh_ritz", "cheb_combine", "orth",
 * "coarse_chol", "local_solve" (the apply's local solves), "symv" and
 * "symv_cols" (its coarse product).  While timing is
 * on, the eigen sweeps read their convergence flags after every sweep
 * (instead of one sweep late), so that the byte counts follow the active
 * set exactly.
 */
void geneo_prof_enable(int on);
int geneo_prof_query(const char* kernel, double* total_ms, int* launches, double* bytes,
                     double* flops);

#ifdef __cplusplus
}
#endif
#endif /* GENEO_H */
