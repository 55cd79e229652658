// PCG device state and solve-phase launchers.
#pragma once
#include "internal.h"

namespace geneo {

#define PCG_NB 512  // fixed number of partial sums per reduction
#define PCG_NB_SPMV 2048  // blocks (and p.q partial sums) of the fused p / SpMV launch

struct PcgScalars {
  double rz, pq, rr, alpha, beta, tol2, bb;
  int iters, maxit, converged, pad;
};

hipError_t spmv(const geneo_csr_t* A, const double* x, double* y, int lpr, const int* done,
                hipStream_t st);
int spmv_lanes(const geneo_csr_t* A);
hipError_t gather_local(const double* r, const int* dglob, const double* dscale, int64_t nvec,
                        double* xl, const int* done, hipStream_t st);
hipError_t restrict_coarse(const double* r, const double* Z, const int* zoff, const int* m,
                           const int* nd, const int* dglob, const int* dvoff, const int* coff,
                           int nsub, double* rH, const int* done, hipStream_t st);
// oent[p]: owner entry p resolved to (D-vector position or -1, offset of
// its row of Z_j, coarse offset of j, m_j)
hipError_t owner_entries(const int2* olist, int64_t nent, const int* sub_ptr, const int* dmap,
                         const int* dvoff, const int* zoff, const int* m, const int* coff,
                         int4* oent, hipStream_t st);
hipError_t combine(const double* r, const int* optr, const int4* oent, const double* dscale,
                   const double* yl, const double* Z, const double* yH, int ndof, int use_coarse,
                   double* z, const int* done, double* rz_partial,
                   hipStream_t st);  // rz_partial (may be NULL): r.z per 256-row block
hipError_t dot_partial(const double* x, const double* y, int n, double* partial, const int* done,
                       hipStream_t st);
// device-side start: stage 0 from the b.b partials (scalars reset, tol2,
// done for b = 0), stage 1 from the r0.r0 partials (done if within tol2)
hipError_t pcg_start(const double* partial, int stage, PcgScalars* sc, int* done, double rtol2,
                     int maxit, hipStream_t st);
hipError_t residual0(const double* b, const double* q, double* r, int n, hipStream_t st);
// r = b - A x, each row summed in double-double and rounded once
hipError_t residual_dd(const geneo_csr_t* A, const double* b, const double* x, double* r,
                       hipStream_t st);
hipError_t add_into(double* x, const double* d, int n, hipStream_t st);  // x += d
hipError_t fill_i32(int* p, int v, int n, hipStream_t st);
// fused PCG iteration pieces (scalars formed in the consumers)
// p = z + beta p (pin -> pout), q = A p, p.q partials (npq blocks)
hipError_t p_spmv(const geneo_csr_t* A, int lpr, const double* z, const double* pin,
                  double* pout, double* q, const double* rz_part, int nrz, PcgScalars* sc,
                  double* betas, double* pq_part, int npq, const int* done, hipStream_t st);
hipError_t update_xr_alpha(double* x, double* r, const double* p, const double* q, int n,
                           const double* pq_part, int npq, const double* rz_part, int nrz,
                           PcgScalars* sc, double* alphas, double* rr_part, const int* done,
                           hipStream_t st);
hipError_t check_apply_in(const double* r, const int* dglob, const double* dscale, int64_t nvec,
                          double* xl, const double* Z, const int* zoff, const int* m, const int* nd,
                          const int* dvoff, const int* coff, double* rH, int nrestrict,
                          const double* rr_part, PcgScalars* sc, int* done, hipStream_t st);

}  // namespace geneo
