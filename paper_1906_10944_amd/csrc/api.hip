// C ABI of libgeneo: argument checks, buffer ownership and the order of the
// setup phases, the preconditioner apply and the graph-captured PCG loop.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"
#include "pcg.h"
#include "prof.h"
#include "q1.h"

using namespace geneo;

namespace {

thread_local std::string g_last_error;

struct Err {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg) { throw Err{code, msg}; }

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      fail(e_ == hipErrorOutOfMemory ? GENEO_ERR_OOM : GENEO_ERR_HIP,                   \
           std::string(#expr) + " -> " + hipGetErrorString(e_));                        \
  } while (0)

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void alloc(size_t cnt) {
    release();
    if (cnt == 0) cnt = 1;
    HIPCHK(hipMalloc((void**)&p, cnt * sizeof(T)));
    n = cnt;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void upload(const std::vector<T>& v, hipStream_t st) {
    alloc(v.size());
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
};

template <typename T>
std::vector<T> download(const T* d, size_t n, hipStream_t st) {
  std::vector<T> h(n);
  if (n) HIPCHK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return h;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// extreme eigenvalues of a symmetric tridiagonal matrix by Sturm bisection
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    double off = i ? e[i - 1] * e[i - 1] : 0.0;
    q = d[i] - x - (i ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

double tridiag_eig(const std::vector<double>& d, const std::vector<double>& e, int k) {
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < d.size(); ++i) {
    double r = (i ? fabs(e[i - 1]) : 0.0) + (i + 1 < d.size() ? fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (sturm_count(d, e, mid) > k) hi = mid;
    else lo = mid;
    if (hi - lo <= 1e-14 * std::max(fabs(lo), fabs(hi))) break;
  }
  return 0.5 * (lo + hi);
}

double packed(double n) { return n * (n + 1.0) * 0.5; }

}  // namespace

struct geneo_handle_s {
  int n = 0, nsub = 0;
  int64_t nloc = 0;
  geneo_opts_t opts{};
  hipStream_t hs = nullptr;
  LocalLayout LD;
  DBuf<int> sub_ptr, sub_idx, dmap, nd, ntD, voffD, dglob, didx, jobs32, jobs64;
  DBuf<int64_t> toffD, doffD, toff64, doff64;
  DBuf<double> dscale;
  DBuf<float> X32;
  DBuf<double> X64;
  int njobs32 = 0, njobs64 = 0;
  DBuf<int> optr;
  DBuf<int2> olist;
  // coarse space
  int nc = 0, ntc = 0, b = 0;
  DBuf<int> m, zoff, coff, hjob, hnt, hvoff;
  DBuf<int64_t> htoff;
  DBuf<double> Z, XH, rH, tH, yH, AHdense;
  std::vector<int> m_host, nd_host, nN_host, sub_ptr_host;
  std::vector<double> lam_host;
  // apply workspace
  DBuf<double> xl, tl, yl;
  // pcg workspace
  int pcg_cap = 0, pcg_maxit = 0;
  DBuf<double> r, z, p, q, partial, alphas, betas;
  DBuf<PcgScalars> sc;
  DBuf<int> done;
  int lpr = 8;
  double bytes_trmv32 = 0.0, bytes_trmv64 = 0.0;  // algorithmic bytes per launch
  geneo_setup_info_t info{};
  ~geneo_handle_s() {
    if (hs) (void)hipStreamDestroy(hs);
  }
};

namespace {

void check_csr(const geneo_csr_t* A) {
  if (!A || A->n <= 0 || !A->rowptr || !A->col || !A->val || A->nnz <= 0)
    fail(GENEO_ERR_ARG, "invalid CSR matrix");
}

hipError_t apply_enqueue(geneo_handle_s* h, const double* r, double* z, const int* done,
                         hipStream_t st) {
  hipError_t e;
  if ((e = gather_local(r, h->dglob.p, h->dscale.p, h->LD.nvec, h->xl.p, done, st))) return e;
  {
    ProfScope ps(h->njobs32 ? "trmv_lower_f32" : nullptr, st, h->bytes_trmv32, 2.0 * h->bytes_trmv32 / 4.0);
    if ((e = trmv_lower(true, h->X32.p, h->toffD.p, h->ntD.p, h->voffD.p, h->jobs32.p,
                        h->njobs32, h->LD.maxnt, h->xl.p, h->tl.p, done, st)))
      return e;
  }
  {
    ProfScope ps(h->njobs64 ? "trmv_lower_f64" : nullptr, st, h->bytes_trmv64, 2.0 * h->bytes_trmv64 / 8.0);
    if ((e = trmv_lower(false, h->X64.p, h->toff64.p, h->ntD.p, h->voffD.p, h->jobs64.p,
                        h->njobs64, h->LD.maxnt, h->xl.p, h->tl.p, done, st)))
      return e;
  }
  {
    ProfScope ps(h->njobs32 ? "trmv_upperT_f32" : nullptr, st, h->bytes_trmv32, 2.0 * h->bytes_trmv32 / 4.0);
    if ((e = trmv_upperT(true, h->X32.p, h->toffD.p, h->ntD.p, h->voffD.p, h->jobs32.p,
                         h->njobs32, h->LD.maxnt, h->tl.p, h->yl.p, done, st)))
      return e;
  }
  {
    ProfScope ps(h->njobs64 ? "trmv_upperT_f64" : nullptr, st, h->bytes_trmv64, 2.0 * h->bytes_trmv64 / 8.0);
    if ((e = trmv_upperT(false, h->X64.p, h->toff64.p, h->ntD.p, h->voffD.p, h->jobs64.p,
                         h->njobs64, h->LD.maxnt, h->tl.p, h->yl.p, done, st)))
      return e;
  }
  if (h->nc > 0) {
    if ((e = restrict_coarse(r, h->Z.p, h->zoff.p, h->m.p, h->nd.p, h->dglob.p, h->voffD.p,
                             h->coff.p, h->nsub, h->rH.p, done, st)))
      return e;
    if ((e = trmv_lower(false, h->XH.p, h->htoff.p, h->hnt.p, h->hvoff.p, h->hjob.p, 1, h->ntc,
                        h->rH.p, h->tH.p, done, st)))
      return e;
    if ((e = trmv_upperT(false, h->XH.p, h->htoff.p, h->hnt.p, h->hvoff.p, h->hjob.p, 1, h->ntc,
                         h->tH.p, h->yH.p, done, st)))
      return e;
  }
  return combine(h->optr.p, h->olist.p, h->sub_ptr.p, h->dmap.p, h->voffD.p, h->dscale.p,
                 h->yl.p, h->Z.p, h->zoff.p, h->m.p, h->coff.p, h->yH.p, h->n, h->nc > 0, z, done,
                 st);
}

__global__ void k_count_active(const int* a, int n, int* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int c = 0;
    for (int i = 0; i < n; ++i) c += a[i] != 0;
    *out = c;
  }
}

__global__ void k_max_resid(const double* resid, const int* m, int nsub, int b, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double mx = 0.0;
    for (int j = 0; j < nsub; ++j)
      for (int c = 0; c < m[j]; ++c) mx = fmax(mx, resid[(int64_t)j * b + c]);
    *out = mx;
  }
}

void setup_impl(geneo_handle_s* h, const geneo_csr_t* A, const geneo_subdomains_t* S,
                const geneo_csr_batch_t* An, const geneo_csr_batch_t* Ao, hipStream_t st) {
  const geneo_opts_t& o = h->opts;
  const double t_start = now_ms();
  double t_mark = t_start;
  auto phase = [&](int k) {
    HIPCHK(hipStreamSynchronize(st));
    double t = now_ms();
    h->info.t_phase_ms[k] = t - t_mark;
    t_mark = t;
  };
  const int nsub = S->nsub;
  h->n = A->n;
  h->nsub = nsub;
  h->nloc = S->nloc;
  h->lpr = spmv_lanes(A);
  HIPCHK(hipStreamCreateWithFlags(&h->hs, hipStreamNonBlocking));

  // ---- 0. index lists, D_j maps, scaling, owner lists
  h->sub_ptr_host = download(S->sub_ptr, nsub + 1, st);
  const auto& sp = h->sub_ptr_host;
  if (sp[0] != 0 || sp[nsub] != S->nloc) fail(GENEO_ERR_ARG, "sub_ptr does not span nloc");
  h->nN_host.resize(nsub);
  for (int j = 0; j < nsub; ++j) {
    if (sp[j + 1] <= sp[j]) fail(GENEO_ERR_ARG, "empty or decreasing subdomain");
    h->nN_host[j] = sp[j + 1] - sp[j];
  }
  h->sub_ptr.alloc(nsub + 1);
  HIPCHK(hipMemcpyAsync(h->sub_ptr.p, S->sub_ptr, (nsub + 1) * sizeof(int), hipMemcpyDeviceToDevice, st));
  h->sub_idx.alloc(S->nloc);
  HIPCHK(hipMemcpyAsync(h->sub_idx.p, S->sub_idx, S->nloc * sizeof(int), hipMemcpyDeviceToDevice, st));
  h->dmap.alloc(S->nloc);
  h->nd.alloc(nsub);
  HIPCHK(launch_dmap(S->sub_ptr, S->sub_flags, nsub, h->dmap.p, h->nd.p, st));
  h->nd_host = download(h->nd.p, nsub, st);
  h->LD.build(h->nd_host);
  h->ntD.upload(h->LD.nt, st);
  h->voffD.upload(h->LD.voff, st);
  h->toffD.upload(h->LD.toff, st);
  h->doffD.upload(h->LD.doff, st);
  h->dglob.alloc(h->LD.nvec);
  h->didx.alloc(h->LD.nvec);
  h->dscale.alloc(h->LD.nvec);
  HIPCHK(launch_dvec(S->sub_ptr, S->sub_idx, h->dmap.p, h->voffD.p, h->ntD.p, nsub, A,
                     h->dglob.p, h->didx.p, h->dscale.p, st));
  {
    DBuf<int> ocount;
    ocount.alloc(h->n);
    h->optr.alloc(h->n + 1);
    h->olist.alloc(S->nloc);
    HIPCHK(launch_owners(S->sub_ptr, S->sub_idx, nsub, S->nloc, h->n, h->optr.p, ocount.p,
                         h->olist.p, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  phase(0);

  // ---- 1. local Dirichlet factors A_j = R_j A R_j^T and their inverses
  DBuf<int> status;
  status.alloc(nsub);
  std::vector<int> all(nsub);
  for (int j = 0; j < nsub; ++j) all[j] = j;
  std::vector<int> f64list;
  const bool mixed = o.precision == GENEO_PREC_MIXED;
  if (mixed) {
    DBuf<int> jobs;
    jobs.upload(all, st);
    DBuf<float> L32, D32;
    L32.alloc(h->LD.ntiles * TSQ);
    D32.alloc(h->LD.ndiag * TSQ);
    double pk = 0.0, fl = 0.0;
    for (int j = 0; j < nsub; ++j) {
      pk += packed(h->nd_host[j]);
      fl += std::pow((double)h->nd_host[j], 3) / 3.0;
    }
    {
      ProfScope ps("densify_dirichlet", st, 4.0 * h->LD.ntiles * TSQ, 0.0);
      HIPCHK(launch_densify_dirichlet(true, L32.p, h->toffD.p, h->ntD.p, h->voffD.p, jobs.p,
                                      nsub, S->sub_ptr, S->sub_idx, h->dmap.p, h->dglob.p,
                                      h->dscale.p, A, st));
    }
    {
      ProfScope ps("chol_dirichlet_f32", st, 2.0 * 4.0 * pk, fl);
      HIPCHK(launch_chol_batched(true, L32.p, h->toffD.p, h->ntD.p, D32.p, h->doffD.p, status.p,
                                 jobs.p, nsub, o.pivot_tol, st));
    }
    auto stat = download(status.p, nsub, st);
    std::vector<int> ok32;
    for (int j = 0; j < nsub; ++j) (stat[j] ? f64list : ok32).push_back(j);
    h->njobs32 = (int)ok32.size();
    h->jobs32.upload(ok32, st);
    if (!ok32.empty()) {
      std::vector<int2> tj;
      for (int j : ok32)
        for (int c = 0; c < h->LD.nt[j]; ++c) tj.push_back(make_int2(j, c));
      DBuf<int2> tjobs;
      tjobs.upload(tj, st);
      h->X32.alloc(h->LD.ntiles * TSQ);
      double pk32 = 0.0, fl32 = 0.0;
      for (int j : ok32) {
        pk32 += packed(h->nd_host[j]);
        fl32 += std::pow((double)h->nd_host[j], 3) / 3.0;
      }
      ProfScope ps("trtri_dirichlet", st, 2.0 * 4.0 * pk32, fl32);
      HIPCHK(launch_trtri(true, L32.p, D32.p, h->X32.p, h->toffD.p, h->doffD.p, h->ntD.p, tjobs.p,
                          (int)tj.size(), st));
      HIPCHK(hipStreamSynchronize(st));
    }
  } else {
    f64list = all;
  }
  h->info.fallback_fp64 = mixed ? (int)f64list.size() : 0;
  h->njobs64 = (int)f64list.size();
  h->jobs64.upload(f64list, st);
  {
    std::vector<int64_t> toff64(nsub, 0), doff64(nsub, 0);
    int64_t tt = 0, dd = 0;
    for (int j : f64list) {
      toff64[j] = tt;
      doff64[j] = dd;
      tt += tri_tiles(h->LD.nt[j]);
      dd += h->LD.nt[j];
    }
    h->toff64.upload(toff64, st);
    h->doff64.upload(doff64, st);
    if (!f64list.empty()) {
      DBuf<double> L64, D64;
      L64.alloc(tt * TSQ);
      D64.alloc(dd * TSQ);
      double pk64 = 0.0, fl64 = 0.0;
      for (int j : f64list) {
        pk64 += packed(h->nd_host[j]);
        fl64 += std::pow((double)h->nd_host[j], 3) / 3.0;
      }
      {
        ProfScope ps("densify_dirichlet", st, 8.0 * tt * TSQ, 0.0);
        HIPCHK(launch_densify_dirichlet(false, L64.p, h->toff64.p, h->ntD.p, h->voffD.p,
                                        h->jobs64.p, h->njobs64, S->sub_ptr, S->sub_idx,
                                        h->dmap.p, h->dglob.p, h->dscale.p, A, st));
      }
      {
        ProfScope ps("chol_dirichlet_f64", st, 2.0 * 8.0 * pk64, fl64);
        HIPCHK(launch_chol_batched(false, L64.p, h->toff64.p, h->ntD.p, D64.p, h->doff64.p,
                                   status.p, h->jobs64.p, h->njobs64, 0.0, st));
      }
      auto stat = download(status.p, nsub, st);
      for (int j : f64list)
        if (stat[j]) fail(GENEO_ERR_LOCAL_NOT_SPD, "local Dirichlet matrix of subdomain " +
                                                       std::to_string(j) + " is not SPD");
      std::vector<int2> tj;
      for (int j : f64list)
        for (int c = 0; c < h->LD.nt[j]; ++c) tj.push_back(make_int2(j, c));
      DBuf<int2> tjobs;
      tjobs.upload(tj, st);
      h->X64.alloc(tt * TSQ);
      ProfScope ps("trtri_dirichlet", st, 2.0 * 8.0 * pk64, fl64);
      HIPCHK(launch_trtri(false, L64.p, D64.p, h->X64.p, h->toff64.p, h->doff64.p, h->ntD.p,
                          tjobs.p, (int)tj.size(), st));
      HIPCHK(hipStreamSynchronize(st));
    }
  }
  {
    double b32 = 0.0, b64 = 0.0;
    for (int j = 0; j < nsub; ++j) {
      bool is64 = std::find(f64list.begin(), f64list.end(), j) != f64list.end();
      double nn = h->nd_host[j];
      if (is64) b64 += 8.0 * packed(nn) + 16.0 * nn;
      else b32 += 4.0 * packed(nn) + 16.0 * nn;
    }
    h->bytes_trmv32 = b32;
    h->bytes_trmv64 = b64;
  }
  h->info.bytes_local_factors =
      (int64_t)(h->X32.p ? h->LD.ntiles * TSQ * 4 : 0) + (int64_t)h->X64.n * 8;
  phase(1);

  h->m_host.assign(nsub, 0);
  h->nc = 0;
  if (o.coarse) {
    if (!An || !Ao || !An->rowptr || !Ao->rowptr || !S->pou)
      fail(GENEO_ERR_ARG, "coarse space needs the Neumann and overlap matrices and the PoU");
    // ---- 2. shifted matrices C_j = A_N - sigma X A^o X and their Cholesky factors G_j
    LocalLayout LN;
    LN.build(h->nN_host);
    DBuf<int> ntN, voffN, jobsN;
    DBuf<int64_t> toffN, doffN;
    ntN.upload(LN.nt, st);
    voffN.upload(LN.voff, st);
    toffN.upload(LN.toff, st);
    doffN.upload(LN.doff, st);
    jobsN.upload(all, st);
    DBuf<double> G, DG;
    G.alloc(LN.ntiles * TSQ);
    DG.alloc(LN.ndiag * TSQ);
    double pkN = 0.0, flN = 0.0;
    for (int j = 0; j < nsub; ++j) {
      pkN += packed(h->nN_host[j]);
      flN += std::pow((double)h->nN_host[j], 3) / 3.0;
    }
    {
      ProfScope ps("densify_shifted", st, 8.0 * LN.ntiles * TSQ, 0.0);
      HIPCHK(launch_densify_shifted(G.p, toffN.p, ntN.p, nsub, S->sub_ptr, S->pou, An, Ao,
                                    o.sigma, st));
    }
    {
      ProfScope ps("chol_shifted_f64", st, 2.0 * 8.0 * pkN, flN);
      HIPCHK(launch_chol_batched(false, G.p, toffN.p, ntN.p, DG.p, doffN.p, status.p, jobsN.p,
                                 nsub, 0.0, st));
    }
    {
      auto stat = download(status.p, nsub, st);
      for (int j = 0; j < nsub; ++j)
        if (stat[j]) fail(GENEO_ERR_SHIFT_NOT_SPD, "A_N - sigma B of subdomain " +
                                                       std::to_string(j) + " is not SPD");
    }
    phase(2);

    // ---- 3. block subspace iteration on S = G^{-1} B G^{-T}
    const int want = o.tau > 0 ? o.nev_max : o.nev;
    int minnt = LN.nt[0];
    for (int j = 1; j < nsub; ++j) minnt = std::min(minnt, LN.nt[j]);
    int b = o.eig_block;
    if (b <= 0) {
      b = want + std::max(8, want / 2);
      b = ((b + 15) / 16) * 16;
    }
    b = std::min(b, 64);
    b = std::min(b, minnt * TS);
    if (b < 16 || b % 16 || want >= b)
      fail(GENEO_ERR_ARG, "eigen block size " + std::to_string(b) +
                              " cannot hold the requested eigenvectors");
    h->b = b;
    h->info.eig_block = b;
    DBuf<double> U, W, T, Y, theta, resid;
    DBuf<int> active, cnt;
    U.alloc(LN.nvec * b);
    W.alloc(LN.nvec * b);
    T.alloc(LN.nvec * b);
    Y.alloc(LN.nvec * b);
    theta.alloc((size_t)nsub * b);
    resid.alloc((size_t)nsub * b);
    active.alloc(nsub);
    cnt.alloc(1);
    HIPCHK(fill_i32(active.p, 1, nsub, st));
    HIPCHK(launch_eig_init(U.p, S->sub_ptr, voffN.p, ntN.p, nsub, b, o.seed, st));
    HIPCHK(launch_orth(U.p, voffN.p, ntN.p, S->sub_ptr, nsub, b, o.seed, 0, nullptr, st));
    int sweeps = 0, nact = nsub;
    std::vector<int> act(nsub, 1);
    for (int it = 1; it <= o.eig_maxit; ++it) {
      // algorithmic traffic of this sweep: the factor G_j of every active
      // subdomain is read once per triangular solve, plus its b columns
      double gb = 0.0, vb = 0.0, tf = 0.0;
      for (int j = 0; j < nsub; ++j) {
        if (!act[j]) continue;
        double nn = h->nN_host[j];
        gb += 8.0 * packed(nn);
        vb += 2.0 * 8.0 * nn * b;
        tf += 2.0 * packed(nn) * b;
      }
      {
        ProfScope ps("trsm_bwd", st, gb + vb, tf);
        HIPCHK(launch_trsm_bwd(G.p, DG.p, toffN.p, doffN.p, ntN.p, voffN.p, nsub, b, U.p, T.p,
                               active.p, st));
      }
      {
        ProfScope ps("bapply", st, vb, 0.0);
        HIPCHK(launch_bapply(S->sub_ptr, S->pou, Ao, voffN.p, ntN.p, nsub, b, T.p, W.p,
                             active.p, st));
      }
      {
        ProfScope ps("trsm_fwd", st, gb + vb, tf);
        HIPCHK(launch_trsm_fwd(G.p, DG.p, toffN.p, doffN.p, ntN.p, voffN.p, nsub, b, W.p, T.p,
                               active.p, st));
      }
      {
        ProfScope ps("rayleigh_ritz", st, 2.0 * vb, 0.0);
        HIPCHK(launch_rayleigh_ritz(U.p, T.p, Y.p, theta.p, resid.p, active.p, voffN.p, ntN.p,
                                    S->sub_ptr, nsub, b, o.nev, o.tau, o.nev_max, o.sigma,
                                    o.eig_tol, st));
      }
      sweeps = it;
      act = download(active.p, nsub, st);
      nact = 0;
      for (int j = 0; j < nsub; ++j) nact += act[j] != 0;
      if (nact == 0) break;
      {
        ProfScope ps("orth", st, 2.0 * vb, 0.0);
        HIPCHK(launch_orth(U.p, voffN.p, ntN.p, S->sub_ptr, nsub, b, o.seed, it, active.p, st));
      }
    }
    h->info.eig_sweeps = sweeps;
    if (nact > 0)
      fail(GENEO_ERR_EIGEN_NOCONV, std::to_string(nact) + " subdomains did not converge in " +
                                       std::to_string(o.eig_maxit) + " sweeps");
    // eigenvectors p = G^{-T} y
    HIPCHK(launch_trsm_bwd(G.p, DG.p, toffN.p, doffN.p, ntN.p, voffN.p, nsub, b, Y.p, T.p,
                           nullptr, st));
    DBuf<double> lam;
    lam.alloc((size_t)nsub * b);
    h->m.alloc(nsub);
    HIPCHK(launch_select(theta.p, nsub, b, o.nev, o.tau, o.nev_max, o.sigma, h->m.p, lam.p, st));
    h->m_host = download(h->m.p, nsub, st);
    h->lam_host = download(lam.p, (size_t)nsub * b, st);
    phase(3);

    // ---- 4. coarse basis Z, W = A_N Z, A_H = Z^T A Z
    std::vector<int> zoff(nsub), woff(nsub), coff(nsub + 1);
    int64_t zs = 0, ws = 0;
    int nc = 0;
    for (int j = 0; j < nsub; ++j) {
      zoff[j] = (int)zs;
      woff[j] = (int)ws;
      coff[j] = nc;
      zs += (int64_t)h->nd_host[j] * h->m_host[j];
      ws += (int64_t)h->nN_host[j] * h->m_host[j];
      nc += h->m_host[j];
    }
    coff[nsub] = nc;
    h->nc = nc;
    h->zoff.upload(zoff, st);
    h->coff.upload(coff, st);
    h->Z.alloc(zs);
    HIPCHK(launch_basis(T.p, voffN.p, b, S->sub_ptr, S->pou, h->dmap.p, h->m.p, h->zoff.p,
                        h->nd.p, nsub, h->Z.p, st));
    {
      DBuf<double> mr;
      mr.alloc(1);
      hipLaunchKernelGGL(k_max_resid, dim3(1), dim3(1), 0, st, resid.p, h->m.p, nsub, b, mr.p);
      h->info.eig_max_resid = download(mr.p, 1, st)[0];
    }
    HIPCHK(hipStreamSynchronize(st));
    if (nc > 0) {
      DBuf<int> woffd;
      woffd.upload(woff, st);
      DBuf<double> Wg;
      Wg.alloc(ws);
      HIPCHK(launch_galerkin_w(An, S->sub_ptr, h->dmap.p, h->Z.p, h->zoff.p, h->m.p, woffd.p,
                               nsub, Wg.p, st));
      DBuf<uint8_t> adj;
      adj.alloc((size_t)nsub * nsub);
      HIPCHK(launch_adjacency(h->optr.p, h->olist.p, h->n, nsub, adj.p, st));
      DBuf<int> pcnt, poff, npairs;
      pcnt.alloc(nsub);
      poff.alloc(nsub + 1);
      npairs.alloc(1);
      HIPCHK(launch_pairs(adj.p, nsub, pcnt.p, poff.p, nullptr, npairs.p, st, true));
      int np = download(npairs.p, 1, st)[0];
      DBuf<int2> pairs;
      pairs.alloc(np);
      HIPCHK(launch_pairs(adj.p, nsub, pcnt.p, poff.p, pairs.p, npairs.p, st, false));
      h->ntc = (nc + TS - 1) / TS;
      DBuf<double> AHt, DH;
      AHt.alloc(tri_tiles(h->ntc) * TSQ);
      DH.alloc((size_t)h->ntc * TSQ);
      HIPCHK(launch_coarse_init(AHt.p, h->ntc, nc, st));
      HIPCHK(launch_coarse_blocks(pairs.p, np, S->sub_ptr, S->sub_idx, h->didx.p, h->voffD.p,
                                  h->nd.p, h->Z.p, h->zoff.p, Wg.p, woffd.p, h->m.p, h->coff.p,
                                  AHt.p, st));
      h->AHdense.alloc((size_t)nc * nc);
      HIPCHK(launch_coarse_to_dense(AHt.p, h->ntc, nc, h->AHdense.p, st));
      phase(4);
      // ---- 5. coarse Cholesky and inverse factor
      DBuf<int> cst;
      cst.alloc(1);
      {
        ProfScope ps("coarse_chol", st, 8.0 * packed(nc), std::pow((double)nc, 3) / 3.0);
        HIPCHK(coarse_cholesky(AHt.p, DH.p, h->ntc, cst.p, st));
      }
      if (download(cst.p, 1, st)[0]) fail(GENEO_ERR_COARSE_NOT_SPD, "coarse matrix A_H is not SPD");
      h->hjob.upload(std::vector<int>{0}, st);
      h->hnt.upload(std::vector<int>{h->ntc}, st);
      h->hvoff.upload(std::vector<int>{0}, st);
      h->htoff.upload(std::vector<int64_t>{0}, st);
      DBuf<int64_t> hdoff;
      hdoff.upload(std::vector<int64_t>{0}, st);
      std::vector<int2> tj;
      for (int c = 0; c < h->ntc; ++c) tj.push_back(make_int2(0, c));
      DBuf<int2> tjobs;
      tjobs.upload(tj, st);
      h->XH.alloc(tri_tiles(h->ntc) * TSQ);
      HIPCHK(launch_trtri(false, AHt.p, DH.p, h->XH.p, h->htoff.p, hdoff.p, h->hnt.p, tjobs.p,
                          h->ntc, st));
      h->rH.alloc((size_t)h->ntc * TS);
      h->tH.alloc((size_t)h->ntc * TS);
      h->yH.alloc((size_t)h->ntc * TS);
      HIPCHK(hipMemsetAsync(h->rH.p, 0, h->rH.n * sizeof(double), st));
      HIPCHK(hipStreamSynchronize(st));
      phase(5);
    }
  }
  if (h->nc == 0) {
    // placeholders so that the apply kernels always get valid pointers
    if (!h->m.p) h->m.upload(std::vector<int>(nsub, 0), st);
    if (!h->zoff.p) h->zoff.upload(std::vector<int>(nsub, 0), st);
    if (!h->coff.p) h->coff.upload(std::vector<int>(nsub + 1, 0), st);
    if (!h->Z.p) h->Z.alloc(1);
    h->yH.alloc(1);
  }
  h->xl.alloc(h->LD.nvec);
  h->tl.alloc(h->LD.nvec);
  h->yl.alloc(h->LD.nvec);
  HIPCHK(hipStreamSynchronize(st));
  h->info.nsub = nsub;
  h->info.nc = h->nc;
  h->info.t_setup_ms = now_ms() - t_start;
}

void ensure_pcg(geneo_handle_s* h, int maxit) {
  if (h->pcg_cap < h->n) {
    h->r.alloc(h->n);
    h->z.alloc(h->n);
    h->p.alloc(h->n);
    h->q.alloc(h->n);
    h->partial.alloc(PCG_NB);
    h->sc.alloc(1);
    h->done.alloc(1);
    h->pcg_cap = h->n;
  }
  if (h->pcg_maxit < maxit + 1) {
    h->alphas.alloc(maxit + 1);
    h->betas.alloc(maxit + 1);
    h->pcg_maxit = maxit + 1;
  }
}

#define PCG_CHUNK 8

void pcg_one(geneo_handle_s* h, const geneo_csr_t* A, const double* b, double* x, double rtol,
             int maxit, geneo_pcg_info_t* info) {
  hipStream_t st = h->hs;
  const int n = h->n;
  double t0 = now_ms();
  // start: r = b - A x, z = M^{-1} r, p = z
  PcgScalars init{};
  init.maxit = maxit;
  HIPCHK(hipMemcpyAsync(h->sc.p, &init, sizeof(init), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(fill_i32(h->done.p, 0, 1, st));
  HIPCHK(dot_partial(b, b, n, h->partial.p, nullptr, st));
  HIPCHK(scalar_stage(h->partial.p, 3, h->sc.p, h->done.p, h->alphas.p, h->betas.p, st));
  auto sc0 = download(h->sc.p, 1, st)[0];
  const double bb = sc0.rz;
  init.tol2 = rtol * rtol * bb;
  HIPCHK(hipMemcpyAsync(h->sc.p, &init, sizeof(init), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(spmv(A, x, h->q.p, h->lpr, nullptr, st));
  HIPCHK(residual0(b, h->q.p, h->r.p, n, st));
  HIPCHK(dot_partial(h->r.p, h->r.p, n, h->partial.p, nullptr, st));
  HIPCHK(scalar_stage(h->partial.p, 3, h->sc.p, h->done.p, h->alphas.p, h->betas.p, st));
  double rr0 = download(h->sc.p, 1, st)[0].rz;
  int iters = 0, converged = 0;
  double rr = rr0;
  if (bb == 0.0 || rr0 <= init.tol2) {
    converged = 1;
  } else {
    HIPCHK(apply_enqueue(h, h->r.p, h->z.p, nullptr, st));
    HIPCHK(copy_vec(h->z.p, h->p.p, n, st));
    HIPCHK(dot_partial(h->r.p, h->z.p, n, h->partial.p, nullptr, st));
    HIPCHK(scalar_stage(h->partial.p, 3, h->sc.p, h->done.p, h->alphas.p, h->betas.p, st));
    // capture PCG_CHUNK iterations
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < PCG_CHUNK; ++k) {
      HIPCHK(spmv(A, h->p.p, h->q.p, h->lpr, h->done.p, st));
      HIPCHK(dot_partial(h->p.p, h->q.p, n, h->partial.p, h->done.p, st));
      HIPCHK(scalar_stage(h->partial.p, 0, h->sc.p, h->done.p, h->alphas.p, h->betas.p, st));
      HIPCHK(update_xr(x, h->r.p, h->p.p, h->q.p, n, h->sc.p, h->partial.p, h->done.p, st));
      HIPCHK(scalar_stage(h->partial.p, 1, h->sc.p, h->done.p, h->alphas.p, h->betas.p, st));
      HIPCHK(apply_enqueue(h, h->r.p, h->z.p, h->done.p, st));
      HIPCHK(dot_partial(h->r.p, h->z.p, n, h->partial.p, h->done.p, st));
      HIPCHK(scalar_stage(h->partial.p, 2, h->sc.p, h->done.p, h->alphas.p, h->betas.p, st));
      HIPCHK(update_p(h->p.p, h->z.p, n, h->sc.p, h->done.p, st));
    }
    HIPCHK(hipStreamEndCapture(st, &graph));
    HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    int dn = 0;
    for (int rep = 0; rep * PCG_CHUNK < maxit + PCG_CHUNK; ++rep) {
      HIPCHK(hipGraphLaunch(exec, st));
      dn = download(h->done.p, 1, st)[0];
      if (dn) break;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    PcgScalars s = download(h->sc.p, 1, st)[0];
    iters = s.iters;
    converged = s.converged;
    rr = s.rr;
  }
  info->iters = iters;
  info->converged = converged;
  info->relres = bb > 0 ? sqrt(rr / bb) : 0.0;
  info->kappa_est = 1.0;
  if (iters > 0) {
    auto al = download(h->alphas.p, iters, st);
    auto be = download(h->betas.p, std::max(iters - 1, 1), st);
    std::vector<double> d(iters), e(iters > 1 ? iters - 1 : 0);
    for (int i = 0; i < iters; ++i) {
      d[i] = 1.0 / al[i] + (i > 0 ? be[i - 1] / al[i - 1] : 0.0);
      if (i + 1 < iters) e[i] = sqrt(be[i]) / al[i];
    }
    double lmin = tridiag_eig(d, e, 0), lmax = tridiag_eig(d, e, iters - 1);
    info->kappa_est = lmin > 0 ? lmax / lmin : INFINITY;
  }
  info->t_solve_ms = now_ms() - t0;
}

int finish(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char* geneo_strerror(int code) {
  switch (code) {
    case GENEO_OK: return "ok";
    case GENEO_ERR_ARG: return "invalid argument";
    case GENEO_ERR_OOM: return "device out of memory";
    case GENEO_ERR_LOCAL_NOT_SPD: return "local Dirichlet matrix not SPD";
    case GENEO_ERR_EIGEN_NOCONV: return "eigen sweeps did not converge";
    case GENEO_ERR_COARSE_NOT_SPD: return "coarse matrix not SPD";
    case GENEO_ERR_MAXIT: return "PCG reached maxit";
    case GENEO_ERR_HIP: return "HIP runtime error";
    case GENEO_ERR_SHIFT_NOT_SPD: return "shifted local matrix not SPD";
    default: return "unknown error";
  }
}

const char* geneo_last_error(void) { return g_last_error.c_str(); }

const char* geneo_version(void) { return "geneo 0.1 gfx950"; }

void geneo_default_opts(geneo_opts_t* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->nev = 8;
  o->tau = 0.0;
  o->nev_max = 16;
  o->sigma = -1e-3;
  o->precision = GENEO_PREC_FP64;
  o->pivot_tol = 1e-3;
  o->eig_tol = 1e-10;
  o->eig_maxit = 300;
  o->eig_block = 0;
  o->seed = 0;
  o->coarse = 1;
}

int geneo_q1_sizes(const geneo_grid_t* grid, geneo_q1_sizes_t* sizes) {
  if (!sizes) return finish(GENEO_ERR_ARG, "sizes is NULL");
  Q1Geom g;
  std::string err;
  int rc = q1_make_geom(grid, &g, &err);
  if (rc) return finish(rc, err);
  q1_sizes(g, sizes);
  if (sizes->nnz >= (1ll << 31) || sizes->nnz_loc >= (1ll << 31) || sizes->ndof >= (1ll << 31))
    return finish(GENEO_ERR_ARG, "problem exceeds 32-bit indexing");
  return GENEO_OK;
}

int geneo_assemble_q1(const geneo_grid_t* grid, const double* coeff, int* A_rowptr, int* A_col,
                      double* A_val, double* b, int* sub_ptr, int* sub_idx, uint8_t* sub_flags,
                      double* pou, int* loc_rowptr, int* loc_col, double* an_val, double* ao_val,
                      void* stream) {
  try {
    Q1Geom g;
    std::string err;
    int rc = q1_make_geom(grid, &g, &err);
    if (rc) fail(rc, err);
    if (!coeff || !A_rowptr || !A_col || !A_val || !b || !sub_ptr || !sub_idx || !sub_flags ||
        !pou || !loc_rowptr || !loc_col || !an_val || !ao_val)
      fail(GENEO_ERR_ARG, "NULL output array");
    geneo_q1_sizes_t s;
    q1_sizes(g, &s);
    hipStream_t st = (hipStream_t)stream;
    DBuf<Q1Geom> dg;
    dg.alloc(1);
    HIPCHK(hipMemcpyAsync(dg.p, &g, sizeof(g), hipMemcpyHostToDevice, st));
    DBuf<int64_t> nzoff;
    nzoff.alloc(g.nsub + 1);
    HIPCHK(q1_launch_all(dg.p, g, s, coeff, A_rowptr, A_col, A_val, b, sub_ptr, sub_idx, sub_flags,
                         pou, loc_rowptr, loc_col, an_val, ao_val, nzoff.p, st));
    HIPCHK(hipStreamSynchronize(st));
    return GENEO_OK;
  } catch (Err& e) {
    return finish(e.code, e.msg);
  }
}

int geneo_setup(const geneo_csr_t* A, const geneo_subdomains_t* S, const geneo_csr_batch_t* An,
                const geneo_csr_batch_t* Ao, const geneo_opts_t* opts, void* stream,
                geneo_handle_t* out) {
  if (!out) return finish(GENEO_ERR_ARG, "out is NULL");
  *out = nullptr;
  try {
    check_csr(A);
    if (!S || S->nsub <= 0 || !S->sub_ptr || !S->sub_idx || !S->sub_flags || S->nloc <= 0)
      fail(GENEO_ERR_ARG, "invalid subdomain lists");
    std::unique_ptr<geneo_handle_s> h(new geneo_handle_s());
    if (opts) h->opts = *opts;
    else geneo_default_opts(&h->opts);
    const geneo_opts_t& o = h->opts;
    if (!(o.sigma < 0)) fail(GENEO_ERR_ARG, "sigma must be negative");
    if (o.precision != GENEO_PREC_FP64 && o.precision != GENEO_PREC_MIXED)
      fail(GENEO_ERR_ARG, "unknown precision mode");
    if (o.coarse && (o.tau > 0 ? o.nev_max < 1 : o.nev < 0))
      fail(GENEO_ERR_ARG, "invalid eigenvector count");
    if (o.eig_block && (o.eig_block % 16 || o.eig_block > 64))
      fail(GENEO_ERR_ARG, "eig_block must be a multiple of 16 up to 64");
    if (o.eig_maxit < 1 || !(o.eig_tol > 0)) fail(GENEO_ERR_ARG, "invalid eigen tolerances");
    setup_impl(h.get(), A, S, An, Ao, (hipStream_t)stream);
    *out = h.release();
    return GENEO_OK;
  } catch (Err& e) {
    return finish(e.code, e.msg);
  }
}

int geneo_apply(geneo_handle_t h, const double* r, double* z, void* stream) {
  if (!h || !r || !z || r == z) return finish(GENEO_ERR_ARG, "invalid apply arguments");
  hipError_t e = apply_enqueue(h, r, z, nullptr, (hipStream_t)stream);
  if (e != hipSuccess) return finish(GENEO_ERR_HIP, hipGetErrorString(e));
  return GENEO_OK;
}

void geneo_destroy(geneo_handle_t h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  delete h;
}

int geneo_get_setup_info(geneo_handle_t h, geneo_setup_info_t* info) {
  if (!h || !info) return finish(GENEO_ERR_ARG, "NULL argument");
  *info = h->info;
  return GENEO_OK;
}

int geneo_get_eigenvalues(geneo_handle_t h, int* m, double* lam, int ldl) {
  if (!h || !m || !lam || ldl < 1) return finish(GENEO_ERR_ARG, "NULL argument");
  for (int j = 0; j < h->nsub; ++j) {
    m[j] = h->m_host[j];
    for (int c = 0; c < ldl; ++c)
      lam[(int64_t)j * ldl + c] = (c < h->b && !h->lam_host.empty())
                                      ? h->lam_host[(int64_t)j * h->b + c]
                                      : INFINITY;
  }
  return GENEO_OK;
}

int geneo_get_coarse(geneo_handle_t h, int* zoff, double* z, int64_t zsize, double* ah) {
  if (!h || !zoff) return finish(GENEO_ERR_ARG, "NULL argument");
  try {
    hipStream_t st = h->hs;
    int64_t tot = 0;
    for (int j = 0; j < h->nsub; ++j) {
      zoff[j] = (int)tot;
      tot += (int64_t)h->nN_host[j] * h->m_host[j];
    }
    zoff[h->nsub] = (int)tot;
    if (z) {
      if (zsize < tot) fail(GENEO_ERR_ARG, "z buffer too small");
      std::vector<double> zin;
      if (h->nc > 0) {
        int64_t zs = 0;
        for (int j = 0; j < h->nsub; ++j) zs += (int64_t)h->nd_host[j] * h->m_host[j];
        zin = download(h->Z.p, zs, st);
      }
      auto dm = download(h->dmap.p, h->nloc, st);
      int64_t zi = 0;
      for (int j = 0; j < h->nsub; ++j) {
        int mj = h->m_host[j];
        for (int a = 0; a < h->nN_host[j]; ++a) {
          int d = dm[h->sub_ptr_host[j] + a];
          for (int c = 0; c < mj; ++c)
            z[zoff[j] + (int64_t)a * mj + c] = d >= 0 ? zin[zi + (int64_t)d * mj + c] : 0.0;
        }
        zi += (int64_t)h->nd_host[j] * mj;
      }
    }
    if (ah && h->nc > 0) {
      auto v = download(h->AHdense.p, (size_t)h->nc * h->nc, st);
      memcpy(ah, v.data(), v.size() * sizeof(double));
    }
    return GENEO_OK;
  } catch (Err& e) {
    return finish(e.code, e.msg);
  }
}

int pcg_solve(const geneo_csr_t* A, geneo_handle_t h, const double* b, double* x, int nrhs,
              double rtol, int maxit, geneo_pcg_info_t* info, void* stream) {
  try {
    check_csr(A);
    if (!h || !b || !x || !info || nrhs < 1 || maxit < 1 || !(rtol > 0))
      fail(GENEO_ERR_ARG, "invalid pcg arguments");
    if (A->n != h->n) fail(GENEO_ERR_ARG, "matrix size differs from the preconditioner's");
    hipStream_t us = (hipStream_t)stream;
    ensure_pcg(h, maxit);
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, us));
    HIPCHK(hipStreamWaitEvent(h->hs, ev, 0));
    int rc = GENEO_OK;
    for (int k = 0; k < nrhs; ++k) {
      pcg_one(h, A, b + (int64_t)k * h->n, x + (int64_t)k * h->n, rtol, maxit, &info[k]);
      if (!info[k].converged) rc = GENEO_ERR_MAXIT;
    }
    HIPCHK(hipEventRecord(ev, h->hs));
    HIPCHK(hipStreamWaitEvent(us, ev, 0));
    HIPCHK(hipEventDestroy(ev));
    if (rc) return finish(rc, "PCG did not converge within maxit");
    return GENEO_OK;
  } catch (Err& e) {
    return finish(e.code, e.msg);
  }
}

int geneo_spmv(const geneo_csr_t* A, const double* x, double* y, void* stream) {
  try {
    check_csr(A);
    if (!x || !y) fail(GENEO_ERR_ARG, "NULL vector");
    HIPCHK(spmv(A, x, y, spmv_lanes(A), nullptr, (hipStream_t)stream));
    return GENEO_OK;
  } catch (Err& e) {
    return finish(e.code, e.msg);
  }
}

}  // extern "C"
