// C ABI of libgeneo: argument checks, buffer ownership and the order of the
// setup phases, the preconditioner apply and the graph-captured PCG loop.
#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <mutex>
#include <thread>
#include <shared_mutex>
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

// Graph captures against device-wide synchronisation.  A device-wide
// synchronisation, or a driver allocation or free (which may synchronise),
// in one thread invalidates a stream capture running in another.  Captures
// hold this lock shared; those calls hold it exclusively (re-entrant within
// a thread, so nested uses do not deadlock).
std::shared_mutex g_capture_mu;
thread_local int t_driver_depth = 0;
struct DriverLock {
  DriverLock() {
    if (t_driver_depth++ == 0) g_capture_mu.lock();
  }
  ~DriverLock() {
    if (--t_driver_depth == 0) g_capture_mu.unlock();
  }
  DriverLock(const DriverLock&) = delete;
  DriverLock& operator=(const DriverLock&) = delete;
};

// Pinned host staging for the small uploads of a setup (index lists, job
// lists, offsets), so that they are asynchronous: one arena per host
// thread, reused by consecutive setups of that thread.  A setup resets it
// at the start; every copy that reads it has completed by then, since each
// setup ends (also on failure) with the device synchronised.
struct PinnedArena {
  std::vector<std::pair<char*, size_t>> chunks;
  size_t chunk = 0, used = 0;
  bool active = false;
  void begin() {
    chunk = used = 0;
    active = true;
  }
  void end() { active = false; }
  void* take(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    while (chunk < chunks.size() && used + bytes > chunks[chunk].second) {
      ++chunk;
      used = 0;
    }
    if (chunk == chunks.size()) {
      const size_t cap = std::max(bytes, (size_t)4 << 20);
      char* p = nullptr;
      DriverLock dl;
      if (hipHostMalloc((void**)&p, cap, hipHostMallocDefault) != hipSuccess) return nullptr;
      chunks.push_back({p, cap});
      used = 0;
    }
    void* r = chunks[chunk].first + used;
    used += bytes;
    return r;
  }
  ~PinnedArena() {
    if (chunks.empty()) return;
    DriverLock dl;
    for (auto& c : chunks) (void)hipHostFree(c.first);
  }
};
thread_local PinnedArena t_arena;

// Small pinned host blocks that outlive their handles: a destroyed handle
// returns its blocks here for the next one, and none is ever freed, since
// freeing pinned memory synchronises the device (and would break a graph
// capture running in another thread).
class PinnedPool {
 public:
  static PinnedPool& get() {
    static PinnedPool* p = new PinnedPool();  // never destroyed
    return *p;
  }
  // a block of at least `bytes` (power-of-two size class, 256 B minimum)
  void* take(size_t bytes) {
    size_t cls = 256;
    while (cls < bytes) cls <<= 1;
    {
      std::lock_guard<std::mutex> g(mu_);
      auto& fl = free_[cls];
      if (!fl.empty()) {
        void* q = fl.back();
        fl.pop_back();
        return q;
      }
    }
    void* q = nullptr;
    {
      DriverLock dl;
      if (hipHostMalloc(&q, cls, hipHostMallocDefault) != hipSuccess) return nullptr;
    }
    std::lock_guard<std::mutex> g(mu_);
    size_[q] = cls;
    return q;
  }
  void give(void* q) {
    if (!q) return;
    std::lock_guard<std::mutex> g(mu_);
    free_[size_[q]].push_back(q);
  }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void*>> free_;
  std::map<void*, size_t> size_;
};

// Device blocks of the library, kept for reuse: a setup of the same shape
// as an earlier one then takes its buffers from here instead of the driver
// (whose allocations, and frees, cost milliseconds each at these sizes and
// whose frees synchronise the device).  A released block goes to a pending
// list of the releasing thread and becomes reusable at settle_thread(),
// which that thread calls once it has synchronised every stream its work
// on the block was enqueued on (each entry point releases buffers only
// after that): no kernel that used the block can still be running, and no
// other thread's work is waited for.  Reuse takes the smallest free block
// of at least the request and at most 1/8 larger.  At most kCacheMax free
// bytes are kept per device; trim() hands all free blocks back (also done,
// with one retry, when the driver reports out of memory).
class DevCache {
 public:
  static constexpr size_t kCacheMax = (size_t)64 << 30;
  static DevCache& get() {
    static DevCache* c = new DevCache;  // never destroyed: no frees at exit
    return *c;
  }
  hipError_t alloc(void** p, size_t bytes, int* dev) {
    HIPCHK(hipGetDevice(dev));
    {
      std::lock_guard<std::mutex> g(mu_);
      auto& f = pools_[*dev].free;
      auto it = f.lower_bound(bytes);
      if (it != f.end() && it->first <= bytes + bytes / 8) {
        *p = it->second;
        sizes_[*p] = it->first;
        pools_[*dev].free_bytes -= it->first;
        f.erase(it);
        return hipSuccess;
      }
    }
    DriverLock dl;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      trim(*dev);
      e = hipMalloc(p, bytes);
    }
    if (e == hipSuccess) {
      std::lock_guard<std::mutex> g(mu_);
      sizes_[*p] = bytes;
    }
    return e;
  }
  void release(void* p, int dev) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = sizes_.find(p);
    const size_t bytes = it != sizes_.end() ? it->second : 0;
    if (it != sizes_.end()) sizes_.erase(it);
    pools_[dev].pending[std::this_thread::get_id()].push_back({bytes, p});
  }
  // The calling thread has synchronised the streams of the work on the
  // blocks it released: they become reusable.
  void settle_thread(int dev) {
    std::vector<void*> drop;
    {
      std::lock_guard<std::mutex> g(mu_);
      Pool& pl = pools_[dev];
      auto it = pl.pending.find(std::this_thread::get_id());
      if (it == pl.pending.end()) return;
      for (auto& b : it->second) {
        pl.free.insert(b);
        pl.free_bytes += b.first;
      }
      pl.pending.erase(it);
      while (pl.free_bytes > kCacheMax && !pl.free.empty()) {
        auto f = std::prev(pl.free.end());
        pl.free_bytes -= f->first;
        drop.push_back(f->second);
        pl.free.erase(f);
      }
    }
    if (drop.empty()) return;
    DriverLock dl;  // hipFree synchronises the device
    for (void* q : drop) (void)hipFree(q);
  }
  void trim(int dev) {
    DriverLock dl;
    std::vector<void*> drop;
    {
      std::lock_guard<std::mutex> g(mu_);
      Pool& pl = pools_[dev];
      for (auto& b : pl.free) drop.push_back(b.second);
      pl.free.clear();
      pl.free_bytes = 0;
    }
    for (void* q : drop) (void)hipFree(q);
  }
  size_t free_bytes(int dev) {
    std::lock_guard<std::mutex> g(mu_);
    return pools_[dev].free_bytes;
  }

 private:
  struct Pool {
    std::multimap<size_t, void*> free;
    std::map<std::thread::id, std::vector<std::pair<size_t, void*>>> pending;
    size_t free_bytes = 0;
  };
  std::mutex mu_;
  std::map<int, Pool> pools_;
  std::map<void*, size_t> sizes_;
};

// The calling thread's released blocks on the current device become
// reusable (its streams have been synchronised).
void settle_thread() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  DevCache::get().settle_thread(dev);
}

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  int dev = 0;
  void alloc(size_t cnt) {
    release();
    if (cnt == 0) cnt = 1;
    void* q = nullptr;
    HIPCHK(DevCache::get().alloc(&q, cnt * sizeof(T), &dev));
    p = (T*)q;
    n = cnt;
  }
  void release() {
    if (p) DevCache::get().release(p, dev);
    p = nullptr;
    n = 0;
  }
  // Copies v to a fresh device buffer on stream st: through the pinned
  // arena without waiting when a setup is running, else synchronously.
  void upload(const std::vector<T>& v, hipStream_t st) {
    alloc(v.size());
    if (v.empty()) return;
    const size_t bytes = v.size() * sizeof(T);
    void* stage = t_arena.active ? t_arena.take(bytes) : nullptr;
    if (stage) {
      memcpy(stage, v.data(), bytes);
      HIPCHK(hipMemcpyAsync(p, stage, bytes, hipMemcpyHostToDevice, st));
    } else {
      HIPCHK(hipMemcpyAsync(p, v.data(), bytes, hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
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

// extreme eigenvalues of a symmetric tridiagonal matrix (diagonal d[0..n),
// off-diagonal e[0..n-1)) by Sturm bisection
int sturm_count(const double* d, const double* e, int n, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < n; ++i) {
    double off = i ? e[i - 1] * e[i - 1] : 0.0;
    q = d[i] - x - (i ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

double tridiag_eig(const double* d, const double* e, int n, int k) {
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    double r = (i ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (sturm_count(d, e, n, mid) > k) hi = mid;
    else lo = mid;
    if (hi - lo <= 1e-14 * std::max(fabs(lo), fabs(hi))) break;
  }
  return 0.5 * (lo + hi);
}

double packed(double n) { return n * (n + 1.0) * 0.5; }

// Work inside tile envelopes (host copy E of the first nonzero tile column
// per tile row, at the diagonal tile offsets doff): per matrix the stored
// tiles, and over all matrices the tile products of a left-looking
// Cholesky, sum over the envelope tiles (i, k) of k - E(i).  Used for the
// algorithmic bytes and flops of the kernels that skip the zero tiles.
struct EnvWork {
  std::vector<double> tiles;  // per matrix (0 for matrices not listed)
  double prods = 0.0;         // Cholesky tile products
  double inv_prods = 0.0;     // tile products of X = L^{-1} (sum over the
                              // tiles (i, c) of i - max(E(i), c))
};
EnvWork env_work(const std::vector<int>& E, const std::vector<int64_t>& doff,
                 const std::vector<int>& nt, const std::vector<int>& jobs) {
  EnvWork w;
  w.tiles.assign(nt.size(), 0.0);
  for (int j : jobs)
    for (int i = 0; i < nt[j]; ++i) {
      const double e = E[doff[j] + i], width = i - e + 1;
      w.tiles[j] += width;
      w.prods += width * (width - 1.0) * 0.5;
      w.inv_prods += (e + 1.0) * (i - e) + (i - e - 1.0) * (i - e) * 0.5;
    }
  return w;
}

}  // namespace

// Kernels of the eigen sweeps' triangular solves (see tune_trsm).
struct TrsmChoice {
  int variant = 0, split_variant = 0, split_limit = 0;
};

struct geneo_handle_s {
  int n = 0, nsub = 0;
  int64_t nloc = 0;
  geneo_opts_t opts{};
  hipStream_t hs = nullptr;
  hipEvent_t shifted_done = nullptr, f32_done = nullptr;
  LocalLayout LD;
  DBuf<int> sub_ptr, sub_idx, dmap, nd, ntD, voffD, dglob, didx, jobs32, jobs64;
  DBuf<int64_t> toffD, doffD, toff64, doff64;
  DBuf<double> dscale;
  // Cholesky factors of the scaled local Dirichlet matrices (packed tiles)
  // with their inverted diagonal tiles and tile envelopes: FP32, and FP64
  // for the subdomains in f64list (tiles at toff64 / doff64)
  DBuf<float> L32, D32;
  DBuf<double> L64, D64;
  DBuf<int> envDE, envDR, env64E, env64R;
  // the envelopes the factorisations and solves use (NULL: dense, option
  // envelope = 0)
  const int *uDE = nullptr, *uDR = nullptr, *u64E = nullptr, *u64R = nullptr;
  // local solves of the apply: GENEO_LOCAL_TRIANGULAR (the factors above)
  // or GENEO_LOCAL_INVERSE (symmetric inverses A_j^{-1} in S32 / S64, FP32
  // / FP64 subdomains, with the partial sums of their products in W32 / W64)
  int local_form = GENEO_LOCAL_TRIANGULAR;
  DBuf<float> S32, W32;
  DBuf<double> S64, W64;
  int njobs32 = 0, njobs64 = 0;
  DBuf<int> optr;
  DBuf<int2> olist;
  DBuf<int4> oent;  // owner entries resolved for the combine
  // coarse space
  int nc = 0, ntc = 0, b = 0;
  DBuf<int> m, zoff, coff, hnt;
  DBuf<double> tau_sub;  // per-subdomain thresholds (opts.tau_sub), else empty
  TrsmChoice trsm;  // kernels of the eigen sweeps' triangular solves
  // job list of the coarse symmetric product: (nsub, 2) for the coarse
  // inverse when there is a coarse space
  DBuf<int2> ajobs;
  // subdomains of the triangular local solves with FP32 and FP64 factors
  DBuf<int> lsj32, lsj64;
  int nlsj32 = 0, nlsj64 = 0;
  DBuf<double> rz_part, rr_part;  // PCG partial sums: r.z per 256 rows, r.r per PCG block
  std::vector<int2> ljobs_host;
  int najobs = 0, amaxnt = 0;
  bool apply_rev = false;  // direction of the next standalone apply
  DBuf<SymvTask> tasks_fwd, tasks_rev;  // symmetric-product tasks, both walk orders
  DBuf<SymvJob> symv_jobs;              // their per-matrix descriptors
  DBuf<int> cstart;        // first row chunk per tile row; row partials per job
  DBuf<double> Rpart;
  int nchunk = 0, ntasks = 0;
  std::vector<int64_t> toff64_host, doff64_host;
  DBuf<int64_t> htoff;
  DBuf<double> Z, SH, WH, rH, yH, AHdense;
  std::vector<int> m_host, nd_host, nN_host, sub_ptr_host;
  std::vector<double> lam_host;
  // apply workspace
  DBuf<double> xl, yl;
  // pcg workspace
  int pcg_cap = 0, pcg_maxit = 0;
  DBuf<double> r, z, p, p2, q, partial, alphas, betas;
  // the iterate of the captured PCG graphs (the caller's x is copied in and
  // out, so the graphs serve every solve) and the refinement residual
  DBuf<double> xs, rb;
  // captured graphs of PCG_CHUNK and PCG_TAIL iterations, reused while the
  // matrix and the work buffers they were captured with stay the same
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  const void* gkey[6] = {};
  DBuf<PcgScalars> sc;
  DBuf<int> done;
  int lpr = 8;
  // algorithmic bytes per apply: local solves (either form), coarse product
  double bytes_local = 0.0, bytes_symvH = 0.0;
  std::vector<int> f64list;                         // subdomains with FP64 local factors
  geneo_setup_info_t info{};
  // pinned host words of the PCG loop: done flags of two chunks, scalars
  int* hflag = nullptr;
  PcgScalars* hsc = nullptr;  // two chunk slots and the final read
  double* hab = nullptr;  // alphas then betas, pcg_maxit each
  hipEvent_t fev[2] = {nullptr, nullptr};
  std::map<hipStream_t, hipEvent_t> apply_ev;  // last geneo_apply per stream
  ~geneo_handle_s() {
    for (auto& se : apply_ev) (void)hipEventDestroy(se.second);
    for (hipGraphExec_t e : gexec)
      if (e) (void)hipGraphExecDestroy(e);
    PinnedPool::get().give(hflag);
    PinnedPool::get().give(hab);
    PinnedPool::get().give(hsc);
    for (hipEvent_t e : fev)
      if (e) (void)hipEventDestroy(e);
    if (shifted_done) (void)hipEventDestroy(shifted_done);
    if (f32_done) (void)hipEventDestroy(f32_done);
    if (hs) (void)hipStreamDestroy(hs);
  }
};

namespace {

void check_csr(const geneo_csr_t* A) {
  if (!A || A->n <= 0 || !A->rowptr || !A->col || !A->val || A->nnz <= 0)
    fail(GENEO_ERR_ARG, "invalid CSR matrix");
}

// Arguments of the symmetric products of the apply (rev: reverse walk):
// the coarse inverse, and the local inverses in the inverse form.
SymvArgs symv_args(const geneo_handle_s* h, bool rev) {
  SymvArgs sa;
  sa.S32 = h->S32.p;
  sa.S64 = h->S64.p;
  sa.toff32 = h->toffD.p;
  sa.toff64 = h->toff64.p;
  sa.nt = h->ntD.p;
  sa.voff = h->voffD.p;
  sa.jobs = h->ajobs.p;
  sa.njobs = h->najobs;
  sa.maxnt = h->amaxnt;
  sa.SH = h->SH.p;
  sa.ntc = h->ntc;
  sa.W32 = h->W32.p;
  sa.W64 = h->W64.p;
  sa.WH = h->WH.p;
  sa.x = h->xl.p;
  sa.y = h->yl.p;
  sa.xH = h->rH.p;
  sa.yH = h->yH.p;
  sa.tasks = rev ? h->tasks_rev.p : h->tasks_fwd.p;
  sa.ntasks = h->ntasks;
  sa.cstart = h->cstart.p;
  sa.nchunk = h->nchunk;
  sa.R = h->Rpart.p;
  return sa;
}

// Arguments of the local solves of the apply.
LocalSolveArgs local_solve_args(const geneo_handle_s* h) {
  LocalSolveArgs a;
  a.L32 = h->L32.p;
  a.D32 = h->D32.p;
  a.L64 = h->L64.p;
  a.D64 = h->D64.p;
  a.toff32 = h->toffD.p;
  a.doff32 = h->doffD.p;
  a.toff64 = h->toff64.p;
  a.doff64 = h->doff64.p;
  a.E32 = h->uDE;
  a.R32 = h->uDR;
  a.E64 = h->u64E;
  a.R64 = h->u64R;
  a.nt = h->ntD.p;
  a.voff = h->voffD.p;
  a.jobs32 = h->lsj32.p;
  a.njobs32 = h->nlsj32;
  a.jobs64 = h->lsj64.p;
  a.njobs64 = h->nlsj64;
  a.maxnt = h->LD.maxnt;
  a.x = h->xl.p;
  a.y = h->yl.p;
  return a;
}

// Device work of one PCG solve: the vectors r, z, the two alternating p
// buffers and q, the partial sums of the reductions, the scalars and the
// done flag, and the alpha / beta records of the Lanczos estimate (cap + 1
// entries each).  Held by the handle (pcg_solve) or carved from the
// library's fixed device array (pcg_solve_noalloc).
struct PcgWork {
  double *r, *z, *p, *p2, *q, *partial, *rr_part, *alphas, *betas;
  PcgScalars* sc;
  int* done;
  int cap;
};

// z = M^{-1} r on stream st.  Inside the PCG loop (w not NULL) the first
// launch also performs the convergence check on the r.r partial sums in w
// and the apply is skipped once w->done is set; the combine step always
// leaves the r.z partial sums (per 256-row block) in h->rz_part.  rev: walk
// the subdomains in reverse order (consecutive applies alternate).
hipError_t apply_enqueue(geneo_handle_s* h, const double* r, double* z, const int* done,
                         hipStream_t st, const PcgWork* w, bool rev) {
  hipError_t e;
  if (w) {
    if ((e = check_apply_in(r, h->dglob.p, h->dscale.p, h->LD.nvec, h->xl.p, h->Z.p, h->zoff.p,
                            h->m.p, h->nd.p, h->voffD.p, h->coff.p, h->rH.p,
                            h->nc > 0 ? h->nsub : 0, w->rr_part, w->sc, w->done, st)))
      return e;
  } else {
    if ((e = gather_local(r, h->dglob.p, h->dscale.p, h->LD.nvec, h->xl.p, done, st))) return e;
    if (h->nc > 0 &&
        (e = restrict_coarse(r, h->Z.p, h->zoff.p, h->m.p, h->nd.p, h->dglob.p, h->voffD.p,
                             h->coff.p, h->nsub, h->rH.p, done, st)))
      return e;
  }
  if (h->local_form == GENEO_LOCAL_TRIANGULAR) {
    ProfScope ps("local_solve", st, h->bytes_local, 0.0);
    if ((e = local_solve(local_solve_args(h), done, st))) return e;
  }
  if (h->najobs > 0) {
    const SymvArgs sa = symv_args(h, rev);
    {
      ProfScope ps("symv", st,
                   h->bytes_symvH + (h->local_form == GENEO_LOCAL_INVERSE ? h->bytes_local : 0.0),
                   0.0);
      if ((e = symv_rows(sa, done, st))) return e;
    }
    {
      ProfScope ps("symv_cols", st, 0.0, 0.0);
      if ((e = symv_cols(sa, done, st))) return e;
    }
  }
  return combine(r, h->optr.p, h->oent.p, h->dscale.p, h->yl.p, h->Z.p, h->yH.p, h->n, h->nc > 0,
                 z, done, h->rz_part.p, st);
}

// Tiles per wavefront of the symmetric product (g row chunks per task): on
// the first setup of a shape each candidate is timed on the device (one
// warm launch, then three timed ones, on stream st) and the fastest is kept
// for that device and shape for the life of the process.  Every candidate
// computes bitwise the same result (the row partials are per chunk).
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int64_t, int, int>, int> g_tune;

int tune_symv_group(geneo_handle_s* h, hipStream_t st,
                    const std::function<void(int, bool)>& build) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const auto key = std::make_tuple(dev, h->najobs, h->amaxnt, (int64_t)h->LD.ntiles,
                                   (int)h->f64list.size(), h->ntc);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  HIPCHK(hipMemsetAsync(h->xl.p, 0, h->xl.n * sizeof(double), st));
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  int best = 1;
  float best_ms = 0.f;
  for (int g : {1, 2, 4}) {
    build(g, false);
    const SymvArgs sa = symv_args(h, false);
    HIPCHK(symv_rows(sa, nullptr, st));
    HIPCHK(hipEventRecord(a, st));
    for (int r = 0; r < 3; ++r) HIPCHK(symv_rows(sa, nullptr, st));
    HIPCHK(hipEventRecord(b, st));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    if (g == 1 || ms < best_ms) {
      best_ms = ms;
      best = g;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = best;
  return best;
}

__global__ void k_count_active(const int* a, int n, int* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int c = 0;
    for (int i = 0; i < n; ++i) c += a[i] != 0;
    *out = c;
  }
}

// Largest Ritz residual of the selected pairs (setup info), one block of
// 256 threads over the subdomains (a maximum: any order gives the same).
__global__ __launch_bounds__(256) void k_max_resid(const double* resid, const int* m, int nsub,
                                                   int b, double* out) {
  __shared__ double sm[256];
  double mx = 0.0;
  for (int j = threadIdx.x; j < nsub; j += blockDim.x)
    for (int c = 0; c < m[j]; ++c) mx = fmax(mx, resid[(int64_t)j * b + c]);
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

// Scratch buffers of one setup call: kept alive until the call returns so
// that no hipFree (which synchronises the device) splits the two streams.
struct SetupScratch {
  DBuf<int> status, status2, jobs, jobsN, ntN, voffN, active, pcnt, poff, npairs, woffd, cst;
  DBuf<int64_t> toffN, doffN, hdoff;
  DBuf<float> XT32;
  DBuf<double> XT64, XTH;
  DBuf<int2> ljobs32, ljobs64, ljobsH;
  DBuf<double> G, DG, U, P, W, T, Y, theta, resid, lam, mr, Wg, AHt, DH, eG, eM, epart,
      cpiv;
  DBuf<int> ebad, scount, sflag, hjob, bcnt, brp, bcol, orderN;
  // tile envelopes (first nonzero tile column per tile row, last nonzero
  // tile row per tile column) of the shifted matrices and the coarse matrix
  // (those of the local Dirichlet factors are kept by the handle)
  DBuf<int> envNE, envNR, envHE, envHR;
  // the shifted envelopes the factorisation and the eigen solves use (NULL:
  // dense, option envelope = 0)
  const int *uNE = nullptr, *uNR = nullptr;
  std::vector<double> envN_tiles;  // stored tiles per shifted factor
  std::vector<int> envD_host;      // host copy of envDE (timing mode only)
  DBuf<double> bval;
  DBuf<int> brpos;
  DBuf<int2> brows;
  bool check_cst = false;  // the coarse factor's status is read at the end
  int nbrows = 0;  // rows of B that hold entries
  int nnzB = 0;    // entries of B
  // pinned copies (NULL without pinned staging): the row count of B with
  // the event after its copy, and the shifted factor's pivot tests
  int* pin_nb = nullptr;
  hipEvent_t ev_nb = nullptr;
  int* pin_st2 = nullptr;
  ~SetupScratch() {
    if (ev_nb) (void)hipEventDestroy(ev_nb);
  }
  DBuf<double> sbest;
  DBuf<int2> tjobs32, tjobs64, tjobsH, pairs;
  DBuf<uint8_t> adj;
  DBuf<int> ocount;
  EigWork wk;
  EigStall stl;
};

// Kernels of the eigen sweeps' triangular solves.  All choices give
// bitwise the same solution; each is timed on the device at the first setup
// of a shape, on the start block (a backward solve into T, which the first
// sweep then overwrites), after one warm launch, and the fastest is kept for
// that device and shape:
//  * variant: the kernel of the unsplit solves, timed over all subdomains;
//  * split: 16-column blocks on b / 16 workgroups per subdomain, for sweeps
//    whose active subdomains (as far as the host knows) number at most
//    split_limit.  Timed against the unsplit kernel on the CUs / (b / 16)
//    largest subdomains (where the unsplit kernel leaves CUs idle that the
//    split one fills) and, if it wins there, over all subdomains as well.
std::mutex g_trsm_mu;
std::map<std::tuple<int, int, int, int64_t, int>, TrsmChoice> g_trsm_tune;

TrsmChoice tune_trsm(geneo_handle_s* h, SetupScratch& X, const LocalLayout& LN, hipStream_t sb) {
  const int b = h->b, nsub = h->nsub;
  const int nsplit = trsm_max_split(b);
  TrsmChoice c;
  c.variant = b <= 32 ? 0 : 1;
  if (b > 48) return c;
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const auto key = std::make_tuple(dev, nsub, LN.maxnt, (int64_t)LN.ntiles, b);
  {
    std::lock_guard<std::mutex> g(g_trsm_mu);
    auto it = g_trsm_tune.find(key);
    if (it != g_trsm_tune.end()) return it->second;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto time = [&](int v, int split, int n) {
    auto run = [&]() {
      HIPCHK(launch_trsm_bwd(X.G.p, X.DG.p, X.toffN.p, X.doffN.p, X.ntN.p, X.voffN.p, n, b, X.U.p,
                             X.T.p, nullptr, X.orderN.p, X.uNE, X.uNR, v, split, sb));
    };
    run();
    HIPCHK(hipEventRecord(e0, sb));
    run();
    HIPCHK(hipEventRecord(e1, sb));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return ms;
  };
  // the fastest of the variants a launch of this shape can take (b = 48
  // unsplit has only the one-row-per-wavefront kernels)
  auto fastest = [&](int split, int n, int& best) {
    float bt = 0.f;
    best = -1;
    for (int v = 0; v < trsm_variants(); ++v) {
      if (b == 48 && split == 1 && (v & 1) == 0) continue;
      const float t = time(v, split, n);
      if (best < 0 || t < bt) bt = t, best = v;
    }
    return bt;
  };
  const float tu = fastest(1, nsub, c.variant);
  if (nsplit > 1) {
    // with at most ncu / nsplit subdomains active the split solves fill
    // the CUs that the unsplit ones leave idle
    const int n1 = std::max(1, std::min(nsub, ncu / nsplit));
    const float tu1 = n1 == nsub ? tu : time(c.variant, 1, n1);
    const float ts1 = fastest(nsplit, n1, c.split_variant);
    if (ts1 < tu1) {
      c.split_limit = n1;
      if (n1 < nsub && time(c.split_variant, nsplit, nsub) < tu) c.split_limit = nsub;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> g(g_trsm_mu);
  g_trsm_tune[key] = c;
  return c;
}

struct PhaseTimer {
  hipEvent_t a = nullptr, b = nullptr;
  void start(hipStream_t st) {
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    HIPCHK(hipEventRecord(a, st));
  }
  void stop(hipStream_t st) { HIPCHK(hipEventRecord(b, st)); }
  double ms() {
    if (!a || !b) return 0.0;
    float t = 0.f;
    HIPCHK(hipEventSynchronize(b));
    HIPCHK(hipEventElapsedTime(&t, a, b));
    return t;
  }
  ~PhaseTimer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Subdomains by decreasing size (stable): the dispatch order of the
// one-workgroup-per-subdomain launches, so that the hardware's workgroup
// queue hands out the longest jobs first (largest-first scheduling over
// uneven subdomains).
std::vector<int> largest_first(const std::vector<int>& size) {
  std::vector<int> o(size.size());
  for (size_t j = 0; j < o.size(); ++j) o[j] = (int)j;
  std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return size[a] > size[b]; });
  return o;
}

// Jobs of the inverse factors: (matrix, first tile column) in blocks of
// trtri_cols_per_job columns, the longest columns (smallest c0) first.
std::vector<int2> trtri_job_list(const std::vector<int>& mats, const std::vector<int>& nt,
                                 bool fp32) {
  const int ncol = trtri_cols_per_job(fp32);
  int maxnt = 0;
  for (int j : mats) maxnt = std::max(maxnt, nt[j]);
  std::vector<int2> tj;
  for (int c0 = 0; c0 < maxnt; c0 += ncol)
    for (int j : mats)
      if (c0 < nt[j]) tj.push_back(make_int2(j, c0));
  return tj;
}

// Up to this many FP64 refactors use the tile-column-step factorisation.
constexpr int kStepCholMax = 32;

// Jobs of S = X^T X: (matrix, I << 16 | J0) for the output tiles (I, J0 ..
// J0 + lauum_tiles_per_job() - 1) of each tile row I, matrix by matrix and
// within a matrix the longest rows (small I) first.
std::vector<int2> lauum_job_list(const std::vector<int>& mats, const std::vector<int>& nt) {
  const int w = lauum_tiles_per_job();
  std::vector<int2> lj;
  for (int j : mats) {
    if (nt[j] >= 32768) fail(GENEO_ERR_ARG, "local matrix too large for the dense inverse");
    for (int I = 0; I < nt[j]; ++I)
      for (int J0 = 0; J0 <= I; J0 += w) lj.push_back(make_int2(j, (I << 16) | J0));
  }
  return lj;
}

// Algorithmic bytes of one local_solve launch: each factor's tiles inside
// its envelope read twice (forward and backward), its inverted diagonal
// tiles in place of the diagonal tiles of L, and its vectors read and
// written once.  E32 / E64: host copies of the envelopes (empty: dense).
double local_solve_bytes(const geneo_handle_s* h, const std::vector<int>& E32,
                         const std::vector<int>& E64) {
  std::vector<char> is64(h->nsub, 0);
  for (int j : h->f64list) is64[j] = 1;
  double bytes = 0.0;
  for (int j = 0; j < h->nsub; ++j) {
    const int nt = h->LD.nt[j];
    const std::vector<int>& E = is64[j] ? E64 : E32;
    const int64_t d0 = is64[j] ? (j < (int)h->doff64_host.size() ? h->doff64_host[j] : 0)
                               : h->LD.doff[j];
    double off = 0.0;
    for (int i = 0; i < nt; ++i)
      off += (size_t)(d0 + i) < E.size() ? i - E[d0 + i] : i;
    bytes += 2.0 * (is64[j] ? 8.0 : 4.0) * TSQ * (off + nt) + 16.0 * nt * TS;
  }
  return bytes;
}

// Form of the local solves of the apply (option local_solve; 0 = by this
// estimate of the time per PCG iteration, from measurements on MI355X):
//  * triangular: forward and backward substitution tile row by tile row,
//    all subdomains at once (two workgroups per CU), each row about 3 us
//    of dependent latency: 2 nt_max rows per round of 2 * CUs subdomains;
//  * inverse: one pass over the packed inverses at about 5 TB/s, plus the
//    inverse factor and the symmetric product of the setup (2 n^3 / 3 flop
//    per subdomain at about 80 TFLOP/s) spread over 50 iterations.
// Small local problems or few subdomains favour the inverse (one fully
// parallel pass), large banded 3D problems the substitution (two reads of
// the envelope instead of one of the dense inverse, and no inverse to
// form).  Both are exact up to rounding; matrices too large for the
// substitution's LDS take the inverse.
int choose_local_form(const geneo_handle_s* h) {
  if (h->opts.local_solve == GENEO_LOCAL_TRIANGULAR || h->opts.local_solve == GENEO_LOCAL_INVERSE)
    return h->opts.local_solve;
  if (local_solve_check(h->LD.maxnt) != hipSuccess) return GENEO_LOCAL_INVERSE;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  // triangular: two passes of maxnt tile-row steps, measured at about
  // 2.4 us per step for FP32 factors (three workgroups per compute unit)
  // and 3 us for FP64 factors (two workgroups per unit)
  const int n64 = (int)h->f64list.size(), n32 = h->nsub - n64;
  const double cu = std::max(ncu, 1);
  const double t_tri = 2.0 * h->LD.maxnt *
                       (2.4e-6 * std::ceil(n32 / (3.0 * cu)) + 3e-6 * std::ceil(n64 / (2.0 * cu)));
  std::vector<char> is64(h->nsub, 0);
  for (int j : h->f64list) is64[j] = 1;
  double bytes = 0.0, flops = 0.0;
  for (int j = 0; j < h->nsub; ++j) {
    const double nn = h->nd_host[j];
    bytes += (is64[j] ? 8.0 : 4.0) * packed(nn);
    flops += 2.0 * nn * nn * nn / 3.0;
  }
  const double t_inv = bytes / 5e12 + flops / 80e12 / 50.0;
  return t_tri <= t_inv ? GENEO_LOCAL_TRIANGULAR : GENEO_LOCAL_INVERSE;
}

// Local Dirichlet factors of A_j = R_j A R_j^T, on stream st.  Returns after the work is enqueued and the pivot tests are
// read back.
std::function<void(hipStream_t)> setup_local(geneo_handle_s* h, SetupScratch& X,
                                             const geneo_csr_t* A, const geneo_subdomains_t* S,
                                             hipStream_t st,
                                             const std::function<void(hipEvent_t)>& after_fp32) {
  const geneo_opts_t& o = h->opts;
  const int nsub = h->nsub;
  std::vector<int> all(nsub);
  for (int j = 0; j < nsub; ++j) all[j] = j;
  std::vector<int> f64list, inv32;
  const bool mixed = o.precision == GENEO_PREC_MIXED;
  X.status.alloc(nsub);
  if (mixed) {
    X.jobs.upload(largest_first(h->nd_host), st);
    h->L32.alloc(h->LD.ntiles * TSQ);
    h->D32.alloc(h->LD.ndiag * TSQ);
    h->envDE.alloc(h->LD.ndiag);
    h->envDR.alloc(h->LD.ndiag);
    {
      ProfScope ps("densify_dirichlet", st, 4.0 * h->LD.ntiles * TSQ, 0.0);
      HIPCHK(hipMemsetAsync(h->L32.p, 0, h->L32.n * sizeof(float), st));
      HIPCHK(launch_env_init(h->envDE.p, h->doffD.p, h->ntD.p, nullptr, nsub, st));
      HIPCHK(launch_densify_dirichlet(true, h->L32.p, h->toffD.p, h->ntD.p, h->voffD.p, X.jobs.p,
                                      nsub, S->sub_ptr, S->sub_idx, h->dmap.p, h->dglob.p,
                                      h->dscale.p, A,
                                      *std::max_element(h->LD.nt.begin(), h->LD.nt.end()),
                                      h->envDE.p, h->doffD.p, st));
      HIPCHK(launch_env_finish(h->envDE.p, h->envDR.p, h->doffD.p, h->ntD.p, nullptr, nsub, st));
      if (o.envelope) h->uDE = h->envDE.p, h->uDR = h->envDR.p;
    }
    {
      // algorithmic work inside the envelopes (read back in the timing mode
      // only, where it is reported)
      double tl = 0.0, fl = 0.0;
      if (prof_on() && h->uDE) {
        X.envD_host = download(h->envDE.p, h->LD.ndiag, st);
        const EnvWork ew = env_work(X.envD_host, h->LD.doff, h->LD.nt, all);
        for (double t : ew.tiles) tl += t;
        fl = 2.0 * TS * TS * TS * ew.prods + (double)TS * TS * TS * tl;
      }
      ProfScope ps("chol_dirichlet_f32", st, 2.0 * 4.0 * TSQ * tl, fl);
      HIPCHK(launch_chol_batched(CholRole::LocalF32, h->L32.p, h->toffD.p, h->ntD.p, h->D32.p, h->doffD.p,
                                 X.status.p, X.jobs.p, nsub, o.pivot_tol, h->uDE, h->uDR,
                                 st));
    }
    // the shifted factorisation follows the FP32 one on the device (an
    // event, no host round trip) while the host reads the pivot tests
    HIPCHK(hipEventCreateWithFlags(&h->f32_done, hipEventDisableTiming));
    HIPCHK(hipEventRecord(h->f32_done, st));
    after_fp32(h->f32_done);
    auto stat = download(X.status.p, nsub, st);
    if (h->shifted_done) HIPCHK(hipStreamWaitEvent(st, h->shifted_done, 0));
    std::vector<int> ok32;
    for (int j = 0; j < nsub; ++j) (stat[j] ? f64list : ok32).push_back(j);
    h->njobs32 = (int)ok32.size();
    h->jobs32.upload(ok32, st);
    inv32 = std::move(ok32);
  } else {
    f64list = all;
    after_fp32(nullptr);
  }
  // The FP64 refactors of the subdomains that failed the pivot test (all
  // subdomains in FP64 mode) and, in the inverse form of the local solves,
  // the inverses go back to the caller as a step to enqueue later: nothing
  // before the PCG needs them, and the eigen sweeps, once few subdomains
  // are active, leave most CUs idle.
  return [h, &X, A, S, nsub, mixed, f64list = std::move(f64list),
          ok32 = std::move(inv32)](hipStream_t st) mutable {
    h->info.fallback_fp64 = mixed ? (int)f64list.size() : 0;
    h->njobs64 = (int)f64list.size();
    h->jobs64.upload(f64list, st);
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
    h->toff64_host = toff64;
    h->doff64_host = doff64;
    {
      std::vector<int2> lj(nsub);
      std::vector<char> f(nsub, 0);
      for (int j : f64list) f[j] = 1;
      for (int j = 0; j < nsub; ++j) lj[j] = make_int2(j, f[j]);
      h->ljobs_host = lj;
    }
    if (!f64list.empty()) {
      h->L64.alloc(tt * TSQ);
      h->D64.alloc(dd * TSQ);
      h->env64E.alloc(dd);
      h->env64R.alloc(dd);
      double pk64 = 0.0, fl64 = 0.0;
      int mx = 0;
      for (int j : f64list) {
        mx = std::max(mx, h->LD.nt[j]);
        pk64 += packed(h->nd_host[j]);
        fl64 += std::pow((double)h->nd_host[j], 3) / 3.0;
      }
      {
        ProfScope ps("densify_dirichlet", st, 8.0 * tt * TSQ, 0.0);
        HIPCHK(hipMemsetAsync(h->L64.p, 0, h->L64.n * sizeof(double), st));
        HIPCHK(launch_env_init(h->env64E.p, h->doff64.p, h->ntD.p, h->jobs64.p, h->njobs64, st));
        HIPCHK(launch_densify_dirichlet(false, h->L64.p, h->toff64.p, h->ntD.p, h->voffD.p,
                                        h->jobs64.p, h->njobs64, S->sub_ptr, S->sub_idx,
                                        h->dmap.p, h->dglob.p, h->dscale.p, A, mx, h->env64E.p,
                                        h->doff64.p, st));
        HIPCHK(launch_env_finish(h->env64E.p, h->env64R.p, h->doff64.p, h->ntD.p, h->jobs64.p,
                                 h->njobs64, st));
        if (h->opts.envelope) h->u64E = h->env64E.p, h->u64R = h->env64R.p;
      }
      {
        // a few refactors (mixed mode): tile-column steps over many short
        // workgroups, which leave the CUs to the eigen sweeps in between
        // (dense); a full batch (FP64 mode): one workgroup per matrix,
        // inside the envelopes
        const bool steps = h->njobs64 <= kStepCholMax;
        if (!steps && prof_on() && h->u64E) {
          const EnvWork ew = env_work(download(h->env64E.p, dd, st), doff64,
                                      h->LD.nt, f64list);
          pk64 = 0.0;
          for (double t : ew.tiles) pk64 += TSQ * t;
          fl64 = 2.0 * TS * TS * TS * ew.prods + (double)TS * pk64;
        }
        ProfScope ps("chol_dirichlet_f64", st, 2.0 * 8.0 * pk64, fl64);
        if (steps) {
          HIPCHK(launch_chol_steps(h->L64.p, h->D64.p, h->toff64.p, h->doff64.p, h->ntD.p,
                                   h->jobs64.p, h->njobs64, mx, X.status.p, st, nullptr,
                                   h->u64R));
        } else {
          HIPCHK(launch_chol_batched(CholRole::LocalF64, h->L64.p, h->toff64.p, h->ntD.p, h->D64.p,
                                     h->doff64.p, X.status.p, h->jobs64.p, h->njobs64, 0.0,
                                     h->u64E, h->u64R, st));
        }
      }
    }
    h->f64list = f64list;
    h->local_form = choose_local_form(h);
    if (h->local_form == GENEO_LOCAL_TRIANGULAR) {
      h->bytes_local = local_solve_bytes(
          h, X.envD_host,
          prof_on() && h->u64E ? download(h->env64E.p, h->env64E.n, st) : std::vector<int>{});
      h->info.bytes_local_factors = (int64_t)(h->L32.n + h->D32.n) * 4 +
                                    (int64_t)(h->L64.n + h->D64.n) * 8;
      return;
    }
    // inverse form: X_j = L_j^{-1}, then A_j^{-1} = X_j^T X_j
    if (!ok32.empty()) {
      std::vector<int2> tj = trtri_job_list(ok32, h->LD.nt, true);
      X.tjobs32.upload(tj, st);
      std::vector<int2> lj = lauum_job_list(ok32, h->LD.nt);
      X.ljobs32.upload(lj, st);
      X.XT32.alloc(h->LD.ntiles * TSQ);
      double pk32 = 0.0, fl32 = 0.0;
      for (int j : ok32) {
        pk32 += packed(h->nd_host[j]);
        fl32 += std::pow((double)h->nd_host[j], 3) / 3.0;
      }
      {
        // the inverse of a banded factor is dense; its products skip the
        // zero tiles of L
        double flt = fl32;
        if (!X.envD_host.empty())
          flt = 2.0 * TS * TS * TS * env_work(X.envD_host, h->LD.doff, h->LD.nt, ok32).inv_prods;
        ProfScope ps("trtri_dirichlet", st, 2.0 * 4.0 * pk32, flt);
        HIPCHK(launch_trtri(true, h->L32.p, h->D32.p, X.XT32.p, h->toffD.p, h->doffD.p, h->ntD.p,
                            X.tjobs32.p, (int)tj.size(), h->uDE, st));
      }
      h->S32.alloc(h->LD.ntiles * TSQ);
      h->W32.alloc(h->LD.ntiles * TS);
      ProfScope ps("lauum_dirichlet", st, 2.0 * 4.0 * pk32, fl32);
      HIPCHK(launch_lauum(true, X.XT32.p, h->S32.p, h->toffD.p, h->ntD.p, X.ljobs32.p,
                          (int)lj.size(), st));
    }
    if (!f64list.empty()) {
      int64_t tt = 0;
      double pk64 = 0.0, fl64 = 0.0;
      for (int j : f64list) {
        tt += tri_tiles(h->LD.nt[j]);
        pk64 += packed(h->nd_host[j]);
        fl64 += std::pow((double)h->nd_host[j], 3) / 3.0;
      }
      std::vector<int2> tj = trtri_job_list(f64list, h->LD.nt, false);
      X.tjobs64.upload(tj, st);
      std::vector<int2> lj = lauum_job_list(f64list, h->LD.nt);
      X.ljobs64.upload(lj, st);
      X.XT64.alloc(tt * TSQ);
      {
        ProfScope ps("trtri_dirichlet", st, 2.0 * 8.0 * pk64, fl64);
        HIPCHK(launch_trtri(false, h->L64.p, h->D64.p, X.XT64.p, h->toff64.p, h->doff64.p,
                            h->ntD.p, X.tjobs64.p, (int)tj.size(), h->u64E, st));
      }
      h->S64.alloc(tt * TSQ);
      h->W64.alloc(tt * TS);
      ProfScope ps("lauum_dirichlet", st, 2.0 * 8.0 * pk64, fl64);
      HIPCHK(launch_lauum(false, X.XT64.p, h->S64.p, h->toff64.p, h->ntD.p, X.ljobs64.p,
                          (int)lj.size(), st));
    }
    double b = 0.0;
    std::vector<char> is64(nsub, 0);
    for (int j : f64list) is64[j] = 1;
    for (int j = 0; j < nsub; ++j) {
      const double nn = h->nd_host[j];
      b += (is64[j] ? 8.0 : 4.0) * packed(nn) + 16.0 * nn;
    }
    h->bytes_local = b;
    h->info.bytes_local_factors =
        (int64_t)(h->S32.p ? h->LD.ntiles * TSQ * 4 : 0) + (int64_t)h->S64.n * 8;
  };
}

// Start of the eigen sweeps, independent of the shifted factors: the
// compact B_j, the pseudo-random start blocks (orthonormalised) and the
// work buffers.  Enqueued on sb ahead of the shifted factorisation: it
// then runs alone (between the FP32 local factorisation and the shifted
// one) instead of beside the inverse-factor kernels, which would hold the
// device while its many short launches wait.
void eigen_prepare(geneo_handle_s* h, SetupScratch& X, const LocalLayout& LN,
                   const geneo_subdomains_t* S, const geneo_csr_batch_t* Ao, int nnz,
                   hipStream_t sb) {
  const geneo_opts_t& o = h->opts;
  const int nsub = h->nsub;
  const int b = h->b;
  {
    // compact B_j = X_j A^o_j X_j, sized by the nnz nonzeros of the A^o batch
    X.bcnt.alloc(h->nloc);
    X.brp.alloc(h->nloc + 1);
    X.bcol.alloc(std::max(nnz, 1));
    X.bval.alloc(std::max(nnz, 1));
    X.nnzB = nnz;
    X.brpos.alloc(h->nloc + 1);
    X.brows.alloc(std::max<int64_t>(h->nloc, 1));
    HIPCHK(launch_bcompact(S->sub_ptr, S->pou, Ao, nsub, h->nloc, LN.maxnt * TS, X.bcnt.p,
                           X.brp.p, X.bcol.p, X.bval.p, X.brpos.p, X.brows.p, sb));
    // the row count goes to pinned memory now; the sweeps read it much later
    X.pin_nb = t_arena.active ? (int*)t_arena.take(sizeof(int)) : nullptr;
    if (X.pin_nb) {
      HIPCHK(hipMemcpyAsync(X.pin_nb, X.brpos.p + h->nloc, sizeof(int), hipMemcpyDeviceToHost, sb));
      HIPCHK(hipEventCreateWithFlags(&X.ev_nb, hipEventDisableTiming));
      HIPCHK(hipEventRecord(X.ev_nb, sb));
    }
  }
  // W = B T is zero away from the rows of B that hold entries: cleared
  // once, the products then write only those rows
  HIPCHK(hipMemsetAsync(X.W.p, 0, X.W.n * sizeof(double), sb));
  HIPCHK(fill_i32(X.active.p, 1, nsub, sb));
  HIPCHK(launch_eig_init(X.U.p, S->sub_ptr, X.voffN.p, X.ntN.p, nsub, b, o.seed, sb));
  EigWork& wk = X.wk;
  wk.ngroups = (LN.maxnt * TS / 16 + 7) / 8;  // SLABS_PER_WG = 8
  X.eG.alloc((size_t)nsub * b * b);
  X.eM.alloc((size_t)nsub * b * b);
  X.epart.alloc((size_t)nsub * wk.ngroups * b);
  X.ebad.alloc((size_t)nsub * b);
  wk.G = X.eG.p;
  wk.M = X.eM.p;
  wk.part = X.epart.p;
  wk.badcol = X.ebad.p;
  EigStall& stl = X.stl;
  X.sbest.alloc(nsub);
  X.scount.alloc(nsub);
  X.sflag.alloc(nsub);
  HIPCHK(hipMemsetAsync(X.sbest.p, 0x7f, nsub * sizeof(double), sb));  // ~1.4e306
  HIPCHK(hipMemsetAsync(X.scount.p, 0, nsub * sizeof(int), sb));
  HIPCHK(hipMemsetAsync(X.sflag.p, 0, nsub * sizeof(int), sb));
  stl.best = X.sbest.p;
  stl.count = X.scount.p;
  stl.stalled = X.sflag.p;
  stl.sweeps = o.eig_stall;
  stl.floor = o.eig_floor;
  HIPCHK(launch_orth2(X.U.p, X.voffN.p, X.ntN.p, nsub, b, o.seed, 0, nullptr, wk, sb));
}

// Shifted matrices C_j = A_N,j - sigma B_j and their factors C_j = G_j G_j^T,
// enqueued on stream sb (no host wait) after the event `after` (may be
// NULL) has completed.
void setup_shifted(geneo_handle_s* h, SetupScratch& X, LocalLayout& LN,
                   const geneo_subdomains_t* S, const geneo_csr_batch_t* An,
                   const geneo_csr_batch_t* Ao, hipStream_t sb, PhaseTimer* tm,
                   hipEvent_t after) {
  const geneo_opts_t& o = h->opts;
  const int nsub = h->nsub;
  std::vector<int> all(nsub);
  for (int j = 0; j < nsub; ++j) all[j] = j;
  LN.build(h->nN_host);
  X.ntN.upload(LN.nt, sb);
  X.voffN.upload(LN.voff, sb);
  X.toffN.upload(LN.toff, sb);
  X.doffN.upload(LN.doff, sb);
  {
    const std::vector<int> ord = largest_first(h->nN_host);
    X.jobsN.upload(ord, sb);
    X.orderN.upload(ord, sb);
  }
  X.status2.alloc(nsub);
  X.G.alloc(LN.ntiles * TSQ);
  X.DG.alloc(LN.ndiag * TSQ);
  // eigen block size
  const int want = (o.tau > 0 || h->tau_sub.p) ? o.nev_max : o.nev;
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
  X.U.alloc(LN.nvec * b);
  if (o.eig_cheb >= 2) X.P.alloc(LN.nvec * b);
  X.W.alloc(LN.nvec * b);
  X.T.alloc(LN.nvec * b);
  X.Y.alloc(LN.nvec * b);
  X.theta.alloc((size_t)nsub * b);
  X.resid.alloc((size_t)nsub * b);
  X.active.alloc(nsub);
  X.lam.alloc((size_t)nsub * b);
  X.mr.alloc(1);
  h->m.alloc(nsub);

  // (read while the stream is still idle)
  const int nnzB = download(Ao->rowptr + h->nloc, 1, sb)[0];
  if (after) HIPCHK(hipStreamWaitEvent(sb, after, 0));
  eigen_prepare(h, X, LN, S, Ao, nnzB, sb);
  tm[0].start(sb);
  X.envNE.alloc(LN.ndiag);
  X.envNR.alloc(LN.ndiag);
  {
    ProfScope ps("densify_shifted", sb, 8.0 * LN.ntiles * TSQ, 0.0);
    HIPCHK(launch_env_init(X.envNE.p, X.doffN.p, X.ntN.p, nullptr, nsub, sb));
    if (o.envelope) {
      // envelope from the patterns, then only its tiles are cleared (option
      // envelope = 2 fills all others with NaN first: a check that nothing
      // reads them)
      HIPCHK(launch_env_shifted(X.ntN.p, nsub, LN.maxnt, S->sub_ptr, An, Ao, X.envNE.p, X.doffN.p,
                                sb));
      HIPCHK(launch_env_finish(X.envNE.p, X.envNR.p, X.doffN.p, X.ntN.p, nullptr, nsub, sb));
      if (o.envelope == 2) HIPCHK(hipMemsetAsync(X.G.p, 0xff, X.G.n * sizeof(double), sb));
      HIPCHK(launch_env_clear(X.G.p, X.toffN.p, X.ntN.p, nsub, LN.maxnt, X.envNE.p, X.doffN.p,
                              sb));
      HIPCHK(launch_densify_shifted(X.G.p, X.toffN.p, X.ntN.p, nsub, S->sub_ptr, S->pou, An, Ao,
                                    o.sigma, nullptr, X.doffN.p, sb));
      X.uNE = X.envNE.p, X.uNR = X.envNR.p;
    } else {
      HIPCHK(hipMemsetAsync(X.G.p, 0, X.G.n * sizeof(double), sb));
      HIPCHK(launch_densify_shifted(X.G.p, X.toffN.p, X.ntN.p, nsub, S->sub_ptr, S->pou, An, Ao,
                                    o.sigma, X.envNE.p, X.doffN.p, sb));
      HIPCHK(launch_env_finish(X.envNE.p, X.envNR.p, X.doffN.p, X.ntN.p, nullptr, nsub, sb));
    }
  }
  // algorithmic work inside the envelopes: read back in the timing mode
  // only (where it is reported); otherwise the dense counts stand in
  double tlN = 0.0, flN = 0.0;
  if (prof_on() && X.uNE) {
    std::vector<int> all(nsub);
    for (int j = 0; j < nsub; ++j) all[j] = j;
    const EnvWork ew = env_work(download(X.envNE.p, LN.ndiag, sb), LN.doff, LN.nt, all);
    X.envN_tiles = ew.tiles;
    for (double t : ew.tiles) tlN += t;
    flN = 2.0 * TS * TS * TS * ew.prods + (double)TS * TS * TS * tlN;
  } else {
    X.envN_tiles.assign(nsub, 0.0);
    for (int j = 0; j < nsub; ++j) X.envN_tiles[j] = packed(LN.nt[j]);
  }
  // few subdomains: tile-column steps over many workgroups (the rows each
  // step reaches come from the envelopes, read back here)
  const bool steps = o.shifted_steps > 0 || (o.shifted_steps == 0 && nsub <= kStepCholMax);
  std::vector<int> rlast;
  if (steps && X.uNR) {
    const std::vector<int> R = download(X.envNR.p, LN.ndiag, sb);
    rlast.assign(LN.maxnt, 0);
    for (int j = 0; j < nsub; ++j)
      for (int k = 0; k < LN.nt[j]; ++k) rlast[k] = std::max(rlast[k], R[LN.doff[j] + k]);
  }
  {
    ProfScope ps("chol_shifted_f64", sb, 2.0 * 8.0 * TSQ * tlN, flN);
    if (steps)
      HIPCHK(launch_chol_steps(X.G.p, X.DG.p, X.toffN.p, X.doffN.p, X.ntN.p, X.jobsN.p, nsub,
                               LN.maxnt, X.status2.p, sb, nullptr, X.uNR,
                               X.uNR ? rlast.data() : nullptr));
    else
      HIPCHK(launch_chol_batched(CholRole::ShiftedF64, X.G.p, X.toffN.p, X.ntN.p, X.DG.p,
                                 X.doffN.p, X.status2.p, X.jobsN.p, nsub, 0.0, X.uNE, X.uNR, sb));
    X.pin_st2 = t_arena.active ? (int*)t_arena.take((size_t)nsub * sizeof(int)) : nullptr;
    if (X.pin_st2)
      HIPCHK(hipMemcpyAsync(X.pin_st2, X.status2.p, (size_t)nsub * sizeof(int),
                            hipMemcpyDeviceToHost, sb));
  }
  tm[0].stop(sb);
  // the FP64 refactors and the FP32 inverse factors on the other stream
  // start after this factorisation and overlap the eigen sweeps instead
  HIPCHK(hipEventCreateWithFlags(&h->shifted_done, hipEventDisableTiming));
  HIPCHK(hipEventRecord(h->shifted_done, sb));
}

// Eigen sweeps, coarse basis, Galerkin product and coarse factor on sb.
// deferred_local (the local step nothing before the PCG needs) is called
// once: after the first sweep that leaves at most local_at subdomains
// active as far as the host knows, else after the last sweep (and before
// any error return that follows it).
void setup_coarse(geneo_handle_s* h, SetupScratch& X, const LocalLayout& LN,
                  const geneo_subdomains_t* S, const geneo_csr_batch_t* An,
                  const geneo_csr_batch_t* Ao, hipStream_t sb, PhaseTimer* tm,
                  const std::function<void()>& deferred_local) {
  const geneo_opts_t& o = h->opts;
  const int nsub = h->nsub;
  const int b = h->b;
  // No host wait before the first sweeps: the row count of B was copied
  // to pinned memory before the shifted factorisation, and the pivot tests
  // of that factorisation are checked at the first read of the sweep flags
  // (a failed factor makes only wrong numbers in the sweeps meanwhile:
  // every loop bound and address is independent of the matrix values).
  if (X.pin_nb) {
    HIPCHK(hipEventSynchronize(X.ev_nb));
    X.nbrows = *X.pin_nb;
    HIPCHK(hipEventDestroy(X.ev_nb));
    X.ev_nb = nullptr;
  } else {
    X.nbrows = download(X.brpos.p + h->nloc, 1, sb)[0];
  }
  bool shift_checked = false;
  auto check_shifted = [&](const int* stat) {
    shift_checked = true;
    for (int j = 0; j < nsub; ++j)
      if (stat[j]) fail(GENEO_ERR_SHIFT_NOT_SPD, "A_N - sigma B of subdomain " +
                                                     std::to_string(j) + " is not SPD");
  };
  if (!X.pin_st2) check_shifted(download(X.status2.p, nsub, sb).data());
  // ---- block subspace iteration on S = G^{-1} B G^{-T}
  tm[1].start(sb);
  if (o.eig_solve > 0 && o.eig_split != 0) {
    h->trsm.variant = h->trsm.split_variant = o.eig_solve - 1;
  } else {
    h->trsm = tune_trsm(h, X, LN, sb);
    if (o.eig_solve > 0) h->trsm.variant = h->trsm.split_variant = o.eig_solve - 1;
  }
  if (b > 32 && (h->trsm.variant & 1) == 0) h->trsm.variant += 1;  // unsplit b = 48
  if (o.eig_split != 0) h->trsm.split_limit = std::min(std::max(o.eig_split, 0), nsub);
  if (trsm_max_split(b) == 1) h->trsm.split_limit = 0;
  h->info.eig_solve = h->trsm.variant + 1;
  h->info.eig_split = h->trsm.split_limit;
  h->info.eig_solve_split = h->trsm.split_variant + 1;
  // kernel and split of the solves while (at most) na subdomains are active
  auto tv = [&](int na) { return na <= h->trsm.split_limit ? h->trsm.split_variant : h->trsm.variant; };
  auto ts = [&](int na) { return na <= h->trsm.split_limit ? trsm_max_split(b) : 1; };
  const EigWork& wk = X.wk;
  const EigStall& stl = X.stl;
  int sweeps = 0, nact = nsub;
  std::vector<int> act(nsub, 1);
  // The active flags of sweep it are copied to pinned memory and read by
  // the host after sweep it+1 has been enqueued, so the device never waits
  // for the host between sweeps.  Every kernel skips inactive subdomains,
  // so a sweep enqueued after the last one needed costs only empty
  // launches and changes nothing.  With per-kernel timing on, each sweep is
  // read at once (its byte counts then follow the active set exactly).
  int* aflag[2] = {nullptr, nullptr};
  struct EvPair {  // destroyed also when a check below throws
    hipEvent_t e[2] = {nullptr, nullptr};
    ~EvPair() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } aevs;
  hipEvent_t* aev = aevs.e;
  bool lag = !prof_on() && t_arena.active;
  for (int k = 0; k < 2 && lag; ++k) {
    aflag[k] = (int*)t_arena.take((size_t)nsub * sizeof(int));
    lag = aflag[k] != nullptr;
  }
  for (int k = 0; k < 2 && lag; ++k) HIPCHK(hipEventCreateWithFlags(&aev[k], hipEventDisableTiming));
  auto read_active = [&](int it) {
    if (lag) {
      HIPCHK(hipEventSynchronize(aev[it & 1]));
      act.assign(aflag[it & 1], aflag[it & 1] + nsub);
    } else {
      act = download(X.active.p, nsub, sb);
    }
    // the pivot-test copy precedes every sweep on sb, so it has landed
    if (!shift_checked) check_shifted(X.pin_st2);
    nact = 0;
    for (int j = 0; j < nsub; ++j) nact += act[j] != 0;
  };
  bool finished = false;
  bool local_done = false;
  // the deferred local step (inverse factors) is enqueued once at most
  // half as many subdomains as CUs are still active: from then on the
  // sweeps leave CUs idle (96^3 layers: 700 -> 694 ms per step, against
  // enqueuing it after the first sweep)
  int local_at = 0;
  {
    int dev = 0, ncu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    local_at = std::max(1, ncu / 2);
  }
  for (int it = 1; it <= o.eig_maxit; ++it) {
    // algorithmic traffic of this sweep: the factor G_j of every active
    // subdomain is read once per triangular solve, plus its b columns
    double gb = 0.0, vb = 0.0, tf = 0.0;
    for (int j = 0; j < nsub; ++j) {
      if (!act[j]) continue;
      double nn = h->nN_host[j];
      gb += 8.0 * TSQ * X.envN_tiles[j];
      vb += 2.0 * 8.0 * nn * b;
      tf += 2.0 * TSQ * X.envN_tiles[j] * b;
    }
    {
      ProfScope ps(ts(nact) > 1 ? "trsm_bwd_split" : "trsm_bwd", sb, gb + vb, tf);
      HIPCHK(launch_trsm_bwd(X.G.p, X.DG.p, X.toffN.p, X.doffN.p, X.ntN.p, X.voffN.p, nsub, b,
                             X.U.p, X.T.p, X.active.p, X.orderN.p, X.uNE, X.uNR,
                             tv(nact), ts(nact), sb));
    }
    {
      // the B entries, the T rows they reach (once each) and the W rows
      // written, over all subdomains
      ProfScope ps("bapply", sb, 12.0 * X.nnzB + 2.0 * 8.0 * X.nbrows * b, 0.0);
      HIPCHK(launch_bapply(S->sub_ptr, X.brp.p, X.bcol.p, X.bval.p, X.brows.p, X.nbrows, X.voffN.p,
                           b, X.T.p, X.W.p, X.active.p, sb));
    }
    {
      ProfScope ps(ts(nact) > 1 ? "trsm_fwd_split" : "trsm_fwd", sb, gb + vb, tf);
      HIPCHK(launch_trsm_fwd(X.G.p, X.DG.p, X.toffN.p, X.doffN.p, X.ntN.p, X.voffN.p, nsub, b,
                             X.W.p, X.T.p, X.active.p, X.orderN.p, X.uNE, X.uNR,
                             tv(nact), ts(nact), sb));
    }
    {
      ProfScope ps("rayleigh_ritz", sb, 2.0 * vb, 0.0);
      HIPCHK(launch_rr2(X.U.p, X.T.p, X.Y.p, X.theta.p, X.resid.p, X.active.p, X.voffN.p,
                        X.ntN.p, nsub, b, o.nev, o.tau, h->tau_sub.p, o.nev_max, o.sigma,
                        o.eig_tol, wk, stl, sb));
    }
    if (lag) {
      HIPCHK(hipMemcpyAsync(aflag[it & 1], X.active.p, (size_t)nsub * sizeof(int),
                            hipMemcpyDeviceToHost, sb));
      HIPCHK(hipEventRecord(aev[it & 1], sb));
    }
    if (lag) {
      if (it > 1) {
        read_active(it - 1);
        if (nact == 0) {
          finished = true;
          break;
        }
      }
    } else {
      read_active(it);
      if (nact == 0) {
        sweeps = it;
        finished = true;
        break;
      }
    }
    if (!local_done && nact <= local_at) {
      local_done = true;
      deferred_local();
    }
    sweeps = it;
    if (o.eig_cheb >= 2 && it >= 3) {
      // Chebyshev filter of degree m on the Ritz block Y (kept intact for
      // the final eigenvectors): U holds S Y from the Rayleigh-Ritz step;
      // Z_1 = (2/a) S Y - Y goes to U, Z_0 is Y itself, and each further
      // degree costs one shifted solve; Z_{k+1} goes to P (then swapped
      // with U), Z_m ends in U.
      // (each launch timed under its kernel's name: the solves and B
      // products count with those of the sweep itself)
      {
        ProfScope ps("cheb_combine", sb, 3.0 * vb / 2.0, 0.0);
        HIPCHK(launch_cheb(X.U.p, nullptr, X.U.p, X.Y.p, X.theta.p, X.voffN.p, X.ntN.p, nsub, b,
                           LN.maxnt, true, X.active.p, sb));
      }
      for (int k = 1; k < o.eig_cheb; ++k) {
        {
          ProfScope ps(ts(nact) > 1 ? "trsm_bwd_split" : "trsm_bwd", sb, gb + vb, tf);
          HIPCHK(launch_trsm_bwd(X.G.p, X.DG.p, X.toffN.p, X.doffN.p, X.ntN.p, X.voffN.p, nsub,
                                 b, X.U.p, X.T.p, X.active.p, X.orderN.p, X.uNE, X.uNR,
                             tv(nact), ts(nact),
                                 sb));
        }
        {
          ProfScope ps("bapply", sb, 12.0 * X.nnzB + 2.0 * 8.0 * X.nbrows * b, 0.0);
          HIPCHK(launch_bapply(S->sub_ptr, X.brp.p, X.bcol.p, X.bval.p, X.brows.p, X.nbrows,
                               X.voffN.p, b, X.T.p, X.W.p, X.active.p, sb));
        }
        {
          ProfScope ps(ts(nact) > 1 ? "trsm_fwd_split" : "trsm_fwd", sb, gb + vb, tf);
          HIPCHK(launch_trsm_fwd(X.G.p, X.DG.p, X.toffN.p, X.doffN.p, X.ntN.p, X.voffN.p, nsub,
                                 b, X.W.p, X.T.p, X.active.p, X.orderN.p, X.uNE, X.uNR,
                             tv(nact), ts(nact),
                                 sb));
        }
        {
          ProfScope ps("cheb_combine", sb, 2.0 * vb, 0.0);
          HIPCHK(launch_cheb(X.P.p, X.U.p, X.T.p, k == 1 ? X.Y.p : X.P.p, X.theta.p, X.voffN.p,
                             X.ntN.p, nsub, b, LN.maxnt, false, X.active.p, sb));
        }
        std::swap(X.U.p, X.P.p);  // Z_{k+1} -> U, Z_k -> P
      }
    }
    {
      ProfScope ps("orth", sb, 2.0 * vb, 0.0);
      HIPCHK(launch_orth2(X.U.p, X.voffN.p, X.ntN.p, nsub, b, o.seed, it, X.active.p, wk, sb));
    }
  }
  if (!local_done) deferred_local();
  if (lag && !finished && sweeps > 0) read_active(sweeps);
  if (!shift_checked) {
    HIPCHK(hipStreamSynchronize(sb));
    check_shifted(X.pin_st2);
  }
  h->info.eig_sweeps = sweeps;
  if (nact > 0) {
    auto best = download(X.sbest.p, nsub, sb);
    int jw = -1;
    for (int j = 0; j < nsub; ++j)
      if (act[j] && (jw < 0 || best[j] > best[jw])) jw = j;
    char msg[256];
    snprintf(msg, sizeof msg,
             "%d subdomains did not converge in %d sweeps (subdomain %d: smallest largest-"
             "wanted Ritz residual %.3e of ||S||, eig_tol %.1e, eig_floor %.1e)",
             nact, o.eig_maxit, jw, best[jw], o.eig_tol, o.eig_floor);
    fail(GENEO_ERR_EIGEN_NOCONV, msg);
  }
  // eigenvectors p = G^{-T} y
  HIPCHK(launch_trsm_bwd(X.G.p, X.DG.p, X.toffN.p, X.doffN.p, X.ntN.p, X.voffN.p, nsub, b, X.Y.p,
                         X.T.p, nullptr, X.orderN.p, X.uNE, X.uNR, tv(nsub), ts(nsub), sb));
  HIPCHK(launch_select(X.theta.p, nsub, b, o.nev, o.tau, h->tau_sub.p, o.nev_max, o.sigma, h->m.p,
                       X.lam.p, sb));
  h->m_host = download(h->m.p, nsub, sb);
  h->lam_host = download(X.lam.p, (size_t)nsub * b, sb);
  tm[1].stop(sb);

  // ---- coarse basis Z, W = A_N Z, A_H = Z^T A Z
  tm[2].start(sb);
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
  h->zoff.upload(zoff, sb);
  h->coff.upload(coff, sb);
  h->Z.alloc(zs);
  HIPCHK(launch_basis(X.T.p, X.voffN.p, b, S->sub_ptr, S->pou, h->dmap.p, h->m.p, h->zoff.p,
                      h->nd.p, nsub, h->Z.p, sb));
  hipLaunchKernelGGL(k_max_resid, dim3(1), dim3(256), 0, sb, X.resid.p, h->m.p, nsub, b, X.mr.p);
  if (nc > 0) {
    X.woffd.upload(woff, sb);
    X.Wg.alloc(ws);
    int64_t maxwork = 0;
    for (int j = 0; j < nsub; ++j)
      maxwork = std::max<int64_t>(maxwork, (int64_t)h->nN_host[j] * h->m_host[j]);
    HIPCHK(launch_galerkin_w(An, S->sub_ptr, h->dmap.p, h->Z.p, h->zoff.p, h->m.p, X.woffd.p,
                             nsub, maxwork, X.Wg.p, sb));
    X.adj.alloc((size_t)nsub * nsub);
    HIPCHK(launch_adjacency(h->optr.p, h->olist.p, h->n, nsub, X.adj.p, sb));
    X.pcnt.alloc(nsub);
    X.poff.alloc(nsub + 1);
    X.npairs.alloc(1);
    HIPCHK(launch_pairs(X.adj.p, nsub, X.pcnt.p, X.poff.p, nullptr, X.npairs.p, sb, true));
    int np = download(X.npairs.p, 1, sb)[0];
    X.pairs.alloc(np);
    HIPCHK(launch_pairs(X.adj.p, nsub, X.pcnt.p, X.poff.p, X.pairs.p, X.npairs.p, sb, false));
    h->ntc = (nc + TS - 1) / TS;
    // tile envelope of A_H: its blocks are nonzero only for adjacent pairs
    // (the rows of subdomain i start at the first adjacent subdomain's
    // columns); box subdomains in lexicographic order make it banded
    // (without the option: E(t) = 0, dense)
    std::vector<int> envHE(h->ntc, 0), envHR(h->ntc, h->ntc - 1);
    if (o.envelope) {
      for (int t = 0; t < h->ntc; ++t) envHE[t] = t;
      const std::vector<int2> pr = download(X.pairs.p, np, sb);
      std::vector<int> first(nsub, nsub);
      for (const int2& q : pr)  // (i, j), j <= i
        if (h->m_host[q.y] > 0) first[q.x] = std::min(first[q.x], q.y);
      for (int i = 0; i < nsub; ++i)
        if (h->m_host[i] > 0 && first[i] < nsub)
          for (int r = coff[i]; r < coff[i + 1]; ++r)
            envHE[r / TS] = std::min(envHE[r / TS], coff[first[i]] / TS);
      for (int t = h->ntc - 2; t >= 0; --t) envHE[t] = std::min(envHE[t], envHE[t + 1]);
      for (int k = h->ntc - 1, i = h->ntc - 1; k >= 0; --k) {
        while (envHE[i] > k) --i;
        envHR[k] = i;
      }
      X.envHE.upload(envHE, sb);
      X.envHR.upload(envHR, sb);
    }
    X.AHt.alloc(tri_tiles(h->ntc) * TSQ);
    X.DH.alloc((size_t)h->ntc * TSQ);
    HIPCHK(launch_coarse_init(X.AHt.p, h->ntc, nc, sb));
    HIPCHK(launch_coarse_blocks(X.pairs.p, np, S->sub_ptr, S->sub_idx, h->didx.p, h->voffD.p,
                                h->nd.p, h->Z.p, h->zoff.p, X.Wg.p, X.woffd.p, h->m.p, h->coff.p,
                                X.AHt.p, sb));
    h->AHdense.alloc((size_t)nc * nc);
    HIPCHK(launch_coarse_to_dense(X.AHt.p, h->ntc, nc, h->AHdense.p, sb));
    tm[2].stop(sb);
    // ---- coarse Cholesky and inverse factor
    tm[3].start(sb);
    X.cst.alloc(1);
    X.cpiv.alloc(1);
    HIPCHK(launch_coarse_pivtol(X.AHt.p, nc, X.cpiv.p, sb));
    h->hnt.upload(std::vector<int>{h->ntc}, sb);
    h->htoff.upload(std::vector<int64_t>{0}, sb);
    X.hdoff.upload(std::vector<int64_t>{0}, sb);
    X.hjob.upload(std::vector<int>{0}, sb);
    {
      const EnvWork ew = env_work(envHE, std::vector<int64_t>{0}, std::vector<int>{h->ntc},
                                  std::vector<int>{0});
      ProfScope ps("coarse_chol", sb, 2.0 * 8.0 * TSQ * ew.tiles[0],
                   2.0 * TS * TS * TS * ew.prods + (double)TS * TS * TS * ew.tiles[0]);
      HIPCHK(launch_chol_steps(X.AHt.p, X.DH.p, h->htoff.p, X.hdoff.p, h->hnt.p, X.hjob.p, 1,
                               h->ntc, X.cst.p, sb, X.cpiv.p, o.envelope ? X.envHR.p : nullptr,
                               o.envelope ? envHR.data() : nullptr));
    }
    X.check_cst = true;  // read at the end of the setup (a failed factor only costs its inverse)
    h->bytes_symvH = 8.0 * packed(nc) + 16.0 * nc;
    std::vector<int2> tj = trtri_job_list(std::vector<int>{0}, std::vector<int>{h->ntc}, false);
    X.tjobsH.upload(tj, sb);
    std::vector<int2> lj = lauum_job_list(std::vector<int>{0}, std::vector<int>{h->ntc});
    X.ljobsH.upload(lj, sb);
    X.XTH.alloc(tri_tiles(h->ntc) * TSQ);
    HIPCHK(launch_trtri(false, X.AHt.p, X.DH.p, X.XTH.p, h->htoff.p, X.hdoff.p, h->hnt.p,
                        X.tjobsH.p, (int)tj.size(), o.envelope ? X.envHE.p : nullptr, sb));
    h->SH.alloc(tri_tiles(h->ntc) * TSQ);
    h->WH.alloc(tri_tiles(h->ntc) * TS);
    HIPCHK(launch_lauum(false, X.XTH.p, h->SH.p, h->htoff.p, h->hnt.p, X.ljobsH.p, (int)lj.size(),
                        sb));
    h->rH.alloc((size_t)h->ntc * TS);
    h->yH.alloc((size_t)h->ntc * TS);
    HIPCHK(hipMemsetAsync(h->rH.p, 0, h->rH.n * sizeof(double), sb));
    tm[3].stop(sb);
  } else {
    tm[2].stop(sb);
  }
}

void setup_impl(geneo_handle_s* h, const geneo_csr_t* A, const geneo_subdomains_t* S,
                const geneo_csr_batch_t* An, const geneo_csr_batch_t* Ao, hipStream_t st) {
  const geneo_opts_t& o = h->opts;
  const double t_start = now_ms();
  const int nsub = S->nsub;
  h->n = A->n;
  h->nsub = nsub;
  h->nloc = S->nloc;
  h->lpr = spmv_lanes(A);
  {
    DriverLock dl;
    HIPCHK(hipStreamCreateWithFlags(&h->hs, hipStreamNonBlocking));
  }
  if (o.tau_sub) {
    // the caller's host array is read here, during the call, and not kept
    std::vector<double> ts(o.tau_sub, o.tau_sub + nsub);
    for (double t : ts)
      if (!(t > 0)) fail(GENEO_ERR_ARG, "tau_sub entries must be positive");
    h->tau_sub.upload(ts, st);
    h->opts.tau_sub = nullptr;
  }
  struct ArenaScope {
    ArenaScope() { t_arena.begin(); }
    ~ArenaScope() { t_arena.end(); }
  } arena_scope;
  SetupScratch X;
  // Destroyed before X (and, on an error, before the handle): every kernel
  // the setup enqueued has finished before any of its buffers is released.
  struct StreamsDone {
    hipStream_t a, b;
    ~StreamsDone() {
      if (a) (void)hipStreamSynchronize(a);
      if (b) (void)hipStreamSynchronize(b);
    }
  } streams_done{st, h->hs};
  PhaseTimer tm0, tmL, tmC[4];

  // ---- 0. index lists, D_j maps, scaling, owner lists (stream st)
  tm0.start(st);
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
  X.ocount.alloc(h->n);
  h->optr.alloc(h->n + 1);
  h->olist.alloc(S->nloc);
  HIPCHK(launch_owners(S->sub_ptr, S->sub_idx, nsub, S->nloc, h->n, h->optr.p, X.ocount.p,
                       h->olist.p, st));
  h->xl.alloc(h->LD.nvec);
  h->yl.alloc(h->LD.nvec);
  tm0.stop(st);

  h->m_host.assign(nsub, 0);
  h->nc = 0;
  const bool coarse = o.coarse != 0;
  if (coarse && (!An || !Ao || !An->rowptr || !Ao->rowptr || !S->pou))
    fail(GENEO_ERR_ARG, "coarse space needs the Neumann and overlap matrices and the PoU");
  // The local Dirichlet factors (stream st) and the coarse-space work
  // (stream hs) are independent: both are enqueued so that they overlap.
  // The shifted factorization goes first on hs; the host then drives the
  // local phase (it reads back the pivot tests) and afterwards the eigen
  // sweeps, whose per-sweep readbacks only wait on hs.
  if (coarse) {
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, st));
    HIPCHK(hipStreamWaitEvent(h->hs, ev, 0));
    HIPCHK(hipEventDestroy(ev));
  }
  // Order: the FP32 local factorization runs alone (it fills the device);
  // the shifted factorization follows it on hs (an event orders them on the
  // device, the host meanwhile reads the pivot tests), and the inverse
  // factors, the FP64 refactors of the failed subdomains and their inverses
  // follow on st during the eigen sweeps, enqueued once few subdomains are
  // still sweeping (the sweeps then leave most CUs idle) rather than
  // competing with the factorization and the full sweeps.  Uploads go
  // through pinned staging, so the host drives both streams without
  // waiting on either.
  LocalLayout LN;
  tmL.start(st);
  std::function<void(hipStream_t)> local_step = setup_local(h, X, A, S, st, [&](hipEvent_t after) {
    if (coarse) setup_shifted(h, X, LN, S, An, Ao, h->hs, tmC, after);
  });
  const std::function<void()> local_rest = [&]() {
    local_step(st);
    tmL.stop(st);
  };
  if (coarse) setup_coarse(h, X, LN, S, An, Ao, h->hs, tmC, local_rest);
  else local_rest();
  HIPCHK(hipStreamSynchronize(st));
  {
    auto stat = download(X.status.p, nsub, st);
    for (int j : h->f64list)
      if (stat[j]) fail(GENEO_ERR_LOCAL_NOT_SPD, "local Dirichlet matrix of subdomain " +
                                                     std::to_string(j) + " is not SPD");
  }
  if (coarse) {
    HIPCHK(hipStreamSynchronize(h->hs));
    // read back once the stream has finished: sweep statistics and the
    // coarse factor's pivot test
    const auto fl = download(X.sflag.p, nsub, h->hs);
    int c = 0;
    for (int v : fl) c += v != 0;
    h->info.eig_stalled = c;
    h->info.eig_max_resid = download(X.mr.p, 1, h->hs)[0];
    if (X.check_cst && download(X.cst.p, 1, h->hs)[0])
      fail(GENEO_ERR_COARSE_NOT_SPD, "coarse matrix A_H is not SPD");
  }
  if (h->nc == 0) {
    // placeholders so that the apply kernels always get valid pointers
    if (!h->m.p) h->m.upload(std::vector<int>(nsub, 0), st);
    else HIPCHK(hipMemsetAsync(h->m.p, 0, nsub * sizeof(int), st));
    if (!h->zoff.p) h->zoff.upload(std::vector<int>(nsub, 0), st);
    if (!h->coff.p) h->coff.upload(std::vector<int>(nsub + 1, 0), st);
    if (!h->Z.p) h->Z.alloc(1);
    h->yH.alloc(1);
  }
  h->rz_part.alloc((size_t)(h->n + 255) / 256);
  h->oent.alloc(h->nloc);
  HIPCHK(owner_entries(h->olist.p, h->nloc, h->sub_ptr.p, h->dmap.p, h->voffD.p, h->zoff.p,
                       h->m.p, h->coff.p, h->oent.p, st));
  {
    {
      std::vector<int> j32, j64;
      for (const int2& jb : h->ljobs_host) (jb.y ? j64 : j32).push_back(jb.x);
      h->nlsj32 = (int)j32.size();
      h->nlsj64 = (int)j64.size();
      h->lsj32.upload(j32, st);
      h->lsj64.upload(j64, st);
    }
    if (h->local_form == GENEO_LOCAL_TRIANGULAR && local_solve_check(h->LD.maxnt) != hipSuccess)
      fail(GENEO_ERR_ARG, "local Dirichlet matrices of " + std::to_string(h->LD.maxnt * TS) +
                              " rows or more exceed the triangular local solves' LDS");
    std::vector<int2> aj;
    if (h->local_form == GENEO_LOCAL_INVERSE) aj = h->ljobs_host;
    if (h->nc > 0) aj.push_back(make_int2(nsub, 2));
    h->ajobs.upload(aj, st);
    h->najobs = (int)aj.size();
    h->amaxnt = std::max(h->local_form == GENEO_LOCAL_INVERSE ? h->LD.maxnt : 1,
                         h->nc > 0 ? h->ntc : 0);
    const int cw = symv_chunk_tiles();
    std::vector<int> cs(h->amaxnt + 1);
    for (int i = 0; i <= h->amaxnt; ++i) cs[i] = (int)symv_tasks_before(i, cw);
    h->nchunk = cs[h->amaxnt];
    h->cstart.upload(cs, st);
    h->Rpart.alloc((size_t)h->najobs * h->nchunk * TS);
    if ((int64_t)h->najobs * h->nchunk * TS > INT32_MAX)
      fail(GENEO_ERR_ARG, "too many row chunks for the symmetric product");
    // tasks of job q: its row chunks in row order, g consecutive chunks of
    // a row per task, generated on the device from one descriptor per job;
    // the two walk orders differ only in the order of the jobs
    auto build = [&](int g, bool both) {
      std::vector<SymvJob> js(h->najobs);
      std::vector<int64_t> cnt(h->najobs);
      for (int q = 0; q < h->najobs; ++q) {
        const int2 jb = aj[q];
        SymvJob& d = js[q];
        d.toff = 0;
        d.xoff = 0;
        d.nt = h->ntc;
        d.kind = jb.y;
        d.pad = 0;
        if (jb.y != 2) {
          d.toff = jb.y ? h->toff64_host[jb.x] : h->LD.toff[jb.x];
          d.xoff = h->LD.voff[jb.x];
          d.nt = h->LD.nt[jb.x];
        }
        cnt[q] = symv_tasks_before(d.nt, g * cw);
      }
      int64_t off = 0;
      for (int q = 0; q < h->najobs; ++q) {
        js[q].off_f = (int)off;
        off += cnt[q];
      }
      if (off > INT32_MAX) fail(GENEO_ERR_ARG, "too many tasks for the symmetric product");
      int64_t offr = 0;
      for (int q = h->najobs - 1; q >= 0; --q) {
        js[q].off_r = (int)offr;
        offr += cnt[q];
      }
      h->ntasks = (int)off;
      h->symv_jobs.upload(js, st);
      h->tasks_fwd.alloc(std::max<int64_t>(off, 1));
      if (both) h->tasks_rev.alloc(std::max<int64_t>(off, 1));
      HIPCHK(symv_make_tasks(h->symv_jobs.p, h->najobs, g, h->nchunk, h->tasks_fwd.p,
                             both ? h->tasks_rev.p : nullptr, st));
    };
    int g = o.symv_tiles / cw;
    if (g == 0) g = h->najobs > 0 ? tune_symv_group(h, st, build) : 1;
    build(g, true);
    h->info.symv_tiles = g * cw;
  }
  HIPCHK(hipStreamSynchronize(st));
  if (h->local_form == GENEO_LOCAL_INVERSE) {
    // the apply reads only the inverses
    h->L32.release();
    h->D32.release();
    h->L64.release();
    h->D64.release();
  }
  h->info.local_solve = h->local_form;
  h->info.t_phase_ms[0] = tm0.ms();
  h->info.t_phase_ms[1] = tmL.ms();
  if (coarse) {
    h->info.t_phase_ms[2] = tmC[0].ms();
    h->info.t_phase_ms[3] = tmC[1].ms();
    h->info.t_phase_ms[4] = tmC[2].ms();
    h->info.t_phase_ms[5] = tmC[3].ms();
  }
  h->info.nsub = nsub;
  h->info.nc = h->nc;
  h->info.t_setup_ms = now_ms() - t_start;
}

void ensure_pcg(geneo_handle_s* h, int maxit) {
  if (h->pcg_cap < h->n) {
    h->r.alloc(h->n);
    h->z.alloc(h->n);
    h->p.alloc(h->n);
    h->p2.alloc(h->n);
    h->q.alloc(h->n);
    h->partial.alloc(std::max(PCG_NB, PCG_NB_SPMV));
    h->rr_part.alloc(PCG_NB);
    h->sc.alloc(1);
    h->done.alloc(1);
    h->xs.alloc(h->n);
    h->rb.alloc(h->n);
    h->pcg_cap = h->n;
  }
  if (!h->hflag) {
    h->hflag = (int*)PinnedPool::get().take(2 * sizeof(int));
    h->hsc = (PcgScalars*)PinnedPool::get().take(3 * sizeof(PcgScalars));
    if (!h->hflag || !h->hsc) fail(GENEO_ERR_OOM, "pinned host memory for the PCG flags");
    for (hipEvent_t& e : h->fev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (h->pcg_maxit < maxit + 1) {
    h->alphas.alloc(maxit + 1);
    h->betas.alloc(maxit + 1);
    PinnedPool::get().give(h->hab);
    h->hab = (double*)PinnedPool::get().take(2 * (size_t)(maxit + 1) * sizeof(double));
    if (!h->hab) fail(GENEO_ERR_OOM, "pinned host memory for the PCG records");
    h->pcg_maxit = maxit + 1;
  }
}

#define PCG_CHUNK 8
#define PCG_TAIL 2

PcgWork handle_work(geneo_handle_s* h) {
  PcgWork w;
  w.r = h->r.p;
  w.z = h->z.p;
  w.p = h->p.p;
  w.p2 = h->p2.p;
  w.q = h->q.p;
  w.partial = h->partial.p;
  w.rr_part = h->rr_part.p;
  w.alphas = h->alphas.p;
  w.betas = h->betas.p;
  w.sc = h->sc.p;
  w.done = h->done.p;
  w.cap = h->pcg_maxit;
  return w;
}

// PCG start, all on the device (stream st): b.b and tol2, r = b - A x, r.r
// (done when already converged), z = M^{-1} r (which also leaves the r.z
// partial sums that the first alpha needs).
void pcg_enqueue_start(geneo_handle_s* h, const geneo_csr_t* A, const double* b, const double* x,
                       double rtol, int maxit, const PcgWork& w, hipStream_t st) {
  const int n = h->n;
  HIPCHK(dot_partial(b, b, n, w.partial, nullptr, st));
  HIPCHK(pcg_start(w.partial, 0, w.sc, w.done, rtol * rtol, maxit, st));
  HIPCHK(spmv(A, x, w.q, h->lpr, nullptr, st));
  HIPCHK(residual0(b, w.q, w.r, n, st));
  HIPCHK(dot_partial(w.r, w.r, n, w.partial, nullptr, st));
  HIPCHK(pcg_start(w.partial, 1, w.sc, w.done, rtol * rtol, maxit, st));
  HIPCHK(apply_enqueue(h, w.r, w.z, w.done, st, nullptr, false));
}

// Global PCG iteration it (0-based): p = z + beta p (from the buffer of
// parity it into the other), q = A p, x and r updated with alpha, the
// convergence check and z = M^{-1} r; every kernel returns at once when
// done is set.  The apply walks the subdomains in reverse order on even
// iterations.
void pcg_enqueue_iteration(geneo_handle_s* h, const geneo_csr_t* A, double* x, const PcgWork& w,
                           int it, hipStream_t st) {
  const int n = h->n;
  const int nrz = (n + 255) / 256;
  double* pb[2] = {w.p, w.p2};
  double* pk = pb[(it + 1) & 1];
  HIPCHK(p_spmv(A, h->lpr, w.z, pb[it & 1], pk, w.q, h->rz_part.p, nrz, w.sc, w.betas, w.partial,
                PCG_NB_SPMV, w.done, st));
  HIPCHK(update_xr_alpha(x, w.r, pk, w.q, n, w.partial, PCG_NB_SPMV, h->rz_part.p, nrz, w.sc,
                         w.alphas, w.rr_part, w.done, st));
  HIPCHK(apply_enqueue(h, w.r, w.z, w.done, st, &w, (it & 1) == 0));
}

// Condition estimate from the CG coefficients: extreme eigenvalues of the
// Lanczos tridiagonal T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1},
// T_{k,k+1} = sqrt(beta_k)/alpha_k, in the caller's d / e storage (iters
// and iters - 1 entries).
double kappa_from_cg(const double* al, const double* be, int iters, double* d, double* e) {
  if (iters <= 0) return 1.0;
  for (int i = 0; i < iters; ++i) {
    d[i] = 1.0 / al[i] + (i > 0 ? be[i - 1] / al[i - 1] : 0.0);
    if (i + 1 < iters) e[i] = sqrt(be[i]) / al[i];
  }
  const double lmin = tridiag_eig(d, e, iters, 0), lmax = tridiag_eig(d, e, iters, iters - 1);
  return lmin > 0 ? lmax / lmin : INFINITY;
}

// Two graphs, of PCG_CHUNK and PCG_TAIL iterations on the iterate h->xs:
// 6 launches each (p update with beta, SpMV and p.Ap; x/r update with
// alpha; check + apply input; symmetric product and its column sums;
// combine with r.z).  p alternates between two buffers (both lengths are
// even, so every replay starts on the first and runs the launches of the
// global iterations of the same parity).  Every kernel returns at once
// when done is set.  Captured at the first solve and again only when the
// matrix or a work buffer has changed: b, rtol and maxit reach the
// iterations through the device scalars, not through the graphs.
void pcg_graphs(geneo_handle_s* h, const geneo_csr_t* A, const PcgWork& w, hipStream_t st) {
  const void* key[6] = {A->rowptr, A->col, A->val, (const void*)(intptr_t)A->n, h->xs.p, w.alphas};
  if (h->gexec[0] && std::equal(key, key + 6, h->gkey)) return;
  for (hipGraphExec_t& e : h->gexec)
    if (e) {
      (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
  // an error inside a capture ends it, so that the stream stays usable
  struct Capture {
    hipStream_t st;
    bool on = false;
    ~Capture() {
      if (!on) return;
      hipGraph_t g = nullptr;
      if (hipStreamEndCapture(st, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    }
  };
  std::shared_lock<std::shared_mutex> capture_lock(g_capture_mu);
  for (int gi = 0; gi < 2; ++gi) {
    hipGraph_t graph = nullptr;
    Capture cap{st};
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    cap.on = true;
    for (int k = 0; k < (gi ? PCG_TAIL : PCG_CHUNK); ++k)
      pcg_enqueue_iteration(h, A, h->xs.p, w, k, st);
    cap.on = false;
    HIPCHK(hipStreamEndCapture(st, &graph));
    const hipError_t ie = hipGraphInstantiate(&h->gexec[gi], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(ie);
  }
  std::copy(key, key + 6, h->gkey);
}

// One PCG solve on the handle's stream.  correction = false: x (start
// vector in, solution out) is copied to the graphs' iterate and back;
// correction = true: the iterate starts at 0 and is added to x at the end
// (a refinement step for A d = b).
void pcg_one(geneo_handle_s* h, const geneo_csr_t* A, const double* b, double* x, double rtol,
             int maxit, geneo_pcg_info_t* info, bool correction = false) {
  hipStream_t st = h->hs;
  double t0 = now_ms();
  const PcgWork w = handle_work(h);
  const size_t nb = (size_t)h->n * sizeof(double);
  if (correction) HIPCHK(hipMemsetAsync(h->xs.p, 0, nb, st));
  else HIPCHK(hipMemcpyAsync(h->xs.p, x, nb, hipMemcpyDeviceToDevice, st));
  pcg_enqueue_start(h, A, b, h->xs.p, rtol, maxit, w, st);
  pcg_graphs(h, A, w, st);
  hipGraphExec_t* ex = h->gexec;
  // Up to two chunks in flight: after each launch the done flag and the
  // scalars are copied to pinned memory, and the host reads a chunk's copy
  // while the next chunk runs, so the device never waits for the host.
  // From the residual history the host predicts the iterations left: no
  // chunk is queued that the chunks in flight are expected to make
  // unnecessary, and the last iterations go in short chunks, which bounds
  // the launches that find done set (each costs a few microseconds).
  struct Slot { int iters; };
  Slot fl[2];
  int head = 0, nfl = 0, queued = 0;  // queued: iterations launched so far
  const int cap = maxit + PCG_CHUNK;
  auto launch = [&](bool tail) {
    const int sl = (head + nfl) & 1;
    HIPCHK(hipGraphLaunch(ex[tail ? 1 : 0], st));
    HIPCHK(hipMemcpyAsync(&h->hflag[sl], h->done.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&h->hsc[sl], h->sc.p, sizeof(PcgScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(h->fev[sl], st));
    fl[sl].iters = tail ? PCG_TAIL : PCG_CHUNK;
    queued += fl[sl].iters;
    ++nfl;
  };
  double rr_a = -1.0;
  int it_a = 0;
  int64_t left = INT64_MAX;  // predicted iterations still needed after the last read
  launch(false);
  for (;;) {
    int ahead = 0;
    for (int u = 0; u < nfl; ++u) ahead += fl[(head + u) & 1].iters;
    if (nfl < 2 && queued < cap && left > ahead)
      launch(left - ahead <= PCG_CHUNK);
    if (nfl == 0) break;  // nothing in flight and nothing worth launching
    HIPCHK(hipEventSynchronize(h->fev[head]));
    const int dn = h->hflag[head];
    const PcgScalars sc = h->hsc[head];
    head ^= 1;
    --nfl;
    if (dn) break;
    // geometric fit of the residual decrease over the last two reads
    left = INT64_MAX;
    if (rr_a > 0.0 && sc.rr > 0.0 && sc.iters > it_a && sc.rr < rr_a && sc.tol2 > 0.0) {
      const double f = std::log(sc.rr / rr_a) / (sc.iters - it_a);  // per iteration
      const double need = std::log(sc.tol2 / sc.rr) / f;
      if (need >= 0.0 && need < 1e9) left = (int64_t)std::ceil(need);
    }
    rr_a = sc.rr;
    it_a = sc.iters;
    if (nfl == 0 && left <= 0) left = 1;  // never stop on a prediction alone
    if (nfl == 0 && queued >= cap) break;
  }
  if (correction) HIPCHK(add_into(x, h->xs.p, h->n, st));
  else HIPCHK(hipMemcpyAsync(x, h->xs.p, nb, hipMemcpyDeviceToDevice, st));
  // drain: every launch is complete before the handle's buffers are read
  // the scalars and the alpha / beta records (for the Lanczos estimate of
  // kappa), read back together
  const size_t nab = (size_t)std::min(maxit + 1, h->pcg_maxit);
  HIPCHK(hipMemcpyAsync(&h->hsc[2], h->sc.p, sizeof(PcgScalars), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(h->hab, h->alphas.p, nab * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(h->hab + h->pcg_maxit, h->betas.p, nab * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const PcgScalars s = h->hsc[2];
  const int iters = s.iters, converged = s.converged;
  const double rr = s.rr, bb = s.bb;
  info->iters = iters;
  info->converged = converged;
  info->relres = bb > 0 ? sqrt(rr / bb) : 0.0;
  {
    std::vector<double> d(std::max(iters, 1)), e(std::max(iters, 1));
    info->kappa_est = kappa_from_cg(h->hab, h->hab + h->pcg_maxit, iters, d.data(), e.data());
  }
  info->t_solve_ms = now_ms() - t0;
}

// |b - A x| / |b| with the residual summed in double-double (rb: work
// vector of n, partial: PCG_NB partial sums, host: PCG_NB host doubles).
double true_relres(const geneo_csr_t* A, const double* b, const double* x, double* rb,
                   double* partial, double* host, hipStream_t st) {
  const int n = A->n;
  double num = 0.0, den = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 0) {
      HIPCHK(residual_dd(A, b, x, rb, st));
      HIPCHK(dot_partial(rb, rb, n, partial, nullptr, st));
    } else {
      HIPCHK(dot_partial(b, b, n, partial, nullptr, st));
    }
    HIPCHK(hipMemcpyAsync(host, partial, PCG_NB * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double t = 0.0;
    for (int i = 0; i < PCG_NB; ++i) t += host[i];
    (pass == 0 ? num : den) = t;
  }
  return den > 0 ? sqrt(num / den) : 0.0;
}

// Iterative refinement after a solve (opts.refine steps): r = b - A x in
// double-double, A d = r by PCG to refine_rtol |r| (solve(b, x, rtol, info,
// correction)), x += d.  The attainable accuracy of x then no longer rests
// on the FP64 rounding of the residual (u kappa(A) for a plain FP64 PCG).
template <typename Solve>
void refine_solution(geneo_handle_s* h, const geneo_csr_t* A, const double* b, double* x,
                     double* rb, geneo_pcg_info_t* info, hipStream_t st, Solve&& solve) {
  info->refine_iters = 0;
  for (int k = 0; k < h->opts.refine; ++k) {
    HIPCHK(residual_dd(A, b, x, rb, st));
    geneo_pcg_info_t ci{};
    solve(rb, x, h->opts.refine_rtol, &ci);
    info->refine_iters += ci.iters;
    if (ci.iters == 0) break;  // the residual is zero or already negligible
  }
}

int finish(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// ------------------------------------------------- allocation-free solve
// The work of pcg_solve_noalloc lives in one fixed device array per GPU,
// laid out as: r, z, p, p2, q, the refinement correction d and residual
// (kNoallocMaxN doubles each), the partial sums (PCG_NB_SPMV, then PCG_NB),
// the alpha and beta records (kNoallocMaxIt + 1 each), the scalars and the
// done flag; every piece starts on a 256-byte boundary.  56.1 MiB in all.
constexpr int kNoallocMaxN = 1 << 20;
constexpr int kNoallocMaxIt = 4096;
constexpr int64_t kAlign = 32;  // doubles
constexpr int64_t al_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
constexpr int64_t kOffPartial = 7 * (int64_t)kNoallocMaxN;
constexpr int64_t kOffRr = kOffPartial + al_up(PCG_NB_SPMV > PCG_NB ? PCG_NB_SPMV : PCG_NB);
constexpr int64_t kOffAlpha = kOffRr + al_up(PCG_NB);
constexpr int64_t kOffBeta = kOffAlpha + al_up(kNoallocMaxIt + 1);
constexpr int64_t kOffSc = kOffBeta + al_up(kNoallocMaxIt + 1);
constexpr int64_t kOffDone = kOffSc + al_up((sizeof(PcgScalars) + 7) / 8);
constexpr int64_t kScratchDoubles = kOffDone + kAlign;

}  // namespace

// file scope: its device address is taken once per device (below)
static __device__ __align__(256) double pcg_scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of pcg_scratch on the current device, looked up once per
// device with that device current (each device holds its own copy).
double* scratch_on_current_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(GENEO_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(pcg_scratch)));
    g_scratch_dev[dev] = (double*)ptr;
  }
  return g_scratch_dev[dev];
}

// alpha / beta records and the Lanczos tridiagonal of the last solve, per
// host thread (no host allocation during the solve)
thread_local double t_noalloc_ab[2 * (kNoallocMaxIt + 1)];
thread_local double t_noalloc_de[2 * (kNoallocMaxIt + 1)];
thread_local double t_noalloc_part[PCG_NB];

// PCG without graphs, on the caller's stream: chunks of PCG_CHUNK
// iterations are enqueued and the done flag is read after each, so past
// convergence at most one chunk of launches finds done set.  The launches
// are those of pcg_one in the same order, hence the same results.  The
// correction mode iterates on d (from 0) and adds it to x at the end.
void pcg_one_noalloc(geneo_handle_s* h, const geneo_csr_t* A, const double* b, double* x,
                     double rtol, int maxit, geneo_pcg_info_t* info, const PcgWork& w,
                     hipStream_t st, double* d = nullptr) {
  const double t0 = now_ms();
  double* xi = x;
  if (d) {
    HIPCHK(hipMemsetAsync(d, 0, (size_t)h->n * sizeof(double), st));
    xi = d;
  }
  pcg_enqueue_start(h, A, b, xi, rtol, maxit, w, st);
  int it = 0;
  PcgScalars hs{};
  int hdone = 0;
  for (;;) {
    for (int k = 0; k < PCG_CHUNK; ++k) pcg_enqueue_iteration(h, A, xi, w, it++, st);
    HIPCHK(hipMemcpyAsync(&hdone, w.done, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hdone || it >= maxit + PCG_CHUNK) break;
  }
  if (d) HIPCHK(add_into(x, d, h->n, st));
  HIPCHK(hipMemcpyAsync(&hs, w.sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, st));
  const int nab = std::min(maxit + 1, kNoallocMaxIt + 1);
  HIPCHK(hipMemcpyAsync(t_noalloc_ab, w.alphas, nab * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(t_noalloc_ab + kNoallocMaxIt + 1, w.betas, nab * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  info->iters = hs.iters;
  info->converged = hs.converged;
  info->relres = hs.bb > 0 ? sqrt(hs.rr / hs.bb) : 0.0;
  info->kappa_est = kappa_from_cg(t_noalloc_ab, t_noalloc_ab + kNoallocMaxIt + 1, hs.iters,
                                  t_noalloc_de, t_noalloc_de + kNoallocMaxIt + 1);
  info->t_solve_ms = now_ms() - t0;
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
  o->eig_tol = 1e-8;
  o->eig_maxit = 300;
  o->eig_block = 0;
  o->seed = 0;
  o->coarse = 1;
  o->eig_stall = 10;
  o->eig_floor = 1e-6;
  o->eig_cheb = 4;
  o->symv_tiles = 0;
  o->tau_sub = nullptr;
  o->refine = 0;
  o->refine_rtol = 1e-6;
  o->eig_solve = 0;
  o->eig_split = 0;
  o->envelope = 1;
  o->shifted_steps = 0;
  o->local_solve = 0;
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

int geneo_q1_thm1_tau(const geneo_grid_t* grid, double* tau) {
  if (!tau) return finish(GENEO_ERR_ARG, "tau is NULL");
  Q1Geom g;
  std::string err;
  int rc = q1_make_geom(grid, &g, &err);
  if (rc) return finish(rc, err);
  q1_thm1_tau(g, tau);
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
    dg.release();
    nzoff.release();
    settle_thread();
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
    if (o.coarse && ((o.tau > 0 || o.tau_sub) ? o.nev_max < 1 : o.nev < 0))
      fail(GENEO_ERR_ARG, "invalid eigenvector count");
    if (o.eig_block && (o.eig_block % 16 || o.eig_block > 64))
      fail(GENEO_ERR_ARG, "eig_block must be a multiple of 16 up to 64");
    if (o.eig_maxit < 1 || !(o.eig_tol > 0) || o.eig_stall < 0 || !(o.eig_floor >= 0))
      fail(GENEO_ERR_ARG, "invalid eigen tolerances");
    if (o.eig_cheb < 0 || o.eig_cheb > 6)
      fail(GENEO_ERR_ARG, "eig_cheb must be 0..6");
    if (o.symv_tiles != 0 && o.symv_tiles != 8 && o.symv_tiles != 16 && o.symv_tiles != 32)
      fail(GENEO_ERR_ARG, "symv_tiles must be 0, 8, 16 or 32");
    if (o.refine < 0 || o.refine > 8 || !(o.refine_rtol > 0 && o.refine_rtol < 1))
      fail(GENEO_ERR_ARG, "refine must be 0..8 with 0 < refine_rtol < 1");
    if (o.eig_solve < 0 || o.eig_solve > trsm_variants())
      fail(GENEO_ERR_ARG, "eig_solve must be 0 .. " + std::to_string(trsm_variants()));
    if (o.eig_split < -1) fail(GENEO_ERR_ARG, "eig_split must be -1, 0 or positive");
    if (o.envelope < 0 || o.envelope > 2) fail(GENEO_ERR_ARG, "envelope must be 0, 1 or 2");
    if (o.shifted_steps < -1 || o.shifted_steps > 1)
      fail(GENEO_ERR_ARG, "shifted_steps must be -1, 0 or 1");
    if (o.local_solve < 0 || o.local_solve > 2)
      fail(GENEO_ERR_ARG, "local_solve must be 0, 1 or 2");
    setup_impl(h.get(), A, S, An, Ao, (hipStream_t)stream);
    *out = h.release();
    settle_thread();  // the setup's scratch blocks become reusable
    return GENEO_OK;
  } catch (Err& e) {
    // setup_impl synchronised its streams before its buffers were released
    settle_thread();
    return finish(e.code, e.msg);
  }
}

int geneo_apply(geneo_handle_t h, const double* r, double* z, void* stream) {
  if (!h || !r || !z || r == z) return finish(GENEO_ERR_ARG, "invalid apply arguments");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = apply_enqueue(h, r, z, nullptr, st, nullptr, h->apply_rev);
  h->apply_rev = !h->apply_rev;
  if (e == hipSuccess) {
    // remember the stream's last use of the handle for geneo_destroy
    auto it = h->apply_ev.find(st);
    if (it == h->apply_ev.end()) {
      hipEvent_t ev = nullptr;
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) it = h->apply_ev.emplace(st, ev).first;
    }
    if (e == hipSuccess) e = hipEventRecord(it->second, st);
  }
  if (e != hipSuccess) return finish(GENEO_ERR_HIP, hipGetErrorString(e));
  return GENEO_OK;
}

void geneo_destroy(geneo_handle_t h) {
  if (!h) return;
  // the work enqueued with the handle: its own stream and the streams of
  // the geneo_apply calls (an event recorded after each)
  if (h->hs) (void)hipStreamSynchronize(h->hs);
  for (auto& se : h->apply_ev) (void)hipEventSynchronize(se.second);
  delete h;
  settle_thread();
}

int geneo_trim(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return finish(GENEO_ERR_HIP, "hipGetDevice failed");
  settle_thread();
  DevCache::get().trim(dev);
  return GENEO_OK;
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

int geneo_get_local_precision(geneo_handle_t h, int* fp64) {
  if (!h || !fp64) return finish(GENEO_ERR_ARG, "NULL argument");
  for (int j = 0; j < h->nsub; ++j) fp64[j] = h->ljobs_host[j].y;
  return GENEO_OK;
}

int geneo_get_coarse(geneo_handle_t h, int64_t* zoff, double* z, int64_t zsize, double* ah) {
  if (!h || !zoff) return finish(GENEO_ERR_ARG, "NULL argument");
  try {
    hipStream_t st = h->hs;
    int64_t tot = 0;
    for (int j = 0; j < h->nsub; ++j) {
      zoff[j] = tot;
      tot += (int64_t)h->nN_host[j] * h->m_host[j];
    }
    zoff[h->nsub] = tot;
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
    std::vector<double> host(PCG_NB);
    for (int k = 0; k < nrhs; ++k) {
      const double* bk = b + (int64_t)k * h->n;
      double* xk = x + (int64_t)k * h->n;
      const double t0 = now_ms();
      pcg_one(h, A, bk, xk, rtol, maxit, &info[k]);
      if (!info[k].converged) rc = GENEO_ERR_MAXIT;
      refine_solution(h, A, bk, xk, h->rb.p, &info[k], h->hs,
                      [&](const double* rb, double* xx, double rt, geneo_pcg_info_t* ci) {
                        pcg_one(h, A, rb, xx, rt, maxit, ci, true);
                      });
      info[k].true_relres = true_relres(A, bk, xk, h->rb.p, h->partial.p, host.data(), h->hs);
      info[k].t_solve_ms = now_ms() - t0;
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

int pcg_solve_noalloc(const geneo_csr_t* A, geneo_handle_t h, const double* b, double* x,
                      int nrhs, double rtol, int maxit, geneo_pcg_info_t* info, void* stream) {
  try {
    check_csr(A);
    if (!h || !b || !x || !info || nrhs < 1 || maxit < 1 || !(rtol > 0))
      fail(GENEO_ERR_ARG, "invalid pcg arguments");
    if (A->n != h->n) fail(GENEO_ERR_ARG, "matrix size differs from the preconditioner's");
    if (h->n > kNoallocMaxN || maxit > kNoallocMaxIt)
      fail(GENEO_ERR_ARG, "pcg_solve_noalloc is limited to n <= " +
                              std::to_string(kNoallocMaxN) + " and maxit <= " +
                              std::to_string(kNoallocMaxIt) + " (got n = " +
                              std::to_string(h->n) + ", maxit = " + std::to_string(maxit) + ")");
    hipStream_t st = (hipStream_t)stream;
    double* s0 = scratch_on_current_device();
    PcgWork w;
    w.r = s0;
    w.z = s0 + kNoallocMaxN;
    w.p = s0 + 2 * (int64_t)kNoallocMaxN;
    w.p2 = s0 + 3 * (int64_t)kNoallocMaxN;
    w.q = s0 + 4 * (int64_t)kNoallocMaxN;
    w.partial = s0 + kOffPartial;
    w.rr_part = s0 + kOffRr;
    w.alphas = s0 + kOffAlpha;
    w.betas = s0 + kOffBeta;
    w.sc = (PcgScalars*)(s0 + kOffSc);
    w.done = (int*)(s0 + kOffDone);
    w.cap = kNoallocMaxIt + 1;
    double* dvec = s0 + 5 * (int64_t)kNoallocMaxN;
    double* rvec = s0 + 6 * (int64_t)kNoallocMaxN;
    int rc = GENEO_OK;
    for (int k = 0; k < nrhs; ++k) {
      const double* bk = b + (int64_t)k * h->n;
      double* xk = x + (int64_t)k * h->n;
      const double t0 = now_ms();
      pcg_one_noalloc(h, A, bk, xk, rtol, maxit, &info[k], w, st);
      if (!info[k].converged) rc = GENEO_ERR_MAXIT;
      refine_solution(h, A, bk, xk, rvec, &info[k], st,
                      [&](const double* rb, double* xx, double rt, geneo_pcg_info_t* ci) {
                        pcg_one_noalloc(h, A, rb, xx, rt, maxit, ci, w, st, dvec);
                      });
      info[k].true_relres = true_relres(A, bk, xk, rvec, w.partial, t_noalloc_part, st);
      info[k].t_solve_ms = now_ms() - t0;
    }
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
