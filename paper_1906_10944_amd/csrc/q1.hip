// Structured Q1 assembly on the device (serendipity bricks: s20.hip): the
// global stiffness matrix of the
// Darcy form (eq. (2)) or the elasticity form (eq. (3), no traction) with
// symmetric elimination of homogeneous Dirichlet conditions, the load
// vector, the overlapping box subdomains (Sec. 3) with their sets, the
// piecewise-constant partition of unity (Def. 3, Sec. 4.3) and the batched
// local Neumann and overlap-zone matrices (Sec. 4.3).
//
// Every output entry is produced by one thread that gathers the element
// contributions it needs, so the result is deterministic (no atomics).
#include "q1.h"

namespace geneo {

// ------------------------------------------------------------ geometry ---
__device__ __forceinline__ int nbcount(int i, int nn) { return (i > 0) + 1 + (i < nn - 1); }
// sum_{i' < i} nbcount(i')
__device__ __forceinline__ int64_t nbprefix(int i, int nn) { return i == 0 ? 0 : 3 * (int64_t)i - 1; }
__device__ __forceinline__ int64_t nbtotal(int nn) { return nn == 1 ? 1 : 3 * (int64_t)nn - 2; }

// Element matrix entry between vertex a (component c) and vertex b
// (component cb) of element e.
__device__ double elem_entry(const Q1Geom& g, const double* coeff, int64_t e, int a, int c,
                             int b, int cb) {
  // (rounded product, never fused into the caller's sum)
  if (g.ncomp == 1) return __dmul_rn(coeff[e], g.kref[a][b]);
  // strain rows fed by displacement component c, with the gradient axis:
  // c=0: (e11,x) (g13,z) (g12,y); c=1: (e22,y) (g23,z) (g12,x); c=2: (e33,z) (g23,y) (g13,x)
  const int srow[3][3] = {{0, 4, 5}, {1, 3, 5}, {2, 3, 4}};
  const int gax[3][3] = {{0, 2, 1}, {1, 2, 0}, {2, 1, 0}};
  const double* C21 = coeff + 21 * e;
  double Cm[3][3];
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      int s = srow[c][u], t = srow[cb][v];
      int lo = s < t ? s : t, hi = s < t ? t : s;
      Cm[u][v] = C21[lo * (11 - lo) / 2 + hi];
    }
  double sum = 0.0;
  for (int q = 0; q < 8; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      double gu = g.grad[q][a][gax[c][u]];
#pragma unroll
      for (int v = 0; v < 3; ++v) acc += gu * Cm[u][v] * g.grad[q][b][gax[cb][v]];
    }
    sum += g.wq[q] * acc;
  }
  return sum;
}

__device__ __forceinline__ void node_coords(const Q1Geom& g, int64_t k, int* x) {
  x[0] = (int)(k % g.nn[0]);
  int64_t r = k / g.nn[0];
  x[1] = (int)(r % g.nn[1]);
  x[2] = (int)(r / g.nn[1]);
}

__device__ __forceinline__ bool node_dirichlet(const Q1Geom& g, const int* x) {
  for (int ax = 0; ax < g.dim; ++ax) {
    if (((g.dirichlet >> (2 * ax)) & 1) && x[ax] == 0) return true;
    if (((g.dirichlet >> (2 * ax + 1)) & 1) && x[ax] == g.ne[ax]) return true;
  }
  return false;
}

// Value of (row node x, comp c) x (col node y, comp cb) summed over the
// elements in the element box [blo, bhi) that contain both nodes, and, if
// ovl_only, whose multiplicity is at least two; the contributions are added
// in ascending element order, from 0.
__device__ double pair_value(const Q1Geom& g, const double* coeff, const int* x, int c,
                             const int* y, int cb, const int* blo, const int* bhi,
                             bool ovl_only) {
  int lo[3], hi[3];
  for (int ax = 0; ax < 3; ++ax) {
    if (ax >= g.dim) { lo[ax] = 0; hi[ax] = 0; continue; }
    // elements containing both nodes along this axis
    int a0 = max(x[ax], y[ax]) - 1, a1 = min(x[ax], y[ax]);
    a0 = max(a0, blo[ax]);
    a1 = min(a1, bhi[ax] - 1);
    lo[ax] = a0;
    hi[ax] = a1;
    if (a0 > a1) return 0.0;
  }
  double s = 0.0;
  for (int ez = lo[2]; ez <= hi[2]; ++ez)
    for (int ey = lo[1]; ey <= hi[1]; ++ey)
      for (int ex = lo[0]; ex <= hi[0]; ++ex) {
        int ee[3] = {ex, ey, ez};
        if (ovl_only) {
          int m = 1;
          for (int ax = 0; ax < g.dim; ++ax) {
            int cnt = 0;
            for (int p = 0; p < g.parts[ax]; ++p)
              cnt += (g.elo[ax][p] <= ee[ax] && ee[ax] < g.ehi[ax][p]);
            m *= cnt;
          }
          if (m < 2) continue;
        }
        int a = 0, b = 0;
        for (int ax = 0; ax < g.dim; ++ax) {
          a |= (x[ax] - ee[ax]) << ax;
          b |= (y[ax] - ee[ax]) << ax;
        }
        int64_t e = ex + (int64_t)g.ne[0] * (ey + (int64_t)g.ne[1] * ez);
        s = __dadd_rn(s, elem_entry(g, coeff, e, a, c, b, cb));
      }
  return s;
}

// ------------------------------------------------------- global matrix ---
__global__ void k_q1_global(const Q1Geom* __restrict__ gp, const double* __restrict__ coeff,
                            int* __restrict__ rowptr, int* __restrict__ col,
                            double* __restrict__ val, double* __restrict__ rhs, int64_t nrows) {
  const Q1Geom& g = *gp;
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int nc = g.ncomp;
  int64_t k = r / nc;
  int c = (int)(r % nc);
  int x[3];
  node_coords(g, k, x);
  int nb[3];
  for (int ax = 0; ax < 3; ++ax) nb[ax] = nbcount(x[ax], g.nn[ax]);
  int64_t pre = nbprefix(x[2], g.nn[2]) * nbtotal(g.nn[1]) * nbtotal(g.nn[0]) +
                (int64_t)nb[2] * nbprefix(x[1], g.nn[1]) * nbtotal(g.nn[0]) +
                (int64_t)nb[2] * nb[1] * nbprefix(x[0], g.nn[0]);
  int rowlen = nc * nb[0] * nb[1] * nb[2];
  int64_t start = (int64_t)nc * nc * pre + (int64_t)c * rowlen;
  rowptr[r] = (int)start;
  if (r == nrows - 1) rowptr[nrows] = (int)(start + rowlen);
  const bool rdir = node_dirichlet(g, x);
  int blo[3] = {0, 0, 0}, bhi[3] = {g.ne[0], g.ne[1], g.ne[2]};
  int64_t pos = start;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int y[3] = {x[0] + dx, x[1] + dy, x[2] + dz};
        bool ok = true;
        for (int ax = 0; ax < 3; ++ax) ok = ok && y[ax] >= 0 && y[ax] < g.nn[ax];
        if (!ok) continue;
        int64_t kk = y[0] + (int64_t)g.nn[0] * (y[1] + (int64_t)g.nn[1] * y[2]);
        bool cdir = node_dirichlet(g, y);
        for (int cb = 0; cb < nc; ++cb) {
          double v;
          if (rdir || cdir) v = (kk == k && cb == c) ? 1.0 : 0.0;
          else v = pair_value(g, coeff, x, c, y, cb, blo, bhi, false);
          col[pos] = (int)(kk * nc + cb);
          val[pos] = v;
          ++pos;
        }
      }
  // load: int f_c phi over the (up to 2^d) elements around the node
  double f = 0.0;
  if (!rdir) {
    int ecount = 1;
    for (int ax = 0; ax < g.dim; ++ax) ecount *= (x[ax] > 0) + (x[ax] < g.ne[ax]);
    f = g.load[c] * g.vol / (double)(1 << g.dim) * ecount;
  }
  rhs[r] = f;
}

// --------------------------------------------------------- subdomains ---
// Node box of subdomain j along each axis (element box [elo, ehi]).
__device__ __forceinline__ void sub_box(const Q1Geom& g, int j, int* elo, int* ehi, int* p) {
  p[0] = j % g.parts[0];
  p[1] = (j / g.parts[0]) % g.parts[1];
  p[2] = j / (g.parts[0] * g.parts[1]);
  for (int ax = 0; ax < 3; ++ax) {
    if (ax < g.dim) { elo[ax] = g.elo[ax][p[ax]]; ehi[ax] = g.ehi[ax][p[ax]]; }
    else { elo[ax] = 0; ehi[ax] = 0; }
  }
}

// Prefix sums over the subdomains: sub_ptr and the nnz offsets of the
// batched local matrices.  One block of 1024 threads, one subdomain per
// thread in rounds of 1024 with a running carry (scan in LDS).
__global__ __launch_bounds__(1024) void k_q1_subptr(const Q1Geom* __restrict__ gp,
                                                    int* __restrict__ sub_ptr,
                                                    int64_t* __restrict__ locnnz_off) {
  __shared__ int64_t sn[1024], sz[1024];
  const Q1Geom& g = *gp;
  const int t = threadIdx.x;
  int64_t carry_n = 0, carry_z = 0;
  for (int base = 0; base < g.nsub; base += 1024) {
    const int j = base + t;
    int64_t nodes = 0, nzn = 0;
    if (j < g.nsub) {
      int elo[3], ehi[3], p[3];
      sub_box(g, j, elo, ehi, p);
      nodes = 1;
      nzn = 1;
      for (int ax = 0; ax < 3; ++ax) {
        int nb = ehi[ax] - elo[ax] + 1;
        nodes *= nb;
        nzn *= (nb == 1 ? 1 : 3 * (int64_t)nb - 2);
      }
      nodes *= g.ncomp;
      nzn *= g.ncomp * g.ncomp;
    }
    sn[t] = nodes;
    sz[t] = nzn;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int64_t an = t >= off ? sn[t - off] : 0, az = t >= off ? sz[t - off] : 0;
      __syncthreads();
      sn[t] += an;
      sz[t] += az;
      __syncthreads();
    }
    if (j < g.nsub) {
      sub_ptr[j] = (int)(carry_n + sn[t] - nodes);
      locnnz_off[j] = carry_z + sz[t] - nzn;
    }
    carry_n += sn[1023];
    carry_z += sz[1023];
    __syncthreads();
  }
  if (t == 0) {
    sub_ptr[g.nsub] = (int)carry_n;
    locnnz_off[g.nsub] = carry_z;
  }
}

// Number of parts along `ax` whose node range [elo + (elo>0), ehi - (ehi<ne)]
// contains node i (the parts having the node off their artificial boundary).
__device__ __forceinline__ int interior_count(const Q1Geom& g, int ax, int i) {
  int cnt = 0;
  for (int p = 0; p < g.parts[ax]; ++p) {
    int lo = g.elo[ax][p] + (g.elo[ax][p] > 0);
    int hi = g.ehi[ax][p] - (g.ehi[ax][p] < g.ne[ax]);
    cnt += (lo <= i && i <= hi);
  }
  return cnt;
}

// Distance of node coordinate x from the artificial faces of part p along
// axis ax (those strictly inside the grid), in physical units; +inf if the
// part has none on this axis.
__device__ __forceinline__ double axis_art_dist(const Q1Geom& g, int ax, int p, int x) {
  double d = INFINITY;
  if (g.elo[ax][p] > 0) d = fmin(d, (x - g.elo[ax][p]) * g.h[ax]);
  if (g.ehi[ax][p] < g.ne[ax]) d = fmin(d, (g.ehi[ax][p] - x) * g.h[ax]);
  return d;
}

// Sarkis weight of box (p[0], p[1], p[2]) at node x: its distance from the
// box's artificial boundary (the smallest over the axes; 1 for a box
// without artificial faces) over the sum of the same distance for every box
// containing x.
__device__ double sarkis_weight(const Q1Geom& g, const int* p, const int* x) {
  int plo[3] = {0, 0, 0}, phi[3] = {0, 0, 0};
  for (int ax = 0; ax < g.dim; ++ax) {
    plo[ax] = g.parts[ax];
    phi[ax] = -1;
    for (int q = 0; q < g.parts[ax]; ++q)
      if (g.elo[ax][q] <= x[ax] && x[ax] <= g.ehi[ax][q]) {
        plo[ax] = min(plo[ax], q);
        phi[ax] = max(phi[ax], q);
      }
  }
  auto dist = [&](int q0, int q1, int q2) {
    const int q[3] = {q0, q1, q2};
    double d = INFINITY;
    for (int ax = 0; ax < g.dim; ++ax) d = fmin(d, axis_art_dist(g, ax, q[ax], x[ax]));
    return isinf(d) ? 1.0 : d;
  };
  double tot = 0.0;
  for (int q2 = plo[2]; q2 <= phi[2]; ++q2)
    for (int q1 = plo[1]; q1 <= phi[1]; ++q1)
      for (int q0 = plo[0]; q0 <= phi[0]; ++q0) tot += dist(q0, q1, q2);
  return dist(p[0], p[1], p[2]) / tot;
}

__global__ void k_q1_sublists(const Q1Geom* __restrict__ gp, const int* __restrict__ sub_ptr,
                              int* __restrict__ sub_idx, uint8_t* __restrict__ flags,
                              double* __restrict__ pou) {
  const Q1Geom& g = *gp;
  const int j = blockIdx.x;
  int elo[3], ehi[3], p[3];
  sub_box(g, j, elo, ehi, p);
  int nb[3];
  for (int ax = 0; ax < 3; ++ax) nb[ax] = ehi[ax] - elo[ax] + 1;
  const int n = sub_ptr[j + 1] - sub_ptr[j];
  const int nc = g.ncomp;
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    int ln = a / nc, c = a % nc;
    int l[3] = {ln % nb[0], (ln / nb[0]) % nb[1], ln / (nb[0] * nb[1])};
    int x[3];
    for (int ax = 0; ax < 3; ++ax) x[ax] = elo[ax] + l[ax];
    int64_t k = x[0] + (int64_t)g.nn[0] * (x[1] + (int64_t)g.nn[1] * x[2]);
    bool art = false;
    for (int ax = 0; ax < g.dim; ++ax) {
      if (elo[ax] > 0 && x[ax] == elo[ax]) art = true;
      if (ehi[ax] < g.ne[ax] && x[ax] == ehi[ax]) art = true;
    }
    bool dir = node_dirichlet(g, x);
    int64_t o = sub_ptr[j] + a;
    sub_idx[o] = (int)(k * nc + c);
    flags[o] = (uint8_t)((!art && !dir ? 1 : 0) | (dir ? 2 : 0));
    double mu = 0.0;
    if (!art && !dir) {
      if (g.pou == GENEO_POU_SARKIS) {
        mu = sarkis_weight(g, p, x);
      } else {
        int cnt = 1;
        for (int ax = 0; ax < g.dim; ++ax) cnt *= interior_count(g, ax, x[ax]);
        mu = 1.0 / (double)cnt;
      }
    }
    pou[o] = mu;
  }
}

// Batched local Neumann (all box elements) and overlap-zone matrices with
// local column indices; grid (subdomain, chunk of 256 local rows), one
// thread per local row.
__global__ void k_q1_local(const Q1Geom* __restrict__ gp, const double* __restrict__ coeff,
                           const int* __restrict__ sub_ptr, const int64_t* __restrict__ nzoff,
                           int* __restrict__ loc_rowptr, int* __restrict__ loc_col,
                           double* __restrict__ an, double* __restrict__ ao) {
  const Q1Geom& g = *gp;
  const int j = blockIdx.x;
  int elo[3], ehi[3], p[3];
  sub_box(g, j, elo, ehi, p);
  int nb[3];
  for (int ax = 0; ax < 3; ++ax) nb[ax] = ehi[ax] - elo[ax] + 1;
  const int n = sub_ptr[j + 1] - sub_ptr[j];
  const int nc = g.ncomp;
  int bhi[3] = {ehi[0], ehi[1], ehi[2]};
  for (int ax = g.dim; ax < 3; ++ax) bhi[ax] = 1;
  for (int r = blockIdx.y * blockDim.x + threadIdx.x; r < n; r += blockDim.x * gridDim.y) {
    int ln = r / nc, c = r % nc;
    int l[3] = {ln % nb[0], (ln / nb[0]) % nb[1], ln / (nb[0] * nb[1])};
    int cnt[3];
    for (int ax = 0; ax < 3; ++ax) cnt[ax] = nbcount(l[ax], nb[ax]);
    int64_t pre = nbprefix(l[2], nb[2]) * nbtotal(nb[1]) * nbtotal(nb[0]) +
                  (int64_t)cnt[2] * nbprefix(l[1], nb[1]) * nbtotal(nb[0]) +
                  (int64_t)cnt[2] * cnt[1] * nbprefix(l[0], nb[0]);
    int rowlen = nc * cnt[0] * cnt[1] * cnt[2];
    int64_t start = nzoff[j] + (int64_t)nc * nc * pre + (int64_t)c * rowlen;
    int64_t grow = sub_ptr[j] + r;
    loc_rowptr[grow] = (int)start;
    if (j == g.nsub - 1 && r == n - 1) loc_rowptr[grow + 1] = (int)(start + rowlen);
    int x[3];
    for (int ax = 0; ax < 3; ++ax) x[ax] = elo[ax] + l[ax];
    bool rdir = node_dirichlet(g, x);
    int64_t pos = start;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int m[3] = {l[0] + dx, l[1] + dy, l[2] + dz};
          bool ok = true;
          for (int ax = 0; ax < 3; ++ax) ok = ok && m[ax] >= 0 && m[ax] < nb[ax];
          if (!ok) continue;
          int y[3];
          for (int ax = 0; ax < 3; ++ax) y[ax] = elo[ax] + m[ax];
          bool cdir = node_dirichlet(g, y);
          int lm = m[0] + nb[0] * (m[1] + nb[1] * m[2]);
          for (int cb = 0; cb < nc; ++cb) {
            double vn, vo;
            if (rdir || cdir) {
              vn = vo = (lm == ln && cb == c) ? 1.0 : 0.0;
            } else {
              vn = pair_value(g, coeff, x, c, y, cb, elo, bhi, false);
              vo = pair_value(g, coeff, x, c, y, cb, elo, bhi, true);
            }
            loc_col[pos] = lm * nc + cb;
            an[pos] = vn;
            ao[pos] = vo;
            ++pos;
          }
        }
  }
}

// ------------------------------------------------------------- host side ---
static void axis_ranges(int n, int parts, int ovl, int* elo, int* ehi) {
  int base = n / parts, extra = n % parts, lo = 0;
  for (int p = 0; p < parts; ++p) {
    int sz = base + (p < extra ? 1 : 0);
    elo[p] = lo - ovl < 0 ? 0 : lo - ovl;
    ehi[p] = lo + sz + ovl > n ? n : lo + sz + ovl;
    lo += sz;
  }
}

void q1_thm1_tau(const Q1Geom& g, double* tau) {
  double hmin = g.h[0];
  for (int ax = 1; ax < g.dim; ++ax) hmin = fmin(hmin, g.h[ax]);
  const double delta = 2.0 * g.ovl * hmin;
  for (int j = 0; j < g.nsub; ++j) {
    const int p[3] = {j % g.parts[0], (j / g.parts[0]) % g.parts[1],
                      j / (g.parts[0] * g.parts[1])};
    double d2 = 0.0;
    for (int ax = 0; ax < g.dim; ++ax) {
      const double w = (g.ehi[ax][p[ax]] - g.elo[ax][p[ax]]) * g.h[ax];
      d2 += w * w;
    }
    tau[j] = delta / sqrt(d2);
  }
}

int q1_make_geom(const geneo_grid_t* grid, Q1Geom* g, std::string* err) {
  if (!grid) { *err = "grid is NULL"; return GENEO_ERR_ARG; }
  memset(g, 0, sizeof(*g));
  g->dim = grid->dim;
  g->ncomp = grid->ncomp;
  if (g->dim != 2 && g->dim != 3) { *err = "dim must be 2 or 3"; return GENEO_ERR_ARG; }
  if (!(g->ncomp == 1 || (g->ncomp == 3 && g->dim == 3))) {
    *err = "ncomp must be 1, or 3 in 3D"; return GENEO_ERR_ARG;
  }
  if (grid->ovl < 1) { *err = "overlap must be at least one element layer"; return GENEO_ERR_ARG; }
  g->ovl = grid->ovl;
  g->dirichlet = grid->dirichlet;
  if (grid->pou != GENEO_POU_CONSTANT && grid->pou != GENEO_POU_SARKIS) {
    *err = "unknown partition of unity";
    return GENEO_ERR_ARG;
  }
  g->pou = grid->pou;
  if (grid->element != GENEO_ELEM_Q1 && grid->element != GENEO_ELEM_S20) {
    *err = "unknown element";
    return GENEO_ERR_ARG;
  }
  g->element = grid->element;
  if (g->element == GENEO_ELEM_S20 && (g->dim != 3 || g->ncomp != 3 || g->pou != GENEO_POU_CONSTANT)) {
    *err = "serendipity bricks: 3D elasticity with the piecewise-constant partition of unity";
    return GENEO_ERR_ARG;
  }
  g->nsub = 1;
  double vol = 1.0;
  for (int ax = 0; ax < 3; ++ax) {
    if (ax < g->dim) {
      g->ne[ax] = grid->ne[ax];
      g->nn[ax] = grid->ne[ax] + 1;
      g->parts[ax] = grid->parts[ax];
      g->h[ax] = grid->h[ax];
      if (g->ne[ax] < 1 || g->parts[ax] < 1 || g->parts[ax] > g->ne[ax] ||
          g->parts[ax] > Q1_MAXP || !(g->h[ax] > 0)) {
        *err = "invalid ne/parts/h on an axis"; return GENEO_ERR_ARG;
      }
      vol *= g->h[ax];
      axis_ranges(g->ne[ax], g->parts[ax], g->ovl, g->elo[ax], g->ehi[ax]);
    } else {
      g->ne[ax] = 1; g->nn[ax] = 1; g->parts[ax] = 1; g->h[ax] = 1.0;
    }
    g->nsub *= g->parts[ax];
  }
  for (int c = 0; c < g->ncomp; ++c) g->load[c] = grid->load[c];
  g->vol = vol;
  // 2^d-point Gauss rule on the reference box, physical gradients
  const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  const int nv = 1 << g->dim;
  for (int q = 0; q < 8; ++q) {
    if (q >= nv) { g->wq[q] = 0.0; continue; }
    double xi[3];
    for (int ax = 0; ax < g->dim; ++ax) xi[ax] = gp[(q >> ax) & 1];
    g->wq[q] = vol / (double)nv;
    for (int a = 0; a < nv; ++a)
      for (int dax = 0; dax < g->dim; ++dax) {
        double v = 1.0;
        for (int ax = 0; ax < g->dim; ++ax) {
          int bit = (a >> ax) & 1;
          if (ax == dax) v *= (bit ? 1.0 : -1.0) / g->h[ax];
          else v *= bit ? xi[ax] : 1.0 - xi[ax];
        }
        g->grad[q][a][dax] = v;
      }
  }
  // Darcy element matrix in closed form (the 2-point rule above is exact
  // for it): with the 1D stiffness k = +-1 and the 1D mass (1/3, 1/6) =
  // mi / 6 (mi = 2, 1), K_ab = 6^{1-d} sum_x (prod_{y != x} h_y / h_x)
  // k(a_x, b_x) prod_{y != x} mi(a_y, b_y); the integer factor is a power
  // of two, so only the edge-length ratio and the final division round.
  for (int a = 0; a < nv; ++a)
    for (int b = 0; b < nv; ++b) {
      double s = 0.0;
      for (int ax = 0; ax < g->dim; ++ax) {
        double c = 1.0;
        for (int o = 0; o < g->dim; ++o)
          if (o != ax) c = c * g->h[o];
        c = c / g->h[ax];
        int f = (((a >> ax) & 1) == ((b >> ax) & 1)) ? 1 : -1;
        for (int o = 0; o < g->dim; ++o)
          if (o != ax) f *= (((a >> o) & 1) == ((b >> o) & 1)) ? 2 : 1;
        const double t = c * (double)f;
        s = s + t;
      }
      g->kref[a][b] = s / (g->dim == 2 ? 6.0 : 36.0);
    }
  if (g->element == GENEO_ELEM_S20) s20_tables(g);
  return GENEO_OK;
}

void q1_sizes(const Q1Geom& g, geneo_q1_sizes_t* s) {
  if (g.element == GENEO_ELEM_S20) {
    s20_sizes(g, s);
    return;
  }
  int64_t nodes = 1, nzn = 1;
  for (int ax = 0; ax < 3; ++ax) {
    nodes *= g.nn[ax];
    nzn *= (g.nn[ax] == 1 ? 1 : 3 * (int64_t)g.nn[ax] - 2);
  }
  s->ndof = nodes * g.ncomp;
  s->nnz = nzn * g.ncomp * g.ncomp;
  s->nsub = g.nsub;
  int64_t nloc = 0, nzl = 0, nmax = 0;
  for (int j = 0; j < g.nsub; ++j) {
    int p[3] = {j % g.parts[0], (j / g.parts[0]) % g.parts[1], j / (g.parts[0] * g.parts[1])};
    int64_t bn = 1, bz = 1;
    for (int ax = 0; ax < 3; ++ax) {
      int nb = ax < g.dim ? g.ehi[ax][p[ax]] - g.elo[ax][p[ax]] + 1 : 1;
      bn *= nb;
      bz *= (nb == 1 ? 1 : 3 * (int64_t)nb - 2);
    }
    nloc += bn * g.ncomp;
    nzl += bz * g.ncomp * g.ncomp;
    if (bn * g.ncomp > nmax) nmax = bn * g.ncomp;
  }
  s->nloc = nloc;
  s->nnz_loc = nzl;
  s->nmax = nmax;
}

hipError_t q1_launch_all(const Q1Geom* dgeom, const Q1Geom& g, const geneo_q1_sizes_t& s,
                         const double* coeff, int* A_rowptr, int* A_col, double* A_val,
                         double* b, int* sub_ptr, int* sub_idx, uint8_t* flags, double* pou,
                         int* loc_rowptr, int* loc_col, double* an, double* ao,
                         int64_t* nzoff, hipStream_t st) {
  if (g.element == GENEO_ELEM_S20)
    return s20_launch_all(dgeom, g, s, coeff, A_rowptr, A_col, A_val, b, sub_ptr, sub_idx, flags,
                          pou, loc_rowptr, loc_col, an, ao, st);
  int64_t nrows = s.ndof;
  int bs = 256;
  hipLaunchKernelGGL(k_q1_global, dim3((unsigned)((nrows + bs - 1) / bs)), dim3(bs), 0, st,
                     dgeom, coeff, A_rowptr, A_col, A_val, b, nrows);
  hipLaunchKernelGGL(k_q1_subptr, dim3(1), dim3(1024), 0, st, dgeom, sub_ptr, nzoff);
  hipLaunchKernelGGL(k_q1_sublists, dim3(g.nsub), dim3(256), 0, st, dgeom, sub_ptr, sub_idx,
                     flags, pou);
  const unsigned rchunks = (unsigned)std::max<int64_t>(1, (s.nmax + 255) / 256);
  hipLaunchKernelGGL(k_q1_local, dim3(g.nsub, rchunks), dim3(256), 0, st, dgeom, coeff, sub_ptr,
                     nzoff, loc_rowptr, loc_col, an, ao);
  return hipGetLastError();
}

}  // namespace geneo
