// Structured assembly with 20-node serendipity bricks (the quadratic
// element of the paper's composite experiments, Sec. 5.3) for the
// elasticity form (eq. (3), no traction): global matrix with symmetric
// Dirichlet elimination, load vector, the overlapping box subdomains
// (Sec. 3) with their sets and the piecewise-constant partition of unity
// (Def. 3, Sec. 4.3), and the batched local Neumann and overlap-zone
// matrices (Sec. 4.3).
//
// Nodes sit on the lattice of half-edge steps (coordinates 0 .. 2 ne per
// axis) at the points with at most one odd coordinate: the brick vertices
// (all even) and the edge midpoints; they are numbered lexicographically
// (x fastest) over those points.  Element integrals use the tensor 3-point
// Gauss rule (exact for these integrands).  As in the Q1 assembly, every
// output entry is produced by one thread that adds its element
// contributions in ascending element order (no atomics); the row and
// column structure (which is fixed by the mesh) is counted on the host.
#include "q1.h"

#include <vector>

namespace geneo {

// ------------------------------------------------------------ lattice ---
__host__ __device__ __forceinline__ bool s20_valid(int x, int y, int z) {
  return (x & 1) + (y & 1) + (z & 1) <= 1;
}

// Number of the valid point (x, y, z) of the lattice of an n[0] x n[1] x
// n[2] brick mesh (lexicographic over the valid points).
__host__ __device__ __forceinline__ int64_t s20_id(const int* n, int x, int y, int z) {
  const int64_t nx = n[0], ny = n[1];
  const int64_t even_layer = (ny + 1) * (2 * nx + 1) + ny * (nx + 1);
  const int64_t odd_layer = (nx + 1) * (ny + 1);
  const int64_t base = (int64_t)((z + 1) / 2) * even_layer + (int64_t)(z / 2) * odd_layer;
  if ((z & 1) == 0)
    return base + (int64_t)((y + 1) / 2) * (2 * nx + 1) + (int64_t)(y / 2) * (nx + 1) +
           ((y & 1) == 0 ? x : x / 2);
  return base + (int64_t)(y / 2) * (nx + 1) + x / 2;
}

// Lattice range of the points coupled to coordinate v along one axis (the
// points of the elements containing v), clipped to [lo, hi].
__host__ __device__ __forceinline__ void s20_range(int v, int lo, int hi, int* a, int* b) {
  if (v & 1) {
    *a = v - 1;
    *b = v + 1;
  } else {
    *a = v - 2;
    *b = v + 2;
  }
  if (*a < lo) *a = lo;
  if (*b > hi) *b = hi;
}

// Valid points in the lattice box [a0, b0] x [a1, b1] x [a2, b2].
__host__ __device__ __forceinline__ int64_t s20_box_count(const int* a, const int* b) {
  int64_t E[3], O[3];
  for (int ax = 0; ax < 3; ++ax) {
    const int ev = b[ax] / 2 - (a[ax] + 1) / 2 + 1;  // even values in [a, b]
    E[ax] = ev < 0 ? 0 : ev;
    O[ax] = (b[ax] - a[ax] + 1) - E[ax];
  }
  return E[0] * E[1] * E[2] + O[0] * E[1] * E[2] + E[0] * O[1] * E[2] + E[0] * E[1] * O[2];
}

// Local node of element e (lattice origin 2 e) at lattice offset o.
__device__ __forceinline__ int s20_local(const int* o) {
  int ax = -1;
  for (int i = 0; i < 3; ++i)
    if (o[i] & 1) ax = i;
  if (ax < 0) return (o[0] >> 1) + 2 * (o[1] >> 1) + 4 * (o[2] >> 1);
  const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
  return 8 + 4 * ax + (o[o1] >> 1) + 2 * (o[o2] >> 1);
}

__device__ __forceinline__ bool s20_dirichlet(const Q1Geom& g, const int* x) {
  for (int ax = 0; ax < 3; ++ax) {
    if (((g.dirichlet >> (2 * ax)) & 1) && x[ax] == 0) return true;
    if (((g.dirichlet >> (2 * ax + 1)) & 1) && x[ax] == 2 * g.ne[ax]) return true;
  }
  return false;
}

// Element matrix entry (node a, component c) x (node b, component cb) of
// element e: sum over the 27 points of w (grad_a)^T C (grad_b) restricted to
// the strain rows the two components feed (engineering shear).
__device__ double s20_entry(const Q1Geom& g, const double* coeff, int64_t e, int a, int c, int b,
                            int cb) {
  const int srow[3][3] = {{0, 4, 5}, {1, 3, 5}, {2, 3, 4}};
  const int gax[3][3] = {{0, 2, 1}, {1, 2, 0}, {2, 1, 0}};
  const double* C21 = coeff + 21 * e;
  double Cm[3][3];
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const int s = srow[c][u], t = srow[cb][v];
      const int lo = s < t ? s : t, hi = s < t ? t : s;
      Cm[u][v] = C21[lo * (11 - lo) / 2 + hi];
    }
  double sum = 0.0;
  for (int q = 0; q < 27; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const double gu = g.s20grad[q][a][gax[c][u]];
#pragma unroll
      for (int v = 0; v < 3; ++v) acc += gu * Cm[u][v] * g.s20grad[q][b][gax[cb][v]];
    }
    sum += g.s20wq[q] * acc;
  }
  return sum;
}

// Element multiplicity test (the overlap zone: elements in at least two
// subdomain boxes).
__device__ __forceinline__ bool s20_overlap_elem(const Q1Geom& g, const int* ee) {
  int m = 1;
  for (int ax = 0; ax < 3; ++ax) {
    int cnt = 0;
    for (int p = 0; p < g.parts[ax]; ++p) cnt += (g.elo[ax][p] <= ee[ax] && ee[ax] < g.ehi[ax][p]);
    m *= cnt;
  }
  return m >= 2;
}

// (row node x, comp c) x (col node y, comp cb) summed over the elements of
// the element box [blo, bhi) containing both (and, with ovl_only, lying in
// the overlap zone), in ascending element order from 0.
__device__ double s20_pair(const Q1Geom& g, const double* coeff, const int* x, int c, const int* y,
                           int cb, const int* blo, const int* bhi, bool ovl_only) {
  int lo[3], hi[3];
  for (int ax = 0; ax < 3; ++ax) {
    // elements containing lattice coordinate v: v/2 - 1 and v/2 (even v), (v-1)/2 (odd v)
    const int xl = (x[ax] & 1) ? (x[ax] - 1) / 2 : x[ax] / 2 - 1, xh = x[ax] / 2;
    const int yl = (y[ax] & 1) ? (y[ax] - 1) / 2 : y[ax] / 2 - 1, yh = y[ax] / 2;
    lo[ax] = max(max(xl, yl), blo[ax]);
    hi[ax] = min(min(xh, yh), bhi[ax] - 1);
    if (lo[ax] > hi[ax]) return 0.0;
  }
  double s = 0.0;
  for (int ez = lo[2]; ez <= hi[2]; ++ez)
    for (int ey = lo[1]; ey <= hi[1]; ++ey)
      for (int ex = lo[0]; ex <= hi[0]; ++ex) {
        const int ee[3] = {ex, ey, ez};
        if (ovl_only && !s20_overlap_elem(g, ee)) continue;
        int ox[3], oy[3];
        for (int ax = 0; ax < 3; ++ax) {
          ox[ax] = x[ax] - 2 * ee[ax];
          oy[ax] = y[ax] - 2 * ee[ax];
        }
        const int64_t e = ex + (int64_t)g.ne[0] * (ey + (int64_t)g.ne[1] * ez);
        s = __dadd_rn(s, s20_entry(g, coeff, e, s20_local(ox), c, s20_local(oy), cb));
      }
  return s;
}

// ------------------------------------------------------- global matrix ---
// One thread per (lattice point, component); invalid points return.
__global__ void k_s20_global(const Q1Geom* __restrict__ gp, const double* __restrict__ coeff,
                             const int* __restrict__ rowptr, int* __restrict__ col,
                             double* __restrict__ val, double* __restrict__ rhs, int64_t npts) {
  const Q1Geom& g = *gp;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= npts * 3) return;
  const int c = (int)(t % 3);
  const int64_t pt = t / 3;
  const int L0 = 2 * g.ne[0] + 1, L1 = 2 * g.ne[1] + 1;
  const int x[3] = {(int)(pt % L0), (int)((pt / L0) % L1), (int)(pt / ((int64_t)L0 * L1))};
  if (!s20_valid(x[0], x[1], x[2])) return;
  const int64_t k = s20_id(g.ne, x[0], x[1], x[2]);
  const int64_t r = 3 * k + c;
  const bool rdir = s20_dirichlet(g, x);
  const int blo[3] = {0, 0, 0}, bhi[3] = {g.ne[0], g.ne[1], g.ne[2]};
  int a[3], b[3];
  for (int ax = 0; ax < 3; ++ax) s20_range(x[ax], 0, 2 * g.ne[ax], &a[ax], &b[ax]);
  int64_t pos = rowptr[r];
  for (int z = a[2]; z <= b[2]; ++z)
    for (int yy = a[1]; yy <= b[1]; ++yy)
      for (int xx = a[0]; xx <= b[0]; ++xx) {
        if (!s20_valid(xx, yy, z)) continue;
        const int y[3] = {xx, yy, z};
        const int64_t kk = s20_id(g.ne, xx, yy, z);
        const bool cdir = s20_dirichlet(g, y);
        for (int cb = 0; cb < 3; ++cb) {
          double v;
          if (rdir || cdir) v = (kk == k && cb == c) ? 1.0 : 0.0;
          else v = s20_pair(g, coeff, x, c, y, cb, blo, bhi, false);
          col[pos] = (int)(kk * 3 + cb);
          val[pos] = v;
          ++pos;
        }
      }
  // load: the integral of the shape function over each element around the node
  double f = 0.0;
  if (!rdir) {
    int lo[3], hi[3];
    for (int ax = 0; ax < 3; ++ax) {
      lo[ax] = max((x[ax] & 1) ? (x[ax] - 1) / 2 : x[ax] / 2 - 1, 0);
      hi[ax] = min(x[ax] / 2, g.ne[ax] - 1);
    }
    for (int ez = lo[2]; ez <= hi[2]; ++ez)
      for (int ey = lo[1]; ey <= hi[1]; ++ey)
        for (int ex = lo[0]; ex <= hi[0]; ++ex) {
          const int o[3] = {x[0] - 2 * ex, x[1] - 2 * ey, x[2] - 2 * ez};
          f = __dadd_rn(f, __dmul_rn(g.load[c], g.s20load[s20_local(o)]));
        }
  }
  rhs[r] = f;
}

// --------------------------------------------------------- subdomains ---
__device__ __forceinline__ void s20_sub_box(const Q1Geom& g, int j, int* elo, int* ehi) {
  const int p[3] = {j % g.parts[0], (j / g.parts[0]) % g.parts[1], j / (g.parts[0] * g.parts[1])};
  for (int ax = 0; ax < 3; ++ax) {
    elo[ax] = g.elo[ax][p[ax]];
    ehi[ax] = g.ehi[ax][p[ax]];
  }
}

// Parts along ax having lattice coordinate v off their artificial boundary.
__device__ __forceinline__ int s20_interior_count(const Q1Geom& g, int ax, int v) {
  int cnt = 0;
  for (int p = 0; p < g.parts[ax]; ++p) {
    const int lo = 2 * g.elo[ax][p] + (g.elo[ax][p] > 0);
    const int hi = 2 * g.ehi[ax][p] - (g.ehi[ax][p] < g.ne[ax]);
    cnt += (lo <= v && v <= hi);
  }
  return cnt;
}

// One block per subdomain; threads over (box lattice point, component).
__global__ void k_s20_sublists(const Q1Geom* __restrict__ gp, const int* __restrict__ sub_ptr,
                               int* __restrict__ sub_idx, uint8_t* __restrict__ flags,
                               double* __restrict__ pou) {
  const Q1Geom& g = *gp;
  const int j = blockIdx.x;
  int elo[3], ehi[3];
  s20_sub_box(g, j, elo, ehi);
  const int nb[3] = {ehi[0] - elo[0], ehi[1] - elo[1], ehi[2] - elo[2]};
  const int L0 = 2 * nb[0] + 1, L1 = 2 * nb[1] + 1, L2 = 2 * nb[2] + 1;
  const int64_t npts = (int64_t)L0 * L1 * L2;
  for (int64_t t = threadIdx.x; t < npts * 3; t += blockDim.x) {
    const int c = (int)(t % 3);
    const int64_t pt = t / 3;
    const int l[3] = {(int)(pt % L0), (int)((pt / L0) % L1), (int)(pt / ((int64_t)L0 * L1))};
    if (!s20_valid(l[0], l[1], l[2])) continue;
    int x[3];
    for (int ax = 0; ax < 3; ++ax) x[ax] = 2 * elo[ax] + l[ax];
    bool art = false;
    for (int ax = 0; ax < 3; ++ax) {
      if (elo[ax] > 0 && x[ax] == 2 * elo[ax]) art = true;
      if (ehi[ax] < g.ne[ax] && x[ax] == 2 * ehi[ax]) art = true;
    }
    const bool dir = s20_dirichlet(g, x);
    const int64_t o = sub_ptr[j] + 3 * s20_id(nb, l[0], l[1], l[2]) + c;
    sub_idx[o] = (int)(3 * s20_id(g.ne, x[0], x[1], x[2]) + c);
    flags[o] = (uint8_t)((!art && !dir ? 1 : 0) | (dir ? 2 : 0));
    double mu = 0.0;
    if (!art && !dir) {
      int cnt = 1;
      for (int ax = 0; ax < 3; ++ax) cnt *= s20_interior_count(g, ax, x[ax]);
      mu = 1.0 / (double)cnt;
    }
    pou[o] = mu;
  }
}

// Batched local Neumann (all box elements) and overlap-zone matrices with
// local column indices; grid (subdomain, chunk of 256 threads), one thread
// per (box lattice point, component).
__global__ void k_s20_local(const Q1Geom* __restrict__ gp, const double* __restrict__ coeff,
                            const int* __restrict__ sub_ptr, const int* __restrict__ loc_rowptr,
                            int* __restrict__ loc_col, double* __restrict__ an,
                            double* __restrict__ ao) {
  const Q1Geom& g = *gp;
  const int j = blockIdx.x;
  int elo[3], ehi[3];
  s20_sub_box(g, j, elo, ehi);
  const int nb[3] = {ehi[0] - elo[0], ehi[1] - elo[1], ehi[2] - elo[2]};
  const int L0 = 2 * nb[0] + 1, L1 = 2 * nb[1] + 1, L2 = 2 * nb[2] + 1;
  const int64_t npts = (int64_t)L0 * L1 * L2;
  for (int64_t t = blockIdx.y * (int64_t)blockDim.x + threadIdx.x; t < npts * 3;
       t += (int64_t)blockDim.x * gridDim.y) {
    const int c = (int)(t % 3);
    const int64_t pt = t / 3;
    const int l[3] = {(int)(pt % L0), (int)((pt / L0) % L1), (int)(pt / ((int64_t)L0 * L1))};
    if (!s20_valid(l[0], l[1], l[2])) continue;
    int x[3];
    for (int ax = 0; ax < 3; ++ax) x[ax] = 2 * elo[ax] + l[ax];
    const int64_t ln = s20_id(nb, l[0], l[1], l[2]);
    const bool rdir = s20_dirichlet(g, x);
    int a[3], b[3];
    for (int ax = 0; ax < 3; ++ax) s20_range(l[ax], 0, 2 * nb[ax], &a[ax], &b[ax]);
    int64_t pos = loc_rowptr[sub_ptr[j] + 3 * ln + c];
    for (int z = a[2]; z <= b[2]; ++z)
      for (int yy = a[1]; yy <= b[1]; ++yy)
        for (int xx = a[0]; xx <= b[0]; ++xx) {
          if (!s20_valid(xx, yy, z)) continue;
          const int m[3] = {xx, yy, z};
          int y[3];
          for (int ax = 0; ax < 3; ++ax) y[ax] = 2 * elo[ax] + m[ax];
          const bool cdir = s20_dirichlet(g, y);
          const int64_t lm = s20_id(nb, xx, yy, z);
          for (int cb = 0; cb < 3; ++cb) {
            double vn, vo;
            if (rdir || cdir) {
              vn = vo = (lm == ln && cb == c) ? 1.0 : 0.0;
            } else {
              vn = s20_pair(g, coeff, x, c, y, cb, elo, ehi, false);
              vo = s20_pair(g, coeff, x, c, y, cb, elo, ehi, true);
            }
            loc_col[pos] = (int)(lm * 3 + cb);
            an[pos] = vn;
            ao[pos] = vo;
            ++pos;
          }
        }
  }
}

// ------------------------------------------------------------- host side ---
// Structure of the matrices (row lengths, offsets): host counts, the same
// lattice formulas as the kernels.
namespace {
struct S20Counts {
  std::vector<int> rowptr;      // global CSR row offsets [ndof + 1]
  std::vector<int> sub_ptr;     // [nsub + 1]
  std::vector<int> loc_rowptr;  // [nloc + 1]
  int64_t nnz = 0, nloc = 0, nnz_loc = 0, nmax = 0;
};

void s20_count(const Q1Geom& g, S20Counts* out, bool offsets) {
  const int L[3] = {2 * g.ne[0] + 1, 2 * g.ne[1] + 1, 2 * g.ne[2] + 1};
  int64_t nodes = 0, nnz = 0;
  if (offsets) out->rowptr.assign(1, 0);
  for (int z = 0; z < L[2]; ++z)
    for (int y = 0; y < L[1]; ++y)
      for (int x = 0; x < L[0]; ++x) {
        if (!s20_valid(x, y, z)) continue;
        ++nodes;
        const int v[3] = {x, y, z};
        int a[3], b[3];
        for (int ax = 0; ax < 3; ++ax) s20_range(v[ax], 0, L[ax] - 1, &a[ax], &b[ax]);
        const int64_t len = 3 * s20_box_count(a, b);
        for (int c = 0; c < 3; ++c) {
          nnz += len;
          if (offsets) out->rowptr.push_back((int)nnz);
        }
      }
  out->nnz = nnz;
  int64_t nloc = 0, nzl = 0, nmax = 0;
  if (offsets) {
    out->sub_ptr.assign(1, 0);
    out->loc_rowptr.assign(1, 0);
  }
  for (int j = 0; j < g.nsub; ++j) {
    const int p[3] = {j % g.parts[0], (j / g.parts[0]) % g.parts[1], j / (g.parts[0] * g.parts[1])};
    int nb[3], Lb[3];
    for (int ax = 0; ax < 3; ++ax) {
      nb[ax] = g.ehi[ax][p[ax]] - g.elo[ax][p[ax]];
      Lb[ax] = 2 * nb[ax] + 1;
    }
    int64_t bn = 0;
    for (int z = 0; z < Lb[2]; ++z)
      for (int y = 0; y < Lb[1]; ++y)
        for (int x = 0; x < Lb[0]; ++x) {
          if (!s20_valid(x, y, z)) continue;
          ++bn;
          const int v[3] = {x, y, z};
          int a[3], b[3];
          for (int ax = 0; ax < 3; ++ax) s20_range(v[ax], 0, Lb[ax] - 1, &a[ax], &b[ax]);
          const int64_t len = 3 * s20_box_count(a, b);
          for (int c = 0; c < 3; ++c) {
            nzl += len;
            if (offsets) out->loc_rowptr.push_back((int)nzl);
          }
        }
    nloc += 3 * bn;
    nmax = std::max<int64_t>(nmax, 3 * bn);
    if (offsets) out->sub_ptr.push_back((int)nloc);
  }
  out->nloc = nloc;
  out->nnz_loc = nzl;
  out->nmax = nmax;
}
}  // namespace

void s20_tables(Q1Geom* g) {
  // 3-point Gauss on [-1, 1] per axis, x fastest; reference gradients of the
  // 20 shape functions scaled to the brick (2 / h per axis)
  const double gp[3] = {-sqrt(0.6), 0.0, sqrt(0.6)};
  const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
  const double jac = g->h[0] * g->h[1] * g->h[2] / 8.0;
  int off[20][3];
  for (int a = 0; a < 8; ++a)
    for (int i = 0; i < 3; ++i) off[a][i] = 2 * ((a >> i) & 1);
  for (int ax = 0; ax < 3; ++ax) {
    const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
    for (int b = 0; b < 4; ++b) {
      int* o = off[8 + 4 * ax + b];
      o[ax] = 1;
      o[o1] = 2 * (b & 1);
      o[o2] = 2 * (b >> 1);
    }
  }
  for (int a = 0; a < 20; ++a) g->s20load[a] = 0.0;
  for (int q = 0; q < 27; ++q) {
    const int iq[3] = {q % 3, (q / 3) % 3, q / 9};
    const double xi[3] = {gp[iq[0]], gp[iq[1]], gp[iq[2]]};
    g->s20wq[q] = gw[iq[0]] * gw[iq[1]] * gw[iq[2]] * jac;
    for (int a = 0; a < 20; ++a) {
      double c[3], t[3];
      int zc = -1;
      for (int i = 0; i < 3; ++i) {
        c[i] = off[a][i] - 1.0;
        t[i] = 1.0 + c[i] * xi[i];
        if (c[i] == 0.0) zc = i;
      }
      double N, dN[3];
      if (zc < 0) {
        const double s = c[0] * xi[0] + c[1] * xi[1] + c[2] * xi[2] - 2.0;
        const double p = t[0] * t[1] * t[2];
        N = p * s / 8.0;
        for (int i = 0; i < 3; ++i) {
          double pi = 1.0;
          for (int k = 0; k < 3; ++k)
            if (k != i) pi *= t[k];
          dN[i] = (c[i] * pi * s + p * c[i]) / 8.0;
        }
      } else {
        const int o1 = zc == 0 ? 1 : 0, o2 = zc == 2 ? 1 : 2;
        const double qv = 1.0 - xi[zc] * xi[zc];
        N = qv * t[o1] * t[o2] / 4.0;
        dN[zc] = -2.0 * xi[zc] * t[o1] * t[o2] / 4.0;
        dN[o1] = qv * c[o1] * t[o2] / 4.0;
        dN[o2] = qv * c[o2] * t[o1] / 4.0;
      }
      for (int i = 0; i < 3; ++i) g->s20grad[q][a][i] = dN[i] * 2.0 / g->h[i];
      g->s20load[a] += g->s20wq[q] * N;
    }
  }
}

void s20_sizes(const Q1Geom& g, geneo_q1_sizes_t* s) {
  S20Counts c;
  s20_count(g, &c, false);
  int64_t nodes = 1, corners = 1;
  for (int ax = 0; ax < 3; ++ax) corners *= g.ne[ax] + 1;
  nodes = corners;
  for (int ax = 0; ax < 3; ++ax) nodes += g.ne[ax] * (corners / (g.ne[ax] + 1));
  s->ndof = 3 * nodes;
  s->nnz = c.nnz;
  s->nsub = g.nsub;
  s->nloc = c.nloc;
  s->nnz_loc = c.nnz_loc;
  s->nmax = c.nmax;
}

hipError_t s20_launch_all(const Q1Geom* dgeom, const Q1Geom& g, const geneo_q1_sizes_t& s,
                          const double* coeff, int* A_rowptr, int* A_col, double* A_val,
                          double* b, int* sub_ptr, int* sub_idx, uint8_t* flags, double* pou,
                          int* loc_rowptr, int* loc_col, double* an, double* ao,
                          hipStream_t st) {
  S20Counts c;
  s20_count(g, &c, true);
  if ((int64_t)c.rowptr.size() != s.ndof + 1 || (int64_t)c.loc_rowptr.size() != s.nloc + 1)
    return hipErrorInvalidValue;
  // (pageable copies: the caller synchronises the stream before returning)
  hipError_t e = hipMemcpyAsync(A_rowptr, c.rowptr.data(), c.rowptr.size() * sizeof(int),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sub_ptr, c.sub_ptr.data(), c.sub_ptr.size() * sizeof(int),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(loc_rowptr, c.loc_rowptr.data(), c.loc_rowptr.size() * sizeof(int),
                       hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  // the host vectors must outlive the copies
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  const int64_t npts = (int64_t)(2 * g.ne[0] + 1) * (2 * g.ne[1] + 1) * (2 * g.ne[2] + 1);
  hipLaunchKernelGGL(k_s20_global, dim3((unsigned)((3 * npts + 255) / 256)), dim3(256), 0, st,
                     dgeom, coeff, A_rowptr, A_col, A_val, b, npts);
  hipLaunchKernelGGL(k_s20_sublists, dim3(g.nsub), dim3(256), 0, st, dgeom, sub_ptr, sub_idx,
                     flags, pou);
  int64_t maxpts = 1;
  for (int j = 0; j < g.nsub; ++j) {
    const int p[3] = {j % g.parts[0], (j / g.parts[0]) % g.parts[1], j / (g.parts[0] * g.parts[1])};
    int64_t np = 1;
    for (int ax = 0; ax < 3; ++ax) np *= 2 * (g.ehi[ax][p[ax]] - g.elo[ax][p[ax]]) + 1;
    maxpts = std::max(maxpts, np);
  }
  const unsigned chunks = (unsigned)std::max<int64_t>(1, (3 * maxpts + 255) / 256);
  hipLaunchKernelGGL(k_s20_local, dim3(g.nsub, chunks), dim3(256), 0, st, dgeom, coeff, sub_ptr,
                     loc_rowptr, loc_col, an, ao);
  return hipGetLastError();
}

}  // namespace geneo
