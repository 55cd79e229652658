// Structured Q1 problem description shared by the assembly kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <string>

#include "geneo.h"

namespace geneo {

#define Q1_MAXP 128  // maximum parts per axis

struct Q1Geom {
  int dim, ncomp, nsub, ovl, dirichlet, pou;
  int element;              // GENEO_ELEM_Q1 or GENEO_ELEM_S20
  int ne[3], nn[3], parts[3];
  double h[3], load[3], vol;
  double wq[8];             // Gauss weight times element volume
  double grad[8][8][3];     // physical shape-function gradients [point][vertex][axis]
  double kref[8][8];        // Darcy element matrix for kappa = 1
  int elo[3][Q1_MAXP], ehi[3][Q1_MAXP];  // overlapping element range per part
  // serendipity bricks: physical shape-function gradients at the 27 Gauss
  // points [point][node][axis], weights times the Jacobian, and the
  // integral of every shape function over a brick
  double s20grad[27][20][3];
  double s20wq[27];
  double s20load[20];
};

int q1_make_geom(const geneo_grid_t* grid, Q1Geom* g, std::string* err);
void q1_sizes(const Q1Geom& g, geneo_q1_sizes_t* s);
// tau[j] = delta_j / H_j for every subdomain (host): see geneo_q1_thm1_tau
void q1_thm1_tau(const Q1Geom& g, double* tau);
// 20-node serendipity bricks (s20.hip): tables of the reference element,
// sizes and the assembly launches (same outputs as for Q1)
void s20_tables(Q1Geom* g);
void s20_sizes(const Q1Geom& g, geneo_q1_sizes_t* s);
hipError_t s20_launch_all(const Q1Geom* dgeom, const Q1Geom& g, const geneo_q1_sizes_t& s,
                          const double* coeff, int* A_rowptr, int* A_col, double* A_val,
                          double* b, int* sub_ptr, int* sub_idx, uint8_t* flags, double* pou,
                          int* loc_rowptr, int* loc_col, double* an, double* ao,
                          hipStream_t st);
hipError_t q1_launch_all(const Q1Geom* dgeom, const Q1Geom& g, const geneo_q1_sizes_t& s,
                         const double* coeff, int* A_rowptr, int* A_col, double* A_val,
                         double* b, int* sub_ptr, int* sub_idx, uint8_t* flags, double* pou,
                         int* loc_rowptr, int* loc_col, double* an, double* ao,
                         int64_t* nzoff, hipStream_t st);

}  // namespace geneo
