// Internal device helpers shared by the libgeneo kernels (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Dense local factors are stored as packed lower-triangular arrays of
// TS x TS row-major tiles: tile (i, k), k <= i, of a matrix with nt tile
// rows sits at tile index i*(i+1)/2 + k.  Matrices are padded to nt*TS with
// an identity block, so a padded factor is diag(L, I).
#define TS 32
#define TSQ (TS * TS)

__host__ __device__ inline int64_t tri_tiles(int64_t nt) { return nt * (nt + 1) / 2; }
__host__ __device__ inline int64_t tile_idx(int i, int k) { return (int64_t)i * (i + 1) / 2 + k; }

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core product, D = A*B + C on one wavefront of 64 lanes.
// Operand lane layout (both types): lane l supplies A[l%16][l/16] and
// B[l/16][l%16].  Accumulator element v of lane l holds
//   f32: D[4*(l/16) + v][l%16]        f64: D[l/16 + 4*v][l%16]
// (both checked on gfx950 by feeding random operands and matching every
// output slot against the reference product).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4_t acc;
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef f4_t acc;
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <typename T> __device__ __forceinline__ typename Mfma<T>::acc acc_zero() {
  typename Mfma<T>::acc z;
  z[0] = z[1] = z[2] = z[3] = (T)0;
  return z;
}

// Row of accumulator element v for this lane, and its column.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int v);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int acc_col(int lane) { return lane & 15; }

// Quadrant products over a K = 32 contraction.  X and Y point at the first
// row of the 16-row (or, for the transposed forms, first column of the
// 16-column) slice; ld is the row stride in elements.  TM is the storage
// type of the operands (float or double), TA the arithmetic type.
//
//   D += X[0:16, 0:32] * Y[0:16, 0:32]^T
template <typename TA, typename TX, typename TY>
__device__ __forceinline__ void q_xyT(typename Mfma<TA>::acc& acc, const TX* X, int ldx,
                                      const TY* Y, int ldy, int lane) {
  const int i = lane & 15, k = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
    acc = Mfma<TA>::run((TA)X[i * ldx + kk * 4 + k], (TA)Y[i * ldy + kk * 4 + k], acc);
}
//   D += X[0:16, 0:32] * Y[0:32, 0:16]
template <typename TA, typename TX, typename TY>
__device__ __forceinline__ void q_xy(typename Mfma<TA>::acc& acc, const TX* X, int ldx,
                                     const TY* Y, int ldy, int lane) {
  const int i = lane & 15, k = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
    acc = Mfma<TA>::run((TA)X[i * ldx + kk * 4 + k], (TA)Y[(kk * 4 + k) * ldy + i], acc);
}
//   D += X[0:32, 0:16]^T * Y[0:32, 0:16]
template <typename TA, typename TX, typename TY>
__device__ __forceinline__ void q_xTy(typename Mfma<TA>::acc& acc, const TX* X, int ldx,
                                      const TY* Y, int ldy, int lane) {
  const int i = lane & 15, k = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
    acc = Mfma<TA>::run((TA)X[(kk * 4 + k) * ldx + i], (TA)Y[(kk * 4 + k) * ldy + i], acc);
}

// Ordering point for LDS traffic exchanged between lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void block_sync() {
  __threadfence_block();
  __syncthreads();
}

// Deterministic counter-based uniform in (-1, 1): SplitMix64 finaliser of
// (seed, stream, index).
__device__ __forceinline__ double hash_uniform(uint64_t seed, uint64_t a, uint64_t b) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (a * 0x100000001B3ull + b + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return ((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}
