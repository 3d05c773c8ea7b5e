// gcp_encode.h -- operand encodings of the GPU purification path.
//
// An iterate X (D or D^2) is stored as its off-diagonal operand encoding
// (NP planes of M x M elements) plus an exact FP64 diagonal kept in separate
// vectors.  The encoded value of an off-diagonal element IS the master value
// of that element; the diagonal residual r_i = X_ii - dec(enc(X_ii)) is
// corrected exactly in the product epilogues.  enc/dec below are the only
// definition of each encoding and are used by every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gcp.h"

namespace gcp {

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round-to-nearest-even float -> bfloat16 (NaN payloads may become inf,
  // which is still non-finite)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double bf2d(uint16_t h) {
  return (double)__uint_as_float((uint32_t)h << 16);
}
__device__ __forceinline__ uint16_t f2h(float f) {
  // float -> float16, round to nearest even.  The empty asm keeps f a float
  // in a register: without it the compiler folds a preceding double -> float
  // conversion into one double -> float16 conversion, which has no
  // instruction and is emulated in about 35 integer operations per element.
  asm volatile("" : "+v"(f));
  _Float16 h = (_Float16)f;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ double h2d(uint16_t b) {
  return (double)(float)__builtin_bit_cast(_Float16, b);
}

// kind: 0 = FP64 MFMA, 1 = FP32 MFMA, 2 = BF16 MFMA, 3 = FP16 MFMA
template <int P> struct Enc;

template <> struct Enc<GCP_FP64> {
  using T = double;
  static constexpr int NP = 1, KIND = 0, NPROD = 1;
  static constexpr double PROD_SCALE = 1.0;
  __device__ static void enc(double x, T *p) { p[0] = x; }
  __device__ static double dec(const T *p) { return p[0]; }
};

template <> struct Enc<GCP_FP32> {
  using T = float;
  static constexpr int NP = 1, KIND = 1, NPROD = 1;
  static constexpr double PROD_SCALE = 1.0;
  __device__ static void enc(double x, T *p) { p[0] = (float)x; }
  __device__ static double dec(const T *p) { return (double)p[0]; }
};

template <> struct Enc<GCP_BF16> {
  using T = uint16_t;
  static constexpr int NP = 1, KIND = 2, NPROD = 1;
  static constexpr double PROD_SCALE = 1.0;
  __device__ static void enc(double x, T *p) { p[0] = f2bf((float)x); }
  __device__ static double dec(const T *p) { return bf2d(p[0]); }
};

template <> struct Enc<GCP_BF16X3> {
  using T = uint16_t;
  static constexpr int NP = 2, KIND = 2, NPROD = 3;
  static constexpr double PROD_SCALE = 1.0;
  __device__ static void enc(double x, T *p) {
    p[0] = f2bf((float)x);
    p[1] = f2bf((float)(x - bf2d(p[0])));
  }
  __device__ static double dec(const T *p) { return bf2d(p[0]) + bf2d(p[1]); }
};

template <> struct Enc<GCP_BF16X6> {
  using T = uint16_t;
  static constexpr int NP = 3, KIND = 2, NPROD = 6;
  static constexpr double PROD_SCALE = 1.0;
  __device__ static void enc(double x, T *p) {
    p[0] = f2bf((float)x);
    const double r1 = x - bf2d(p[0]);
    p[1] = f2bf((float)r1);
    p[2] = f2bf((float)(r1 - bf2d(p[1])));
  }
  __device__ static double dec(const T *p) { return bf2d(p[0]) + bf2d(p[1]) + bf2d(p[2]); }
};

// float16 encodings store 2^10 x: |x| <= 64 stays finite, and the low part
// of the split stays a normal float16 down to |x| ~ 1e-4.
constexpr double kF16Scale = 1024.0;
constexpr double kF16InvScale = 1.0 / 1024.0;

template <> struct Enc<GCP_FP16> {
  using T = uint16_t;
  static constexpr int NP = 1, KIND = 3, NPROD = 1;
  static constexpr double PROD_SCALE = kF16InvScale * kF16InvScale;
  __device__ static void enc(double x, T *p) { p[0] = f2h((float)(x * kF16Scale)); }
  __device__ static double dec(const T *p) { return h2d(p[0]) * kF16InvScale; }
};

template <> struct Enc<GCP_FP16X3> {
  using T = uint16_t;
  static constexpr int NP = 2, KIND = 3, NPROD = 3;
  static constexpr double PROD_SCALE = kF16InvScale * kF16InvScale;
  __device__ static void enc(double x, T *p) {
    const double y = x * kF16Scale;
    p[0] = f2h((float)y);
    p[1] = f2h((float)(y - h2d(p[0])));
  }
  __device__ static double dec(const T *p) { return (h2d(p[0]) + h2d(p[1])) * kF16InvScale; }
};

// Element (i, j) of plane p in the padded Mp x Mp storage of an encoding.
// Split encodings interleave their planes in blocks of 32 columns, so that
// the 32-column K slice of every plane of a row is one contiguous segment
// (128 bytes for two planes, 192 for three):
//   [row i][block j/32][plane p][j % 32].
// Single-plane encodings are one row-major matrix.
template <int P>
__host__ __device__ __forceinline__ int64_t eoff(int64_t i, int64_t j, int p, int64_t Mp) {
  constexpr int NP = Enc<P>::NP;
  if constexpr (NP >= 2)
    return i * (NP * Mp) + (j >> 5) * (32 * NP) + p * 32 + (j & 31);
  else
    return i * Mp + j;
}

}  // namespace gcp
