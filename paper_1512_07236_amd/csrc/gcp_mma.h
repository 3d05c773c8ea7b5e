// gcp_mma.h -- MFMA building blocks shared by the forward and adjoint kernels.
//
// A 128 x 128 output tile of an A * B^T product of row panels (A rows
// arow0.., B rows brow0.., both Mp x Mp row-major, K contiguous) computed by
// 4 waves in a 2 x 2 grid of 64 x 64, each a 4 x 4 grid of 16 x 16 MFMA
// blocks.  FP64 uses v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcp_encode.h"
#include "gcp_kernels.h"

namespace gcp {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int TILE = 128;   // output tile edge
constexpr int NTH = 256;    // threads per tile: 4 waves in a 2 x 2 grid of 64 x 64

template <int KIND> struct AccType { using type = v4f; };
template <> struct AccType<0> { using type = v4d; };

// 16x16 output block per MFMA; lane l holds column l%16 and four rows r = 0..3:
// rows 4*(l/16)+r for the FP32-accumulating instructions, rows (l/16)+4r for
// the FP64 one.  A/B fragments: lane l supplies row l%16 of its operand at K
// offsets determined by l/16 (the same for A and B, so the K order inside an
// instruction never matters).
template <int KIND>
__device__ __forceinline__ int acc_row(int lg, int r) {
  return KIND == 0 ? lg + 4 * r : 4 * lg + r;
}
__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <int KIND>
__device__ __forceinline__ v4f mfma16(v4u a, v4u b, v4f c) {
  if constexpr (KIND == 2)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8b, a),
                                                   __builtin_bit_cast(v8b, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a),
                                                  __builtin_bit_cast(v8h, b), c, 0, 0, 0);
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }

// Upper-triangle tiles are ordered in G x G groups of the tile grid (the
// diagonal groups are triangular), row-major inside a group; tile_of_index
// gives tile L of that order.
constexpr int TILE_GROUP = 8;

__device__ __forceinline__ void tile_of_index(int L, int nt, int &ti, int &tj) {
  const int ng = (nt + TILE_GROUP - 1) / TILE_GROUP;
  for (int gr = 0; gr < ng; ++gr) {
    const int r0 = gr * TILE_GROUP, r1 = min(nt, r0 + TILE_GROUP);
    for (int gc = gr; gc < ng; ++gc) {
      const int c0 = gc * TILE_GROUP, c1 = min(nt, c0 + TILE_GROUP);
      for (int t = r0; t < r1; ++t) {
        const int first = (gc == gr) ? t : c0;   // diagonal group: tj >= ti
        const int len = c1 - first;
        if (L < len) {
          ti = t;
          tj = first + L;
          return;
        }
        L -= len;
      }
    }
  }
  ti = tj = 0;   // not reached for L < nt (nt + 1) / 2
}

// Tile of block b of the first nblk blocks, which cover tiles 0 .. nblk-1 of
// that order.  Blocks are dispatched round-robin over the 8 XCDs; each XCD
// gets a contiguous run of the order, so the ~64 tiles resident on one XCD
// at a time fall in one group and read about 2G row panels, which its L2
// serves.
__device__ __forceinline__ void tile_of_block(int b, int nblk, int nt, int &ti, int &tj, int &lin) {
  const int xcd = b & 7, loc = b >> 3, q = nblk >> 3, r = nblk & 7;
  lin = xcd * q + (xcd < r ? xcd : r) + loc;
  tile_of_index(lin, nt, ti, tj);
}

__device__ __forceinline__ void tile_of_block(int b, int nt, int &ti, int &tj, int &lin) {
  tile_of_block(b, nt * (nt + 1) / 2, nt, ti, tj, lin);
}

// LDS geometry of the FP64 / FP32 tile product: K stages of 128 bytes per
// row, double-buffered through registers, one 16-byte chunk of row padding.
template <int P> struct MmaCfg {
  using T = typename Enc<P>::T;
  static constexpr int NP = Enc<P>::NP, ES = (int)sizeof(T);
  static constexpr int KT = 128 / ES;              // K per LDS stage
  static constexpr int EPC = 16 / ES;              // elements per 16-byte chunk
  static constexpr int LDR = KT + EPC;             // LDS row stride
  static constexpr int CPR = KT / EPC;             // chunks per row per plane
  static constexpr int CPT = TILE * CPR / NTH;     // chunks per thread per operand per plane
  static constexpr int SMEM = 2 * NP * TILE * LDR; // elements of LDS
};

// acc[bi][bj] = A[arow0 + wm*64 + bi*16 .. , K] * B[brow0 + wn*64 + bj*16 .., K]^T
// over the K stages [kb, ke) of KT values each (ke < 0: the whole K = Mp).
// Planes of a multi-plane operand are PS elements apart (FP64 / FP32 storage
// has one).  FP32 accumulates each run of `fold` K stages in a chunk
// accumulator and adds it into a running total (fold <= 0: fp32_fold(Mp));
// FP64 keeps one accumulator.  Ends with a barrier: smem is free.
template <int P>
__device__ __forceinline__ void mma_tile(const typename Enc<P>::T *__restrict__ Ag,
                                         const typename Enc<P>::T *__restrict__ Bg,
                                         int64_t arow0, int64_t brow0, int64_t Mp, int64_t PS,
                                         typename Enc<P>::T *smem, int fold,
                                         typename AccType<Enc<P>::KIND>::type (&acc)[4][4],
                                         int kb = 0, int ke = -1) {
  using C = MmaCfg<P>;
  using T = typename C::T;
  constexpr int NP = C::NP, KT = C::KT, EPC = C::EPC, LDR = C::LDR, CPR = C::CPR, CPT = C::CPT;
  static_assert(Enc<P>::KIND <= 1, "16-bit encodings use the paired-tile kernel");
  using Acc = typename AccType<Enc<P>::KIND>::type;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, l16 = lane & 15, lg = lane >> 4;
  T *As = smem;
  T *Bs = smem + NP * TILE * LDR;

  v4u ra[NP][CPT], rb[NP][CPT];
  auto gload = [&](int kt) {
    const int64_t k0 = (int64_t)kt * KT;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int ch = tid + c * NTH, row = ch / CPR, kc = ch % CPR;
        ra[p][c] = *(const v4u *)(Ag + p * PS + (arow0 + row) * Mp + k0 + kc * EPC);
        rb[p][c] = *(const v4u *)(Bg + p * PS + (brow0 + row) * Mp + k0 + kc * EPC);
      }
  };
  auto swrite = [&]() {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int ch = tid + c * NTH, row = ch / CPR, kc = ch % CPR;
        *(v4u *)(As + (p * TILE + row) * LDR + kc * EPC) = ra[p][c];
        *(v4u *)(Bs + (p * TILE + row) * LDR + kc * EPC) = rb[p][c];
      }
  };

  constexpr bool FOLD = Enc<P>::KIND == 1;
  Acc tot[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = tot[bi][bj] = Acc{};

  const int nk = ke < 0 ? (int)(Mp / KT) : ke;
  const int f = fold > 0 ? fold : fp32_fold(Mp);
  gload(kb);
  swrite();
  __syncthreads();
  for (int kt = kb; kt < nk; ++kt) {
    if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      T bf[4];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) bf[bj] = Bs[(wn * 64 + bj * 16 + l16) * LDR + ks * 4 + lg];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) {
        const T af = As[(wm * 64 + bi * 16 + l16) * LDR + ks * 4 + lg];
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma(af, bf[bj], acc[bi][bj]);
      }
    }
    if (FOLD && ((kt - kb + 1) % f == 0 || kt == nk - 1)) {
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
          tot[bi][bj] += acc[bi][bj];
          acc[bi][bj] = Acc{};
        }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      swrite();
      __syncthreads();
    }
  }
  if constexpr (FOLD) {
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = tot[bi][bj];
  }
}

}  // namespace gcp
