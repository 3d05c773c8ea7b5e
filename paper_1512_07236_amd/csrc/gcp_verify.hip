// gcp_verify.hip -- FP64 checks of a density matrix against H (gfx950).
//
// For a symmetric D and H (both read as their symmetric parts):
//   Tr D and ||D||_F^2      -- a projector has both equal to N (the trace and
//                              Frobenius tests that follow the convergence
//                              discussion; ||D||_F^2 is read as the square)
//   ||D^2 - D||_F           -- idempotency, from an FP64 MFMA product D D
//   Tr(D H) = sum D o H     -- the energy, equal to the sum of the N lowest
//                              eigenvalues of H for the ground-state projector
//   ||H D - D H||_F         -- the commutator, from an FP64 MFMA product H D
//                              (D H = (H D)^T for symmetric H and D)
// Every sum is FP64 and reduced in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcp_encode.h"
#include "gcp_kernels.h"
#include "gcp_mma.h"

namespace gcp {

// MODE 0: D D over upper tiles, per-tile sums of w_ij (X_ij - D_ij)^2 (no
// store).  MODE 1: H D over all tiles (rows of H against rows of D), stored.
template <int MODE>
__global__ __launch_bounds__(NTH, 2) void k_vgemm(VerifyArgs a) {
  using T = double;
  __shared__ __attribute__((aligned(16))) T smem[MmaCfg<GCP_FP64>::SMEM];
  const int64_t Mp = a.Mp;
  int ti, tj, lin = 0;
  if constexpr (MODE == 1) {
    const int L = (int)blockIdx.x;
    ti = L / a.nt;
    tj = L % a.nt;
  } else {
    tile_of_block(blockIdx.x, a.nt, ti, tj, lin);
  }
  const int64_t arow0 = (int64_t)ti * TILE, brow0 = (int64_t)tj * TILE;
  const T *__restrict__ D = a.D;
  const T *Al = MODE == 0 ? D : a.H;
  v4d acc[4][4];
  mma_tile<GCP_FP64>(Al, D, arow0, brow0, Mp, Mp * Mp, smem, 0, acc);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, l16 = lane & 15, lg = lane >> 4;
  const bool diag_tile = ti == tj;
  double tsum = 0.0;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = arow0 + wm * 64 + bi * 16 + acc_row<0>(lg, r);
        const int64_t j = brow0 + wn * 64 + bj * 16 + l16;
        const double v = acc[bi][bj][r];
        if constexpr (MODE == 1) {
          a.HD[i * Mp + j] = v;
        } else {
          if (diag_tile && i > j) continue;
          const double d = v - D[i * Mp + j];
          tsum += (i == j ? 1.0 : 2.0) * d * d;
        }
      }
  if constexpr (MODE == 0) {
    __shared__ double red[4];
    tsum += shfl_xor_d(tsum, 1);
    tsum += shfl_xor_d(tsum, 2);
    tsum += shfl_xor_d(tsum, 4);
    tsum += shfl_xor_d(tsum, 8);
    tsum += shfl_xor_d(tsum, 16);
    tsum += shfl_xor_d(tsum, 32);
    if (lane == 0) red[wave] = tsum;
    __syncthreads();
    if (tid == 0) a.tpart[lin] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

// Per row i (one block): sum_{j>i} (HD_ij - HD_ji)^2, sum_j D_ij H_ij,
// sum_j D_ij^2 and D_ii into rows[k * Mp + i].
__global__ __launch_bounds__(256) void k_vrows(VerifyArgs a) {
  __shared__ double s[3][256];
  const int64_t i = blockIdx.x, Mp = a.Mp;
  double c = 0.0, e = 0.0, f = 0.0;
  for (int64_t j = threadIdx.x; j < Mp; j += 256) {
    const double d = a.D[i * Mp + j];
    e += d * a.H[i * Mp + j];
    f += d * d;
    if (j > i) {
      const double x = a.HD[i * Mp + j] - a.HD[j * Mp + i];
      c += x * x;
    }
  }
  s[0][threadIdx.x] = c;
  s[1][threadIdx.x] = e;
  s[2][threadIdx.x] = f;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.rows[i] = s[0][0];
    a.rows[Mp + i] = s[1][0];
    a.rows[2 * Mp + i] = s[2][0];
    a.rows[3 * Mp + i] = a.D[i * Mp + i];
  }
}

// out[0..3] = fixed-order sums of the four row vectors, out[4] = sum of the
// idempotency tile partials.
__global__ __launch_bounds__(256) void k_vsum(VerifyArgs a) {
  __shared__ double s[5][256];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < a.Mp; i += 256)
    for (int k = 0; k < 4; ++k) v[k] += a.rows[k * a.Mp + i];
  for (int t = threadIdx.x; t < a.ntri; t += 256) v[4] += a.tpart[t];
  for (int k = 0; k < 5; ++k) s[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 5; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) a.out[threadIdx.x] = s[threadIdx.x][0];
}

hipError_t launch_verify(const VerifyArgs &a, hipStream_t st) {
  const unsigned ntri = (unsigned)(a.nt * (a.nt + 1) / 2);
  k_vgemm<0><<<ntri, NTH, 0, st>>>(a);
  k_vgemm<1><<<(unsigned)(a.nt * a.nt), NTH, 0, st>>>(a);
  k_vrows<<<(unsigned)a.Mp, 256, 0, st>>>(a);
  k_vsum<<<1, 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace gcp
