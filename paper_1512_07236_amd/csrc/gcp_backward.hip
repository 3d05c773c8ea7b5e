// gcp_backward.hip -- adjoint of the purification (reverse mode), gfx950.
//
// Given Gbar_p = dL/dD_p of the returned matrix, every update
// D' = a D + b D^2 + e D^3, with (a, b, e) functions of
// c = (T2 - T3)/(T1 - T2) (eq. (hpcp3): 1 - 2c, 2 + 2c, -2; eqs.
// (pm1a)/(pm1b) for PMCP; update_coefs), is differentiated by hand for
// symmetric D and Gbar' (= dL/dD'):
//
//   Gbar = a Gbar' + b (D Gbar' + Gbar' D) + e (D^2 Gbar' + Gbar' D^2 + D Gbar' D)
//          + kappa [(2 D - 3 D^2) - c (I - 2 D)] / (T1 - T2),
//   kappa = <Gbar', dD'/dc> = a' <Gbar', D> + b' <Gbar', D^2> + e' <Gbar', D^3>
//
// (Frobenius products; a', b', e' from update_coef_derivs; <Gbar', D^3> =
// <D^2, D Gbar'>, needed only when e' != 0, i.e. for PMCP).
//
// One adjoint step is three launches of 128 x 128 MFMA tile products, all of
// the A * B^T row-panel form of the forward (every operand is symmetric
// except AT and CT, which are only ever read along their rows):
//   mode 0 (upper tiles)  X2 = D D           epilogue: per-tile sums of
//                                            w_ij Gbar'_ij X2_ij and w_ij Gbar'_ij D_ij
//   mode 1 (all tiles)    AT = D Gbar'  and  CT = X2 Gbar'   (one launch;
//                                            PMCP: per-tile sums of X2 o AT)
//   mode 2 (upper tiles)  E  = D (Gbar' D)   epilogue: Gbar_n from Gbar', AT,
//                                            AT^T, CT, CT^T, E, D and X2
// with AT + AT^T = D Gbar' + Gbar' D and CT + CT^T = D^2 Gbar' + Gbar' D^2.
// Algorithmic cost per step: two symmetric products (M^3 each, upper-triangle
// output) and two general ones (2 M^3 each).  kappa is reduced on the device
// in a fixed order, so the whole backward is bitwise reproducible.
//
// The initial guess D_0 = theta I + beta (mu I - H), mu = Tr(H)/M.  With a
// fixed slope rule (eqs. (dmguess),(pmcpguess), or eq. (hpcpguess) with a
// fixed alpha) and the spectral bounds held fixed,
//   dL/dH = -beta Gbar_0 + (I/M) [beta Tr Gbar_0 + beta'(mu) <Gbar_0, mu I - H>],
// where <Gbar_0, mu I - H> = (<Gbar_0, D_0> - theta Tr Gbar_0) / beta, so H is
// not needed again, and beta' belongs to the active branch of the min.  The
// alpha search of eq. (hpcpguessalpha) sets beta = sqrt((target - N theta)/S)
// with S = ||mu I - H||_F^2 (alpha strictly inside (0, 1)); then beta' = 0
// and d beta = (beta / S) <mu I - H, dH> adds
//   (<Gbar_0, mu I - H> / S) (D_0 - theta I)     (= (beta <Gbar_0, g>/S) g).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcp_encode.h"
#include "gcp_kernels.h"
#include "gcp_mma.h"

namespace gcp {

// All tiles of the nt x nt grid, in groups of TILE_GROUP tile rows,
// column-major inside a group: consecutive blocks share the right-hand
// (column) panel and cycle over the group's row panels.
__device__ __forceinline__ void full_tile_of_block(int L, int nt, int &ti, int &tj) {
  const int gr = L / (TILE_GROUP * nt);
  const int r0 = gr * TILE_GROUP, rows = min(TILE_GROUP, nt - r0);
  const int rem = L - gr * TILE_GROUP * nt;
  ti = r0 + rem % rows;
  tj = rem / rows;
}

// Contiguous run of [0, total) for the XCD that block b is dispatched to.
__device__ __forceinline__ int xcd_linear(int b, int total) {
  const int xcd = b & 7, loc = b >> 3, q = total >> 3, r = total & 7;
  return xcd * q + (xcd < r ? xcd : r) + loc;
}

template <int P, int MODE>
__global__ __launch_bounds__(NTH, 2) void k_bgemm(BwdArgs a) {
  using E = Enc<P>;
  using T = typename E::T;
  constexpr int KIND = E::KIND;
  using Acc = typename AccType<KIND>::type;
  static_assert(E::NP == 1, "the adjoint uses single-plane FP64 / FP32 storage");

  __shared__ __attribute__((aligned(16))) T smem[MmaCfg<P>::SMEM];
  __shared__ double red[4];

  const int64_t Mp = a.Mp;
  int ti, tj, lin = 0, which = 0;
  if constexpr (MODE == 1) {
    const int nfull = a.nt * a.nt;
    int L = xcd_linear(blockIdx.x, 2 * nfull);
    which = L >= nfull;
    full_tile_of_block(L - which * nfull, a.nt, ti, tj);
  } else {
    tile_of_block(blockIdx.x, a.nt, ti, tj, lin);
  }
  const int64_t arow0 = (int64_t)ti * TILE, brow0 = (int64_t)tj * TILE;
  const T *__restrict__ D = (const T *)a.D;
  const T *__restrict__ X2 = (const T *)a.X2;
  const T *__restrict__ G = (const T *)a.G;
  const T *__restrict__ AT = (const T *)a.AT;
  const T *__restrict__ CT = (const T *)a.CT;
  const T *Al, *Bl;
  if constexpr (MODE == 0) {
    Al = D;
    Bl = D;
  } else if constexpr (MODE == 1) {
    Al = which ? X2 : D;
    Bl = G;
  } else {
    Al = D;
    Bl = AT;
  }

  Acc acc[4][4];
  mma_tile<P>(Al, Bl, arow0, brow0, Mp, Mp * Mp, smem, 0, acc);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, l16 = lane & 15, lg = lane >> 4;

  if constexpr (MODE == 1) {
    T *__restrict__ O = (T *)(which ? a.out1 : a.out0);
    const bool x3 = a.need_x3 && !which;   // block-uniform
    double xsum = 0.0;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = arow0 + wm * 64 + bi * 16 + acc_row<KIND>(lg, r);
          const int64_t j = brow0 + wn * 64 + bj * 16 + l16;
          const T o = (T)acc[bi][bj][r];
          O[i * Mp + j] = o;
          if (x3) xsum += (double)X2[i * Mp + j] * (double)o;
        }
    if (x3) {
      xsum += shfl_xor_d(xsum, 1);
      xsum += shfl_xor_d(xsum, 2);
      xsum += shfl_xor_d(xsum, 4);
      xsum += shfl_xor_d(xsum, 8);
      xsum += shfl_xor_d(xsum, 16);
      xsum += shfl_xor_d(xsum, 32);
      if (lane == 0) red[wave] = xsum;
      __syncthreads();
      if (tid == 0) {
        const int ntri = a.nt * (a.nt + 1) / 2;
        a.tpart[2 * ntri + ti * a.nt + tj] = ((red[0] + red[1]) + red[2]) + red[3];
      }
    }
    return;
  }

  const bool diag_tile = (ti == tj);
  T *__restrict__ O = (T *)a.out0;
  double tsum = 0.0, dsum = 0.0;
  const double kappa = MODE == 2 ? *a.kappa : 0.0;
  // The inputs of BJC column blocks of a row block are loaded before any of
  // their stores: read per element after the stores before it, each would
  // wait for them (the compiler cannot tell the output from the inputs).
  // (FP64 takes one block at a time, and in mode 2 two of its rows: more
  // would spill.)
  constexpr int BJC = sizeof(T) == 8 ? 1 : 2;
  constexpr int RC = sizeof(T) == 8 && MODE == 2 ? 2 : 4;
  constexpr int NIN = MODE == 0 ? 2 : 7;   // D, G (and X2, AT, AT^T, CT, CT^T)
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int b0 = 0; b0 < 4; b0 += BJC)
#pragma unroll
      for (int r0 = 0; r0 < 4; r0 += RC) {
        T in[BJC][RC][NIN];
#pragma unroll
        for (int q = 0; q < BJC; ++q)
#pragma unroll
          for (int rr = 0; rr < RC; ++rr) {
            const int r = r0 + rr;
            const int64_t i = arow0 + wm * 64 + bi * 16 + acc_row<KIND>(lg, r);
            const int64_t j = brow0 + wn * 64 + (b0 + q) * 16 + l16;
            in[q][rr][0] = D[i * Mp + j];
            in[q][rr][1] = G[i * Mp + j];
            if constexpr (MODE == 2) {
              in[q][rr][2] = X2[i * Mp + j];
              in[q][rr][3] = AT[i * Mp + j];
              in[q][rr][4] = AT[j * Mp + i];
              in[q][rr][5] = CT[i * Mp + j];
              in[q][rr][6] = CT[j * Mp + i];
            }
          }
#pragma unroll
        for (int q = 0; q < BJC; ++q)
#pragma unroll
          for (int rr = 0; rr < RC; ++rr) {
            const int bj = b0 + q, r = r0 + rr;
            const int64_t i = arow0 + wm * 64 + bi * 16 + acc_row<KIND>(lg, r);
            const int64_t j = brow0 + wn * 64 + bj * 16 + l16;
            if (diag_tile && i > j) continue;   // covered by the mirror of (j, i)
            const double v = (double)acc[bi][bj][r];
            const double d = (double)in[q][rr][0];
            double o;
            if constexpr (MODE == 0) {
              o = v;
              const double wg = ((i == j) ? 1.0 : 2.0) * (double)in[q][rr][1];
              tsum += wg * (double)(T)v;
              dsum += wg * d;
            } else {
              const double g = (double)in[q][rr][1];
              const double x2 = (double)in[q][rr][2];
              const double at = (double)in[q][rr][3] + (double)in[q][rr][4];
              const double ct = (double)in[q][rr][5] + (double)in[q][rr][6];
              const double gc = ((2.0 * d - 3.0 * x2) - a.c * ((i == j ? 1.0 : 0.0) - 2.0 * d)) * a.inv_t12;
              o = a.a * g + a.b * at + a.e * (ct + v) + kappa * gc;
            }
            O[i * Mp + j] = (T)o;
            if (i != j) O[j * Mp + i] = (T)o;
          }
      }

  if constexpr (MODE == 0) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      tsum += shfl_xor_d(tsum, m);
      dsum += shfl_xor_d(dsum, m);
    }
    __shared__ double red2[4];
    if (lane == 0) {
      red[wave] = tsum;
      red2[wave] = dsum;
    }
    __syncthreads();
    if (tid == 0) {
      const int ntri = a.nt * (a.nt + 1) / 2;
      a.tpart[lin] = ((red[0] + red[1]) + red[2]) + red[3];
      a.tpart[ntri + lin] = ((red2[0] + red2[1]) + red2[2]) + red2[3];
    }
  }
}

// Sum of tpart[t0 .. t1) in a fixed order by the 256 threads of one block.
__device__ double block_sum(const double *tpart, int t0, int t1, double *s) {
  double v = 0.0;
  for (int t = t0 + (int)threadIdx.x; t < t1; t += 256) v += tpart[t];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

// kappa = da <G, D> + db <G, D^2> + de <G, D^3> from the per-tile sums, in a
// fixed order (one block).
__global__ __launch_bounds__(256) void k_bkappa(const double *tpart, int ntri, int nfull,
                                                double da, double db, double de, double *kappa) {
  __shared__ double s[256];
  const double sx2 = block_sum(tpart, 0, ntri, s);
  const double sd = block_sum(tpart, ntri, 2 * ntri, s);
  const double sx3 = de != 0.0 ? block_sum(tpart, 2 * ntri, 2 * ntri + nfull, s) : 0.0;
  if (threadIdx.x == 0) *kappa = da * sd + db * sx2 + de * sx3;
}

// Iterate D_n of the forward (operand planes of encoding PF plus the exact
// FP64 diagonal) as a plain Mp x Mp matrix in the adjoint's storage type.
template <int PF, int PB>
__global__ __launch_bounds__(256) void k_bstore(const void *planes, const double *dg, int64_t Mp,
                                                void *out) {
  using EF = Enc<PF>;
  using TF = typename EF::T;
  using TB = typename Enc<PB>::T;
  // rows on the x dimension of the grid (no 64K limit), 256 columns per block on y
  const int64_t i = blockIdx.x;
  const int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x;
  double x;
  if (i == j) {
    x = dg[i];
  } else {
    TF p[EF::NP];
#pragma unroll
    for (int q = 0; q < EF::NP; ++q) p[q] = ((const TF *)planes)[eoff<PF>(i, j, q, Mp)];
    x = EF::dec(p);
  }
  ((TB *)out)[i * Mp + j] = (TB)x;
}

// G = (g + g^T)/2 of the caller's M x M gradient over 64 x 64 tiles of the
// padded matrix (zero outside M x M).
template <int PB>
__global__ __launch_bounds__(256) void k_bload(const void *g, int64_t ldg, int dtype, int64_t M,
                                               int64_t Mp, void *G) {
  using TB = typename Enc<PB>::T;
  __shared__ double hs[64][65], ht[64][65];
  const int64_t I = (int64_t)blockIdx.y * 64, J = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x, row = tid >> 2, c0 = (tid & 3) * 16;
  auto ld = [&](int64_t r, int64_t c) -> double {
    if (r >= M || c >= M) return 0.0;
    return dtype == GCP_DTYPE_F64 ? ((const double *)g)[r * ldg + c]
                                  : (double)((const float *)g)[r * ldg + c];
  };
  for (int c = 0; c < 16; ++c) {
    hs[row][c0 + c] = ld(I + row, J + c0 + c);
    ht[row][c0 + c] = ld(J + row, I + c0 + c);
  }
  __syncthreads();
  for (int c = 0; c < 16; ++c) {
    const int64_t i = I + row, j = J + c0 + c;
    ((TB *)G)[i * Mp + j] = (TB)(0.5 * (hs[row][c0 + c] + ht[c0 + c][row]));
  }
}

// Row sums of G0 o D0 and the diagonal of G0 (one block per row).
template <int PB>
__global__ __launch_bounds__(256) void k_bdot(BwdInitArgs a) {
  using TB = typename Enc<PB>::T;
  __shared__ double s[256];
  const int64_t i = blockIdx.x;
  const TB *G0 = (const TB *)a.G0, *D0 = (const TB *)a.D0;
  double v = 0.0;
  for (int64_t j = threadIdx.x; j < a.Mp; j += 256)
    v += (double)G0[i * a.Mp + j] * (double)D0[i * a.Mp + j];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.rows[i] = s[0];
    a.rows[a.Mp + i] = (double)G0[i * a.Mp + i];
  }
}

// sums[0] = <G0, D0>, sums[1] = Tr G0 (fixed order, one block).
__global__ __launch_bounds__(256) void k_bsum(BwdInitArgs a) {
  __shared__ double s0[256], s1[256];
  double v0 = 0.0, v1 = 0.0;
  for (int64_t i = threadIdx.x; i < a.Mp; i += 256) {
    v0 += a.rows[i];
    v1 += a.rows[a.Mp + i];
  }
  s0[threadIdx.x] = v0;
  s1[threadIdx.x] = v1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.sums[0] = s0[0];
    a.sums[1] = s1[0];
  }
}

// dL/dH = sign (-beta G0 + s I) (M x M, leading dimension ldh).
template <int PB>
__global__ __launch_bounds__(256) void k_bdh(BwdInitArgs a) {
  using TB = typename Enc<PB>::T;
  // rows on the x dimension of the grid (no 64K limit), 256 columns per block on y
  const int64_t i = blockIdx.x;
  const int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (j >= a.M) return;
  double s = 0.0, k = 0.0;
  if (a.beta != 0.0) {
    const double gd = a.sums[0], tr = a.sums[1];
    const double g_muh = (gd - a.theta * tr) / a.beta;   // <G0, mu I - H>
    s = (a.beta * tr + a.dbeta * g_muh) / (double)a.M;
    if (a.hdev > 0.0) k = g_muh / a.hdev;               // alpha-searched slope
  }
  double x = -a.beta * (double)((const TB *)a.G0)[i * a.Mp + j];
  if (k != 0.0) x += k * (double)((const TB *)a.D0)[i * a.Mp + j];
  if (i == j) x += s - k * a.theta;
  x *= a.sign;
  if (a.dtype == GCP_DTYPE_F64)
    ((double *)a.dH)[i * a.ldh + j] = x;
  else
    ((float *)a.dH)[i * a.ldh + j] = (float)x;
}

// ---------------------------------------------------------------- dispatch
template <int PF>
static hipError_t store_pf(int bprec, const void *planes, const double *dg, int64_t Mp, void *out,
                           hipStream_t st) {
  const dim3 grid((unsigned)Mp, (unsigned)(Mp / 256));
  if (bprec == GCP_FP64)
    k_bstore<PF, GCP_FP64><<<grid, 256, 0, st>>>(planes, dg, Mp, out);
  else
    k_bstore<PF, GCP_FP32><<<grid, 256, 0, st>>>(planes, dg, Mp, out);
  return hipGetLastError();
}

hipError_t launch_bwd_store(int fprec, int bprec, const void *planes, const double *dg, int64_t Mp,
                            void *out, hipStream_t st) {
  if (bprec != GCP_FP64 && bprec != GCP_FP32) return hipErrorInvalidValue;
  switch (fprec) {
    case GCP_FP64: return store_pf<GCP_FP64>(bprec, planes, dg, Mp, out, st);
    case GCP_FP32: return store_pf<GCP_FP32>(bprec, planes, dg, Mp, out, st);
    case GCP_BF16: return store_pf<GCP_BF16>(bprec, planes, dg, Mp, out, st);
    case GCP_FP16: return store_pf<GCP_FP16>(bprec, planes, dg, Mp, out, st);
    case GCP_BF16X3: return store_pf<GCP_BF16X3>(bprec, planes, dg, Mp, out, st);
    case GCP_FP16X3: return store_pf<GCP_FP16X3>(bprec, planes, dg, Mp, out, st);
    case GCP_BF16X6: return store_pf<GCP_BF16X6>(bprec, planes, dg, Mp, out, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_bwd_load(int bprec, const void *g, int64_t ldg, int dtype, int64_t M,
                           int64_t Mp, void *G, hipStream_t st) {
  const dim3 grid((unsigned)(Mp / 64), (unsigned)(Mp / 64));
  if (bprec == GCP_FP64)
    k_bload<GCP_FP64><<<grid, 256, 0, st>>>(g, ldg, dtype, M, Mp, G);
  else if (bprec == GCP_FP32)
    k_bload<GCP_FP32><<<grid, 256, 0, st>>>(g, ldg, dtype, M, Mp, G);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int P>
static hipError_t bgemm_p(const BwdArgs &a, hipStream_t st) {
  const unsigned ntri = (unsigned)(a.nt * (a.nt + 1) / 2);
  switch (a.mode) {
    case 0: k_bgemm<P, 0><<<ntri, NTH, 0, st>>>(a); break;
    case 1: k_bgemm<P, 1><<<(unsigned)(2 * a.nt * a.nt), NTH, 0, st>>>(a); break;
    case 2: k_bgemm<P, 2><<<ntri, NTH, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bwd_gemm(int bprec, const BwdArgs &a, hipStream_t st) {
  if (bprec == GCP_FP64) return bgemm_p<GCP_FP64>(a, st);
  if (bprec == GCP_FP32) return bgemm_p<GCP_FP32>(a, st);
  return hipErrorInvalidValue;
}

hipError_t launch_bwd_kappa(const double *tpart, int ntri, int nfull, double da, double db,
                            double de, double *kappa, hipStream_t st) {
  k_bkappa<<<1, 256, 0, st>>>(tpart, ntri, nfull, da, db, de, kappa);
  return hipGetLastError();
}

hipError_t launch_bwd_init(int bprec, const BwdInitArgs &a, hipStream_t st) {
  const dim3 gout((unsigned)a.M, (unsigned)((a.M + 255) / 256));
  if (bprec == GCP_FP64) {
    k_bdot<GCP_FP64><<<(unsigned)a.Mp, 256, 0, st>>>(a);
    k_bsum<<<1, 256, 0, st>>>(a);
    k_bdh<GCP_FP64><<<gout, 256, 0, st>>>(a);
  } else if (bprec == GCP_FP32) {
    k_bdot<GCP_FP32><<<(unsigned)a.Mp, 256, 0, st>>>(a);
    k_bsum<<<1, 256, 0, st>>>(a);
    k_bdh<GCP_FP32><<<gout, 256, 0, st>>>(a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gcp
