// gcp_kernels.hip -- device kernels of the purification path (gfx950 / CDNA4).
//
// One purification iteration (eq. (hpcp3) expanded with Dbar = I - D):
//   D_{n+1} = (1 - 2c) D + (2 + 2c) D^2 - 2 D^3,   c = (T2 - T3) / (T1 - T2),
//   T_k = Tr D^k.
// It is two symmetric matrix products, each an MFMA GEMM over the upper
// triangle of 128 x 128 output tiles (results mirrored):
//   K1 (mode 0):  X2 = D D        epilogue: store X2, row sums of X2 o D
//                                 (diag of D^3) and ||X2 - D||_F^2
//   K2 (mode 1):  X3 = X2 D       epilogue: D_{n+1} from D, X2 and X3 (X3 never
//                                 stored), row sums of D_{n+1} o D_{n+1} (diag
//                                 of D_{n+1}^2) and ||D_{n+1} - D_n||_F^2
// Both are A * B^T products of row panels (all iterates are symmetric), so
// both operands are read along contiguous K.  Row sums go to a [slot][row]
// FP64 buffer (one writer per slot) and a reduction kernel adds them in a
// fixed order: every trace, and therefore c_n, is bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gcp_encode.h"
#include "gcp_kernels.h"
#include "gcp_mma.h"

namespace gcp {

// FP64 / FP32 product kernel: one 128 x 128 upper-triangle tile per block of
// 4 waves (2 x 2 grid of 64 x 64), MFMA 16x16x4, two blocks per CU.  Blocks
// [0, nfull) compute whole tiles; each remaining tile is split along K over
// nsplit blocks (the tiles of a last partial round, or every tile of a
// product smaller than one round), whose partial tiles meet in ws and are
// added in FP64, in split order, by the last of them to finish.
template <int P>
__global__ __launch_bounds__(NTH, 2) void k_gemm(GemmArgs g) {
  using E = Enc<P>;
  using T = typename E::T;
  constexpr int NP = E::NP, KIND = E::KIND;
  using Acc = typename AccType<KIND>::type;

  __shared__ __attribute__((aligned(16))) T smem[MmaCfg<P>::SMEM];
  if (g.status && *g.status != 0) return;   // the solve has stopped

  // whole tile, or split s of a tail tile over K stages [kb, ke)
  const int nk_all = (int)(g.Mp / MmaCfg<P>::KT);
  int ti, tj, lin, split = -1, kb = 0, ke = nk_all;
  if ((int)blockIdx.x < g.nfull) {
    tile_of_block(blockIdx.x, g.nfull, g.nt, ti, tj, lin);
  } else {
    // split-major: the blocks in flight together cover the same K range of
    // consecutive tiles
    const int u = (int)blockIdx.x - g.nfull;
    const int ntail = ((int)gridDim.x - g.nfull) / g.nsplit;
    split = u / ntail;
    lin = g.nfull + u % ntail;
    tile_of_index(lin, g.nt, ti, tj);
    kb = split * nk_all / g.nsplit;
    ke = (split + 1) * nk_all / g.nsplit;
  }
  const int64_t Mp = g.Mp, PS = g.pstride;
  const int64_t arow0 = (int64_t)ti * TILE, brow0 = (int64_t)tj * TILE;
  const T *__restrict__ Ag = (const T *)g.A;
  const T *__restrict__ Bg = (const T *)g.B;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, l16 = lane & 15, lg = lane >> 4;

  Acc acc0[4][4];
  mma_tile<P>(Ag, Bg, arow0, brow0, Mp, PS, smem, g.fold, acc0, kb, ke);

  if (split >= 0) {
    // publish this split's partial tile; the last split to arrive adds all
    // of them in split order (the sum does not depend on the arrival order)
    // and runs the epilogue
    const int t = lin - g.nfull;   // index among the split tiles
    Acc *wsp = (Acc *)g.ws + ((int64_t)t * g.nsplit + split) * 16 * NTH;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) wsp[(bi * 4 + bj) * NTH + tid] = acc0[bi][bj];
    __threadfence();
    unsigned *last = (unsigned *)smem;   // the stage buffers are free
    __syncthreads();
    if (tid == 0) *last = (atomicAdd(g.cnt + t, 1u) == (unsigned)g.nsplit - 1);
    __syncthreads();
    if (!*last) return;
    __syncthreads();   // flag read by all before the epilogue reuses smem
    __threadfence();
    const Acc *w0 = (const Acc *)g.ws + (int64_t)t * g.nsplit * 16 * NTH;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 4
        for (int sp = 0; sp < g.nsplit; ++sp) {
          const Acc v = w0[((int64_t)sp * 16 + bi * 4 + bj) * NTH + tid];
          a0 += (double)v[0];
          a1 += (double)v[1];
          a2 += (double)v[2];
          a3 += (double)v[3];
        }
        acc0[bi][bj] = Acc{(T)a0, (T)a1, (T)a2, (T)a3};
      }
    if (tid == 0) g.cnt[t] = 0u;   // ready for the next launch
  }

  // ------------------------------------------------------------ epilogue
  const double S = E::PROD_SCALE;
  const bool diag_tile = (ti == tj);
  T *__restrict__ Og = (T *)g.out;
  double rowacc[4][4], colacc[4], tacc = 0.0;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi) {
    colacc[bi] = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) rowacc[bi][r] = 0.0;
  }
  double a_coef = 0.0, b_coef = 0.0, e_coef = 0.0;
  if (g.mode == 1) update_coefs(g.method, g.coef[0], a_coef, b_coef, e_coef);

  // The element inputs of BJC column blocks of a row block at a time are
  // loaded before any of their stores: read per element after the stores
  // before it, each would wait for them (the compiler cannot tell the output
  // from the inputs), one memory round trip per element.  (FP64 loads half a
  // row block: a whole one would spill.)
  constexpr int BJC = sizeof(T) == 8 ? 1 : 4;
  double rDj[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) rDj[bj] = g.rD[brow0 + wn * 64 + bj * 16 + l16];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi) {
    double rDi[4], s2i[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = arow0 + wm * 64 + bi * 16 + acc_row<KIND>(lg, r);
      rDi[r] = g.rD[i];
      s2i[r] = g.mode == 1 ? g.s2[i] : 0.0;
    }
#pragma unroll
    for (int b0 = 0; b0 < 4; b0 += BJC) {
      T dpb[BJC][4][NP], xpb[BJC][4][NP];
#pragma unroll
      for (int q = 0; q < BJC; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = arow0 + wm * 64 + bi * 16 + acc_row<KIND>(lg, r);
          const int64_t j = brow0 + wn * 64 + (b0 + q) * 16 + l16;
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            dpb[q][r][p] = Bg[p * PS + i * Mp + j];                        // D(i, j)
            xpb[q][r][p] = g.mode == 1 ? Ag[p * PS + i * Mp + j] : T{};    // X2(i, j)
          }
        }
#pragma unroll
      for (int q = 0; q < BJC; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int bj = b0 + q;
          const int64_t i = arow0 + wm * 64 + bi * 16 + acc_row<KIND>(lg, r);
          const int64_t j = brow0 + wn * 64 + bj * 16 + l16;
          if (diag_tile && i > j) continue;   // covered by the mirror of (j, i)
          const double v = (double)acc0[bi][bj][r] * S;
          const T *dp = dpb[q][r];
          T op[NP];
          double prod, diff;
          if (g.mode == 0) {
            // X2 = (D_enc + diag(rD))^2: exact diagonal-residual correction
            double Dm, x2;
            if (i == j) {
              Dm = g.dg[i];
              x2 = g.d2[i];
            } else {
              Dm = E::dec(dp);
              x2 = v + Dm * (rDi[r] + rDj[bj]);
            }
            E::enc(x2, op);
            const double x2m = (i == j) ? x2 : E::dec(op);
            if (i == j) g.s2[i] = x2 - E::dec(op);
            prod = x2m * Dm;
            diff = x2m - Dm;
          } else {
            double Dm, dn;
            if (i == j) {
              Dm = g.dg[i];
              dn = a_coef * Dm + b_coef * g.d2[i] + e_coef * g.d3[i];
            } else {
              Dm = E::dec(dp);
              const double X2m = E::dec(xpb[q][r]);
              // X3 = (X2_enc + diag(s2)) (D_enc + diag(rD))
              const double x3 = v + X2m * rDj[bj] + s2i[r] * Dm;
              dn = a_coef * Dm + b_coef * X2m + e_coef * x3;
            }
            E::enc(dn, op);
            const double dnm = (i == j) ? dn : E::dec(op);
            if (i == j) {
              g.dg_new[i] = dn;
              g.rD_new[i] = dn - E::dec(op);
            }
            prod = dnm * dnm;
            diff = dnm - Dm;
          }
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            Og[p * PS + i * Mp + j] = op[p];
            if (i != j) Og[p * PS + j * Mp + i] = op[p];
          }
          rowacc[bi][r] += prod;
          if (i != j) {
            colacc[bj] += prod;
            tacc += 2.0 * diff * diff;
          } else {
            tacc += diff * diff;
          }
        }
    }
  }

  // lane reductions (fixed order): rows over the 16 lanes of a column group,
  // columns over the 4 row groups, the tile scalar over the wave
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = rowacc[bi][r];
      v += shfl_xor_d(v, 1);
      v += shfl_xor_d(v, 2);
      v += shfl_xor_d(v, 4);
      v += shfl_xor_d(v, 8);
      rowacc[bi][r] = v;
    }
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    double v = colacc[bj];
    v += shfl_xor_d(v, 16);
    v += shfl_xor_d(v, 32);
    colacc[bj] = v;
  }
  tacc += shfl_xor_d(tacc, 1);
  tacc += shfl_xor_d(tacc, 2);
  tacc += shfl_xor_d(tacc, 4);
  tacc += shfl_xor_d(tacc, 8);
  tacc += shfl_xor_d(tacc, 16);
  tacc += shfl_xor_d(tacc, 32);

  double *rp = (double *)smem;    // [2 (wn)][128 rows]
  double *cp = rp + 2 * TILE;     // [2 (wm)][128 cols]
  double *tp = cp + 2 * TILE;     // [4 waves]
  __syncthreads();                // main-loop LDS no longer in use
  if (l16 == 0) {
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        rp[wn * TILE + wm * 64 + bi * 16 + acc_row<KIND>(lg, r)] = rowacc[bi][r];
  }
  if (lg == 0) {
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) cp[wm * TILE + wn * 64 + bj * 16 + l16] = colacc[bj];
  }
  if (lane == 0) tp[wave] = tacc;
  __syncthreads();
  if (tid < TILE) {
    const double rs = rp[tid] + rp[TILE + tid];
    const double cs = cp[tid] + cp[TILE + tid];
    if (!diag_tile) {
      g.part[(int64_t)tj * Mp + arow0 + tid] = rs;
      g.part[(int64_t)ti * Mp + brow0 + tid] = cs;
    } else {
      g.part[(int64_t)ti * Mp + arow0 + tid] = rs + cs;
    }
  }
  if (tid == 0) g.tpart[lin] = ((tp[0] + tp[1]) + tp[2]) + tp[3];
}

// ------------------------------------------------ 16-bit product kernel
// Pairs of horizontally adjacent 128 x 128 tiles, (ti, 2c) and (ti, 2c+1),
// share one row panel of the left operand: a 128 x 256 output per block of
// 8 waves (2 per SIMD), each wave 64 rows x 64 columns of one tile (4 x 4
// MFMA blocks).  The panels stream through a 3-stage LDS ring (2 stages for
// three planes), one K stage of 32 per step.  All split products of a K step
// go into one FP32 chunk accumulator, which is added into a running FP32
// total every `fold` K steps.  With r products per step and n = K/32 steps
// the rounding error then grows like sqrt(r*fold + n/fold) instead of
// sqrt(r*n): fold = sqrt(n/r) (the default) minimises it.  This accumulation
// error, not the operand encoding, bounds the accuracy of the split
// encodings at large M.  A pair may be split along K over several blocks
// (the pairs of a last partial round, or every pair with the ksplit option):
// each split folds its own K range, and the last to finish adds the splits'
// FP32 totals in FP64, in split order.
constexpr int PAIR_COLS = 2;

// Pair (ti, c) of block b, c >= ti/2, in column-major order of the pair
// triangle: consecutive blocks share the column pair (the 256-row B panel)
// and walk down the row panels.  Blocks go round-robin to the 8 XCDs, so at
// any time all XCDs stream the same B panel (served once from the Infinity
// Cache) while each keeps a few A panels in flight.  Measured on the load
// path alone, this order moves 1.3x the data per unit time of an 8 x 8
// grouped order with per-XCD contiguous ranges.
__device__ __forceinline__ void pair_of_block(int b, int nt, int &ti, int &cp, int &lin) {
  const int npc = nt / PAIR_COLS;
  int L = b;
  lin = b;
  for (int c = 0; c < npc; ++c) {
    const int len = min(nt, PAIR_COLS * c + PAIR_COLS);   // rows ti <= 2c + 1
    if (L < len) {
      ti = L;
      cp = c;
      return;
    }
    L -= len;
  }
  ti = cp = 0;
}

typedef __attribute__((address_space(3))) void lds_void;

constexpr int NW16 = 8;              // waves per block of the 16-bit kernel (2 per SIMD)
constexpr int NTH16 = 64 * NW16;

// Eight waves of 64 x 64 with 16x16x32 products (any plane count; the
// three-plane BF16X6 uses 64-byte plane segments per stage).
template <int P>
__global__ __launch_bounds__(NTH16, 1) void k_gemm16(GemmArgs g) {
  using E = Enc<P>;
  using T = uint16_t;
  constexpr int NP = E::NP, KIND = E::KIND;
  constexpr int KT = 32;                         // K per stage: one MFMA step
  constexpr int AR = TILE, BR = PAIR_COLS * TILE;
  constexpr int WCOLS = BR / (NW16 / 2);         // columns per wave (64)
  constexpr int NBJ = WCOLS / 16;                // MFMA blocks per wave row (4)
  // One- and two-plane encodings: a stage is one 128-byte segment of every
  // panel row (64 halves: 64 K values of one plane, or 32 K values of both
  // planes, which the interleaved storage keeps together).  Three-plane
  // encodings: 64-byte segments of each plane (32 K values).
  constexpr bool R128 = NP <= 2;
  constexpr int RH = R128 ? 64 : NP * KT;        // halves per panel row per stage
  constexpr int STAGE = (AR + BR) * RH;          // halves per stage
  // ring of NBUF stages, NBUF - 1 of them in flight while one is consumed
  constexpr int NBUF_FIT = (150 * 1024) / (STAGE * 2);
  constexpr int NBUF = NBUF_FIT > 4 ? 4 : (NBUF_FIT < 2 ? 2 : NBUF_FIT);
  constexpr int PD = NBUF - 1;                   // prefetch distance (stages)
  constexpr int ROWS_PER_LOAD = R128 ? 8 : 16;   // rows filled by one wave instruction
  constexpr int BLK = (R128 ? 1 : NP) * (AR + BR) / ROWS_PER_LOAD;
  static_assert(BLK % NW16 == 0, "whole blocks per wave");
  constexpr int LPS = BLK / NW16;                // loads per stage per wave
  // s_waitcnt immediate: vmcnt <= n, expcnt/lgkmcnt not waited on
  constexpr int WAIT_STEADY = ((PD - 1) * LPS & 0xF) | ((((PD - 1) * LPS) >> 4) << 14) | (0x7 << 4) | (0xF << 8);
  static_assert((PD - 1) * LPS <= 63, "vmcnt range");
  constexpr int EPLD = TILE + 4;                 // epilogue row pitch (floats)
  constexpr int WPT = NW16 / 2;                  // waves per tile in the epilogue
  constexpr int EVEC = 5 * TILE + BR;            // FP64 side vectors staged for the epilogue
  constexpr int EPI =
      (2 * TILE * EPLD * 4 + (2 + 2 * WPT) * TILE * 8 + 2 * WPT * 8 + EVEC * 8) / 2;   // halves
  constexpr int SMEM = NBUF * STAGE > EPI ? NBUF * STAGE : EPI;
  __shared__ __attribute__((aligned(16))) T smem[SMEM];
  if (g.status && *g.status != 0) return;   // the solve has stopped

  // whole pair, or split s of a tail pair over K stages [kbase, kbase + nk)
  const int nk_all = (int)(R128 ? g.Mp * NP / 64 : g.Mp / KT);
  int ti, cpair, lin, split = -1, kbase = 0, nk = nk_all;
  if ((int)blockIdx.x < g.nfull) {
    pair_of_block(blockIdx.x, g.nt, ti, cpair, lin);
  } else {
    const int u = (int)blockIdx.x - g.nfull;
    // split-major: the blocks in flight together work on the same K range
    // of consecutive pairs, which share their panels as whole pairs do
    const int ntail = ((int)gridDim.x - g.nfull) / g.nsplit;
    split = u / ntail;
    pair_of_block(g.nfull + u % ntail, g.nt, ti, cpair, lin);
    kbase = split * nk_all / g.nsplit;
    nk = (split + 1) * nk_all / g.nsplit - kbase;
  }
  const int64_t Mp = g.Mp;
  const int64_t arow0 = (int64_t)ti * TILE, brow0 = (int64_t)cpair * BR;
  const T *__restrict__ Ag = (const T *)g.A;
  const T *__restrict__ Bg = (const T *)g.B;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  // wave (rh, wc): rows rh*64 .. +63 of the panel, pair columns wc*64 .. +63
  const int rh = wave & 1, wc = wave >> 1;
  const int h = (wc * WCOLS) / TILE;             // which tile of the pair
  const int tcol0 = wc * WCOLS - h * TILE;       // first column inside that tile
  const int tj = cpair * PAIR_COLS + h;
  const bool valid = tj >= ti;

  // 128-byte rows: the 8 chunks of stage row R sit at slots c ^ (R % 8), so
  // the 16 rows an MFMA fragment read touches cover every slot twice, with
  // the two rows of a slot of opposite parity.  Measured on gfx950 with the
  // fragment pattern alone: no LDS bank conflicts (SQ_LDS_BANK_CONFLICT = 0)
  // and 176 B/clk per CU, against 2-way conflicts and 117 B/clk for the slot
  // c ^ ((R ^ (R >> 3)) % 8).  64-byte rows (three planes): 4 chunks at slots
  // c ^ ((R >> 1) ^ (R >> 3)) % 4.  Global data goes straight to LDS
  // (global_load_lds, 16 B per lane; one wave instruction fills 8 or 16
  // contiguous rows).
  auto swz = [](int R) { return R128 ? (R & 7) : (((R >> 1) ^ (R >> 3)) & 3); };
  auto issue = [&](int kt, int buf) {
    T *st = smem + buf * STAGE;
#pragma unroll
    for (int q = 0; q < LPS; ++q) {
      const int blk = wave + NW16 * q;
      if constexpr (R128) {
        const int R = blk * 8 + (lane >> 3);
        const int c = (lane & 7) ^ swz(R);
        const T *src = (R < AR ? Ag + (arow0 + R) * (NP * Mp) : Bg + (brow0 + R - AR) * (NP * Mp)) +
                       (int64_t)(kbase + kt) * 64 + c * 8;
        __builtin_amdgcn_global_load_lds((const void *)src, (lds_void *)(st + blk * 8 * 64), 16, 0, 0);
      } else {
        const int p = blk / ((AR + BR) / 16), gq = blk % ((AR + BR) / 16);
        const int R = gq * 16 + (lane >> 2);
        const int c = (lane & 3) ^ swz(R);
        const T *src = (R < AR ? Ag + (arow0 + R) * (NP * Mp) : Bg + (brow0 + R - AR) * (NP * Mp)) +
                       (int64_t)(kbase + kt) * (NP * KT) + p * KT + c * 8;
        __builtin_amdgcn_global_load_lds((const void *)src,
                                         (lds_void *)(st + (p * (AR + BR) + gq * 16) * KT), 16, 0, 0);
      }
    }
  };
  // fragment x (chunk group) of stage row R: 128-byte rows hold two groups
  // of 4 chunks (two planes, or two K halves of one plane)
  auto frag = [&](const T *st, int R, int x) -> v4u {
    if constexpr (R128)
      return *(const v4u *)(st + R * 64 + ((x * 4 + lg) ^ swz(R)) * 8);
    else
      return *(const v4u *)(st + (x * (AR + BR) + R) * KT + (lg ^ swz(R)) * 8);
  };
  constexpr int NX = R128 ? 2 : NP;              // fragment groups per stage row
  // two wave groups half a stage apart (below); the three-plane encodings
  // keep the plain loop (their fragments would not fit in the registers)
  constexpr bool PING = R128;

  v4f acc[4][NBJ], tot[4][NBJ];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < NBJ; ++bj) {
      acc[bi][bj] = v4f{};
      tot[bi][bj] = v4f{};
    }

  // products per stage (group of A, group of B), largest first: split
  // encodings pair the planes; one plane pairs the two K halves
  constexpr int NPR = NP == 1 ? 2 : E::NPROD;
  constexpr int PA[6] = {0, 0, 1, 1, 0, 2};
  constexpr int PB[6] = {0, 1, 0, 1, 2, 0};
  constexpr int QA[2] = {0, 1};

  const int fold = g.fold;   // >= 1 (resolved on the host)
  v4u af[4][NX], bf[NBJ][NX];
  auto read_frags = [&](int kt) {
    const T *st = smem + (kt % NBUF) * STAGE;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int x = 0; x < NX; ++x) af[bi][x] = frag(st, rh * 64 + bi * 16 + l16, x);
#pragma unroll
    for (int bj = 0; bj < NBJ; ++bj)
#pragma unroll
      for (int x = 0; x < NX; ++x) bf[bj][x] = frag(st, AR + wc * WCOLS + bj * 16 + l16, x);
  };
  // the products of stage kt; the chunk accumulator goes into the running
  // total after the last stage of each chunk of `fold` stages
  auto compute = [&](int kt) {
#pragma unroll
    for (int pr = 0; pr < NPR; ++pr)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < NBJ; ++bj) {
          const int xa = NP == 1 ? QA[pr] : PA[pr], xb = NP == 1 ? QA[pr] : PB[pr];
          acc[bi][bj] = mfma16<KIND>(af[bi][xa], bf[bj][xb], acc[bi][bj]);
        }
    if ((kt + 1) % fold == 0 || kt == nk - 1) {
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < NBJ; ++bj) {
          tot[bi][bj] += acc[bi][bj];
          acc[bi][bj] = v4f{};
        }
    }
  };
  // Bare s_barrier: __syncthreads() would add a workgroup release fence,
  // which waits for every outstanding LDS-DMA load and so drains the
  // pipeline.  The empty asm statements keep the compiler from moving LDS
  // accesses across it, the scheduling barriers keep the matrix products on
  // their side of it; the waits before it provide the hardware ordering.
  auto barrier = [] {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" ::: "memory");
  };
  // this wave's loads of stage kt have landed (later stages may still fly)
  // and its fragment reads are complete
  auto wait_stage = [&](int kt) {
    if (kt + PD - 1 < nk)
      __builtin_amdgcn_s_waitcnt(WAIT_STEADY & ~(0xF << 8));
    else
      __builtin_amdgcn_s_waitcnt(0);
  };
  // Waves of a tile below the diagonal run the same instruction stream (their
  // results are discarded).
#pragma unroll
  for (int s0 = 0; s0 < PD; ++s0)
    if (s0 < nk) issue(s0, s0);
  if constexpr (PING) {
    // Two wave groups, waves 0-3 (A) and 4-7 (B), one of each per SIMD, half
    // a stage apart: in the first half of stage kt A reads its fragments of
    // stage kt while B runs its products of stage kt-1; in the second half A
    // runs the products of stage kt while B reads its fragments of it.  Each
    // SIMD's matrix core is fed by one group while the other waits on LDS.
    // Each wave's products and their order are those of the plain loop.
    // A wave whose load cannot issue stalls its whole instruction stream, so
    // each group issues its share of the loads of stage kt+PD (into the
    // buffer freed at the first barrier) in its fragment-read half only.
    const bool grp_b = wave >= NW16 / 2;
    for (int kt = 0; kt <= nk; ++kt) {
      wait_stage(kt);
      barrier();   // stage kt has landed; the buffer of stage kt-1 is free
      if (!grp_b) {
        if (kt + PD < nk) issue(kt + PD, (kt + PD) % NBUF);
        if (kt < nk) read_frags(kt);
      } else if (kt > 0) {
        compute(kt - 1);
      }
      barrier();
      if (kt < nk) {
        if (!grp_b) {
          compute(kt);
        } else {
          if (kt + PD < nk) issue(kt + PD, (kt + PD) % NBUF);
          read_frags(kt);
        }
      }
    }
  } else {
    for (int kt = 0; kt < nk; ++kt) {
      wait_stage(kt);
      barrier();   // ... and everyone's; the buffer of stage kt-1 is free
      if (kt + PD < nk) issue(kt + PD, (kt + PD) % NBUF);
      read_frags(kt);
      compute(kt);
    }
  }
  __syncthreads();   // all waves done with the stage buffers (reused below)

  if (split >= 0) {
    // K-split tail pair: publish this split's FP32 totals; the last split to
    // arrive adds all of them in split order (so the sum does not depend on
    // the arrival order) and runs the epilogue.
    constexpr int NV = 4 * NBJ;   // float4 per thread
    const int pair = lin - g.nfull;  // index among the split pairs
    float4 *wsp = (float4 *)g.ws + ((int64_t)pair * g.nsplit + split) * NV * NTH16;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj) {
        const v4f t = tot[bi][bj];
        wsp[(bi * NBJ + bj) * NTH16 + tid] = make_float4(t[0], t[1], t[2], t[3]);
      }
    __threadfence();
    // The arrival flag lives in the (now idle) stage buffers: a second
    // __shared__ object would make the compiler wait for every LDS-DMA load
    // before each LDS read of the main loop (it cannot tell them apart).
    unsigned *last = (unsigned *)smem;
    __syncthreads();
    if (tid == 0) *last = (atomicAdd(g.cnt + pair, 1u) == (unsigned)g.nsplit - 1);
    __syncthreads();
    if (!*last) return;
    __syncthreads();   // flag read by all before the epilogue reuses smem
    __threadfence();
    const float4 *w0 = (const float4 *)g.ws + (int64_t)pair * g.nsplit * NV * NTH16;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 4
        for (int s = 0; s < g.nsplit; ++s) {
          const float4 v = w0[((int64_t)s * NV + bi * NBJ + bj) * NTH16 + tid];
          a0 += v.x;
          a1 += v.y;
          a2 += v.z;
          a3 += v.w;
        }
        tot[bi][bj] = v4f{(float)a0, (float)a1, (float)a2, (float)a3};
      }
    if (tid == 0) g.cnt[pair] = 0u;   // ready for the next launch
  }

  // ------------------------------------------------------------ epilogue
  // Phase 0: every wave dumps its FP32 results into LDS, V[tile][row][col]
  // with a row pitch of 132 floats.
  float *V = (float *)smem;
  double *rp = (double *)(V + 2 * TILE * EPLD);   // [2 tiles][128] row sums
  double *cpart = rp + 2 * TILE;                  // [2 tiles][WPT waves][128] column sums
  double *tp = cpart + 2 * WPT * TILE;            // [2 tiles][WPT waves] tile sums
  // The FP64 side vectors of the block's rows (rD, s2, dg, d2, d3) and
  // columns (rD) are staged in LDS: read per element from global memory they
  // would each wait for the stores before them (the compiler cannot tell
  // them from the output), one memory round trip per element.
  double *vrow = tp + 2 * WPT;                    // [5][128]
  double *vcol = vrow + 5 * TILE;                 // [256]
  for (int q = tid; q < EVEC; q += NTH16) {
    if (q < 5 * TILE) {
      const int k = q / TILE;
      const int64_t i = arow0 + q % TILE;
      double v = 0.0;
      if (k == 0) v = g.rD[i];
      else if (k == 1) v = g.mode == 1 ? g.s2[i] : 0.0;
      else if (k == 2) v = g.dg[i];
      else if (k == 3) v = g.d2[i];
      else v = g.mode == 1 ? g.d3[i] : 0.0;
      vrow[q] = v;
    } else {
      vcol[q - 5 * TILE] = g.rD[brow0 + q - 5 * TILE];
    }
  }
  if (valid) {
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBJ; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          V[(h * TILE + rh * 64 + bi * 16 + lg * 4 + r) * EPLD + tcol0 + bj * 16 + l16] =
              tot[bi][bj][r];
  }
  __syncthreads();
  // Phase 1: 256 threads per tile, each owning one 8 x 8 block (block row br,
  // block column bc).  Row-contiguous 16-byte loads of D (and X2) and stores
  // of the result; the mirrored store writes the transposed block, again as
  // 16-byte rows.
  const int th = tid >> 8, x = tid & 255;
  const int tjj = cpair * PAIR_COLS + th;
  const bool tvalid = tjj >= ti, dtile = tjj == ti;
  const int br = x >> 4, bc = x & 15;
  const int64_t i0 = arow0 + br * 8;
  const double S = E::PROD_SCALE;
  T *__restrict__ Og = (T *)g.out;
  double a_coef = 0.0, b_coef = 0.0, e_coef = 0.0;
  if (g.mode == 1) update_coefs(g.method, g.coef[0], a_coef, b_coef, e_coef);
  double rsum[8], csum[8], tsum = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r) rsum[r] = csum[r] = 0.0;
  // The 8 x 8 blocks on a tile's diagonal hold the diagonal elements, formed
  // from the FP64 side vectors, and are their own mirrors.  DK = 1 compiles
  // such a block, DK = 0 every other block (the lean path), DK = 2 decides at
  // run time.  Both update modes are compiled separately.
  auto element_block = [&](auto dk_t, auto mode_t) {
    constexpr int DK = decltype(dk_t)::value;
    constexpr int MODE = decltype(mode_t)::value;
    const bool dblk = DK == 1 || (DK == 2 && dtile && br == bc);
    const int64_t j0 = (int64_t)tjj * TILE + bc * 8;
    // Encoded results, row r of the block, 8 halves per plane, kept for the
    // mirrored store.  Planes p < NPARK are parked in this thread's own 8 x 8
    // block of V (32 bytes per row, already consumed when row r is encoded),
    // which keeps them out of the registers; a third plane stays in them.
    constexpr int NPARK = NP < 2 ? NP : 2;
    v4u ob[NP > NPARK ? NP - NPARK : 1][8];
    uint32_t *park = (uint32_t *)(V + (th * TILE + br * 8) * EPLD + bc * 8);   // row r at park + r * EPLD
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int64_t i = i0 + r;
      v4u dv[NP], xv[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        dv[p] = *(const v4u *)(Bg + eoff<P>(i, j0, p, Mp));
        if constexpr (MODE == 1) xv[p] = *(const v4u *)(Ag + eoff<P>(i, j0, p, Mp));
      }
      const float *vr = V + (th * TILE + br * 8 + r) * EPLD + bc * 8;
      uint16_t o[NP][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t j = j0 + e;
        T dp[NP], op[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) dp[p] = (uint16_t)(dv[p][e >> 1] >> (16 * (e & 1)));
        const double v = (double)vr[e] * S;
        double prod, diff;
        if constexpr (MODE == 0) {
          double Dm, x2;
          if (DK != 0 && i == j) {
            Dm = vrow[2 * TILE + br * 8 + r];
            x2 = vrow[3 * TILE + br * 8 + r];
          } else {
            Dm = E::dec(dp);
            x2 = v + Dm * (vrow[br * 8 + r] + vcol[th * TILE + bc * 8 + e]);
          }
          E::enc(x2, op);
          const double x2m = (DK != 0 && i == j) ? x2 : E::dec(op);
          if (DK != 0 && i == j) g.s2[i] = x2 - E::dec(op);
          prod = x2m * Dm;
          diff = x2m - Dm;
        } else {
          double Dm, dn;
          if (DK != 0 && i == j) {
            Dm = vrow[2 * TILE + br * 8 + r];
            dn = a_coef * Dm + b_coef * vrow[3 * TILE + br * 8 + r] + e_coef * vrow[4 * TILE + br * 8 + r];
          } else {
            T xp[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) xp[p] = (uint16_t)(xv[p][e >> 1] >> (16 * (e & 1)));
            Dm = E::dec(dp);
            const double X2m = E::dec(xp);
            const double x3 = v + X2m * vcol[th * TILE + bc * 8 + e] + vrow[TILE + br * 8 + r] * Dm;
            dn = a_coef * Dm + b_coef * X2m + e_coef * x3;
          }
          E::enc(dn, op);
          const double dnm = (DK != 0 && i == j) ? dn : E::dec(op);
          if (DK != 0 && i == j) {
            g.dg_new[i] = dn;
            g.rD_new[i] = dn - E::dec(op);
          }
          prod = dnm * dnm;
          diff = dnm - Dm;
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) o[p][e] = op[p];
        if (dblk && i > j) continue;   // lower half of a diagonal block
        rsum[r] += prod;
        if (DK == 0 || i != j) {
          csum[e] += prod;
          tsum += 2.0 * diff * diff;
        } else {
          tsum += diff * diff;
        }
      }
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        v4u w;
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = (uint32_t)o[p][2 * q] | ((uint32_t)o[p][2 * q + 1] << 16);
        if (p < NPARK)
          *(v4u *)(park + r * EPLD + 4 * p) = w;
        else
          ob[p - NPARK][r] = w;
        if (!dblk) {
          *(v4u *)(Og + eoff<P>(i, j0, p, Mp)) = w;
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (e >= r) Og[eoff<P>(i, j0 + e, p, Mp)] = o[p][e];
        }
      }
    }
    // mirrored (transposed) block: row j0+e gets column e of the block
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      v4u obp[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        if (p < NPARK)
          obp[r] = *(const v4u *)(park + r * EPLD + 4 * p);
        else
          obp[r] = ob[p - NPARK][r];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (!dblk) {
          v4u w;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint32_t lo = (obp[2 * q][e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
            const uint32_t hi = (obp[2 * q + 1][e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
            w[q] = lo | (hi << 16);
          }
          *(v4u *)(Og + eoff<P>(j0 + e, i0, p, Mp)) = w;
        } else {
#pragma unroll
          for (int r = 0; r < 8; ++r)
            if (r < e)
              Og[eoff<P>(j0 + e, i0 + r, p, Mp)] =
                  (uint16_t)((obp[r][e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
        }
      }
    }
  };
  if (tvalid && !(dtile && br > bc)) {   // blocks below the diagonal are mirrors
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    // (three planes: one body for both kinds of block; the split one measured
    // slower there, its main loop scheduled worse)
    if constexpr (NP == 3) {
      if (g.mode == 0) element_block(I2{}, I0{});
      else element_block(I2{}, I1{});
    } else if (dtile && br == bc) {
      if (g.mode == 0) element_block(I1{}, I0{});
      else element_block(I1{}, I1{});
    } else {
      if (g.mode == 0) element_block(I0{}, I0{});
      else element_block(I0{}, I1{});
    }
  }
  // row sums: the 16 threads of a block row (lanes differing in bits 0..3)
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    double v = rsum[r];
    v += shfl_xor_d(v, 1);
    v += shfl_xor_d(v, 2);
    v += shfl_xor_d(v, 4);
    v += shfl_xor_d(v, 8);
    rsum[r] = v;
  }
  // column sums: the 4 block rows of a wave (bits 4..5), then the tile's waves
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    double v = csum[e];
    v += shfl_xor_d(v, 16);
    v += shfl_xor_d(v, 32);
    csum[e] = v;
  }
  tsum += shfl_xor_d(tsum, 1);
  tsum += shfl_xor_d(tsum, 2);
  tsum += shfl_xor_d(tsum, 4);
  tsum += shfl_xor_d(tsum, 8);
  tsum += shfl_xor_d(tsum, 16);
  tsum += shfl_xor_d(tsum, 32);
  const int wt = x >> 6;   // wave within the tile
  if ((x & 15) == 0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) rp[th * TILE + br * 8 + r] = rsum[r];
  }
  if (lg == 0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) cpart[(th * WPT + wt) * TILE + bc * 8 + e] = csum[e];
  }
  if (lane == 0) tp[th * WPT + wt] = tsum;
  __syncthreads();
  if (x < TILE && tvalid) {
    const double rs = rp[th * TILE + x];
    double cs = 0.0;
#pragma unroll
    for (int w = 0; w < WPT; ++w) cs += cpart[(th * WPT + w) * TILE + x];
    if (!dtile) {
      g.part[(int64_t)tjj * Mp + arow0 + x] = rs;
      g.part[(int64_t)ti * Mp + (int64_t)tjj * TILE + x] = cs;
    } else {
      g.part[(int64_t)ti * Mp + arow0 + x] = rs + cs;
    }
  }
  if (tid < 2) {   // 0 for a skipped tile
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < WPT; ++w) t += tp[tid * WPT + w];
    g.tpart[2 * lin + tid] = t;
  }
}

int pair_count(int nt) {
  int n = 0;
  for (int t = 0; t < nt; ++t) n += nt / PAIR_COLS - t / PAIR_COLS;
  return n;
}

int gemm16_blocks(const GemmArgs &g) {
  const int np = pair_count(g.nt);
  return g.nfull + (np - g.nfull) * g.nsplit;
}

// ------------------------------------------------------------------ H stats
// Per row: H_ii and the Gershgorin radius r_i = sum_{j != i} |H_ij|.
__global__ __launch_bounds__(256) void k_hstats(const double *__restrict__ H, int64_t ldh,
                                                int64_t M, double *lo, double *hi,
                                                double *hd) {
  __shared__ double red[256];
  const int64_t i = blockIdx.x;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < M; j += 256)
    if (j != i) s += fabs(H[i * ldh + j]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double d = H[i * ldh + i];
    lo[i] = d - red[0];
    hi[i] = d + red[0];
    hd[i] = d;
  }
}

// Single block: min of lo, max of hi and the (fixed-order) sum of hd.
__global__ __launch_bounds__(256) void k_hfinal(const double *lo, const double *hi,
                                                const double *hd, int64_t M, double *out) {
  __shared__ double smin[256], smax[256], ssum[256];
  double mn = INFINITY, mx = -INFINITY, sm = 0.0;
  for (int64_t i = threadIdx.x; i < M; i += 256) {
    mn = fmin(mn, lo[i]);
    mx = fmax(mx, hi[i]);
    sm += hd[i];
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  ssum[threadIdx.x] = sm;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      ssum[threadIdx.x] += ssum[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smin[0];
    out[1] = smax[0];
    out[2] = ssum[0];
  }
}

// ||(H + H^T)/2 - mu I||_F^2 (the alpha search of the hole-particle guess):
// 64 x 64 tiles, one partial per tile, then a fixed-order sum.
__global__ __launch_bounds__(256) void k_hdev(const double *__restrict__ H, int64_t ldh, int64_t M,
                                              double mu, double *part) {
  __shared__ double hs[64][65], ht[64][65], red[256];
  const int64_t I = (int64_t)blockIdx.y * 64, J = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x, row = tid >> 2, c0 = (tid & 3) * 16;
  for (int c = 0; c < 16; ++c) {
    const int64_t gi = I + row, gj = J + c0 + c;
    hs[row][c0 + c] = (gi < M && gj < M) ? H[gi * ldh + gj] : 0.0;
    const int64_t ti = J + row, tj = I + c0 + c;
    ht[row][c0 + c] = (ti < M && tj < M) ? H[ti * ldh + tj] : 0.0;
  }
  __syncthreads();
  double s = 0.0;
  for (int c = 0; c < 16; ++c) {
    const int64_t i = I + row, j = J + c0 + c;
    if (i < M && j < M) {
      const double x = 0.5 * (hs[row][c0 + c] + ht[c0 + c][row]) - (i == j ? mu : 0.0);
      s += x * x;
    }
  }
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_hdev_sum(const double *part, int n, double *out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += 256) s += part[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------------ initial guess
// D0 = theta I + beta (mu I - (H + H^T)/2) over 64 x 64 tiles of the padded
// matrix; writes the operand planes, the FP64 diagonal (dg, rD) and row sums
// of D0 o D0 into part[tile column][row] (the diagonal of D0^2).  One block
// per mirrored tile pair (I, J), (J, I) with I <= J: each tile of H is read
// once, and (H_ij + H_ji)/2 is the same sum in both output tiles, so D0 is
// exactly symmetric.

// Output tile (I, J) of the pair: hv[q] = H[I + r][J + lane] from the
// block's own load (r = 4q + wave), tr[c][r] = H[J + c][I + r] from LDS.
template <int P>
__device__ __forceinline__ void init_tile(const InitArgs &a, int64_t I, int64_t J,
                                          const double (&hv)[16],
                                          const double (*tr)[65], int wave, int lane) {
  using E = Enc<P>;
  using T = typename E::T;
  constexpr int NP = E::NP;
  T *__restrict__ Og = (T *)a.out;
#pragma unroll 2
  for (int q = 0; q < 16; ++q) {
    const int r = 4 * q + wave;
    const int64_t i = I + r, j = J + lane;
    double x = 0.0;
    if (i < a.M && j < a.M) {
      const double h = 0.5 * (hv[q] + tr[lane][r]);
      x = -a.beta * h;
      if (i == j) x += a.theta + a.beta * a.mu;
    }
    T op[NP];
    E::enc(x, op);
#pragma unroll
    for (int p = 0; p < NP; ++p) Og[eoff<P>(i, j, p, a.Mp)] = op[p];
    const double xm = (i == j) ? x : E::dec(op);
    if (i == j) {
      a.dg[i] = x;
      a.rD[i] = x - E::dec(op);
    }
    // row sum of D0 o D0 over the tile's 64 columns (fixed order)
    double rs = xm * xm;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) rs += __shfl_xor(rs, m, 64);
    if (lane == 0) a.part[(J >> 6) * a.Mp + i] = rs;
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_init(InitArgs a) {
  __shared__ double ta[64][65], tb[64][65];
  // block L -> (u, v), v <= u, of the row-major lower triangle
  const int64_t L = blockIdx.x;
  int64_t u = (int64_t)((sqrt(8.0 * (double)L + 1.0) - 1.0) * 0.5);
  while (u * (u + 1) / 2 > L) --u;
  while ((u + 1) * (u + 2) / 2 <= L) ++u;
  const int64_t v = L - u * (u + 1) / 2;
  const int64_t I = v * 64, J = u * 64;
  const bool diag = u == v;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // ha[q] = H[I+r][J+lane], hb[q] = H[J+r][I+lane]; a wave reads 64
  // consecutive elements (512 bytes) of one row per load
  double ha[16], hb[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = 4 * q + wave;
    const int64_t gi = I + r, gj = J + lane;
    ha[q] = (gi < a.M && gj < a.M) ? a.H[gi * a.ldh + gj] : 0.0;
    const int64_t ti = J + r, tj = I + lane;
    hb[q] = (!diag && ti < a.M && tj < a.M) ? a.H[ti * a.ldh + tj] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = 4 * q + wave;
    ta[r][lane] = ha[q];
    tb[r][lane] = hb[q];
  }
  __syncthreads();
  if (diag) {
    init_tile<P>(a, I, J, ha, ta, wave, lane);
  } else {
    init_tile<P>(a, I, J, ha, tb, wave, lane);
    init_tile<P>(a, J, I, hb, ta, wave, lane);
  }
}

// -------------------------------------------------------------- reductions
// out[i] = sum_s part[s][i]: a block covers 64 rows, wave q of it sums the
// slots s = q (mod 4) in ascending order, and the four wave sums are added in
// wave order.  Per-block sums of out and of extra; the last block to finish
// adds the block sums and the tile partials in a fixed order and runs the
// scalar step for this point of the iteration.
__device__ __forceinline__ double ld_agent(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_reduce(RedArgs a) {
  __shared__ double rq[4][64], s1[256], s2[256], s3[256];
  __shared__ int is_last;
  // a batch enqueued ahead of the host's check: nothing to do once stopped
  // (the status is written by the last block of a mode-1 launch, after
  // every block of that launch has read it here)
  if (a.skip_if_stopped && a.sc->status != 0) return;
  const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  double w = 0.0;
  if (i < a.Mp) {
    // unrolled so that the loads are in flight together; the adds keep
    // their order
#pragma unroll 8
    for (int s = q; s < a.nslots; s += 4) w += a.part[(int64_t)s * a.Mp + i];
  }
  rq[q][lane] = w;
  __syncthreads();
  double v = 0.0, e = 0.0;
  if (q == 0 && i < a.Mp) {
    v = ((rq[0][lane] + rq[1][lane]) + rq[2][lane]) + rq[3][lane];
    a.out[i] = v;
    if (a.extra) e = a.extra[i];
  }
  s1[tid] = v;
  s2[tid] = e;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      s1[tid] += s1[tid + w];
      s2[tid] += s2[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.bpart[2 * blockIdx.x] = s1[0];
    a.bpart[2 * blockIdx.x + 1] = s2[0];
    __threadfence();
    const unsigned ticket = atomicAdd(a.counter, 1u);
    is_last = (ticket == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double b1 = 0.0, b2 = 0.0, b3 = 0.0;
  for (int b = tid; b < (int)gridDim.x; b += 256) {
    b1 += ld_agent(a.bpart + 2 * b);
    b2 += ld_agent(a.bpart + 2 * b + 1);
  }
  if (a.tpart)
    for (int t = tid; t < a.ntiles; t += 256) b3 += a.tpart[t];
  s1[tid] = b1;
  s2[tid] = b2;
  s3[tid] = b3;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      s1[tid] += s1[tid + w];
      s2[tid] += s2[tid + w];
      s3[tid] += s3[tid + w];
    }
    __syncthreads();
  }
  if (tid != 0) return;
  *a.counter = 0u;
  Scalars *sc = a.sc;
  const double sum_out = s1[0], sum_extra = s2[0], sum_tiles = s3[0];
  if (a.mode == 0) {            // after the initial guess
    sc->t2 = sum_out;
    sc->t1 = sum_extra;
  } else if (a.mode == 1) {     // after D^2: decide and form c
    const double t1 = sc->t1, t2 = sc->t2, t3 = sum_out, om = sum_tiles;
    const double ddbar = t1 - t2;
    int status = 0;
    double c = NAN;
    if (!isfinite(t1) || !isfinite(t2) || !isfinite(om)) {
      status = 3;
    } else if (fabs(ddbar) <= a.tol_ddbar || sqrt(om) <= a.tol_idem) {
      status = 1;
    } else if (a.iter >= a.max_iter) {
      status = 2;
    } else {
      if (ddbar > 0.0) c = (t2 - t3) / ddbar;
      // Tr(D Dbar) <= 0 or c outside [0, 1] is a runaway, unless |Tr(D Dbar)|
      // is already within the encoding's rounding floor, where it (and c)
      // is rounding noise and stops decreasing: the iterate is then as
      // idempotent as the encoding allows and the solve stops there.
      const bool bad = !(ddbar > 0.0) || !isfinite(c) || c < 0.0 || c > 1.0;
      const bool stalled = !a.recheck && fabs(ddbar) >= sc->prev_ddbar;
      if ((bad || stalled) && fabs(ddbar) <= a.floor_ddbar) status = 4;
      else if (bad) status = 3;
    }
    if (!a.recheck) sc->prev_ddbar = fabs(ddbar);
    if (status != 0) sc->iter = a.iter;
    sc->t3 = t3;
    sc->omega = om;
    sc->c = c;
    sc->status = status;
    double *h = a.hist + (int64_t)a.iter * 9;
    const double gamma = 1.0 / 3.0 - 2.0 / 3.0 * c;
    h[0] = a.iter; h[1] = t1; h[2] = t2; h[5] = om;
    if (status == 0) {
      h[3] = t3; h[4] = c; h[6] = gamma;
      h[7] = om - gamma * (3.0 * t2 - 2.0 * t3 - a.N);
    } else {
      h[3] = h[4] = h[6] = h[7] = NAN;
    }
    h[8] = NAN;
  } else {                      // after the update: traces of D_{n+1}
    sc->t2 = sum_out;
    sc->t1 = sum_extra;
    sc->step = sum_tiles;
    a.hist[(int64_t)a.iter * 9 + 8] = sqrt(sum_tiles);
    if (!a.early_stop) return;
    // The stops of the mode-1 decision that need only T1 and T2 of D_{n+1},
    // taken here so that the square of the last iterate is never formed:
    // |Tr(D Dbar)| within tol_ddbar, or within the rounding floor while not
    // decreasing or not positive (below max_iter, where mode 1 would report
    // max_iter first).  Everything else (non-finite traces, c outside
    // [0, 1], max_iter) is left to mode 1, which would take the same
    // decision on the same traces.
    const double t1 = sum_extra, t2 = sum_out, ddbar = t1 - t2;
    const int nx = a.iter + 1;
    int status = 0;
    if (isfinite(t1) && isfinite(t2)) {
      if (fabs(ddbar) <= a.tol_ddbar) status = 1;
      else if (nx < a.max_iter && (!(ddbar > 0.0) || fabs(ddbar) >= sc->prev_ddbar) &&
               fabs(ddbar) <= a.floor_ddbar)
        status = 4;
    }
    if (status == 0) return;
    sc->status = status;
    sc->iter = nx;
    sc->on_traces = 1;
    sc->omega = NAN;
    double *h = a.hist + (int64_t)nx * 9;
    h[0] = nx; h[1] = t1; h[2] = t2;
    h[3] = h[4] = h[5] = h[6] = h[7] = h[8] = NAN;
  }
}

// ------------------------------------------------------------------ output
template <int P>
__global__ __launch_bounds__(256) void k_output(OutArgs a) {
  using E = Enc<P>;
  using T = typename E::T;
  constexpr int NP = E::NP;
  // rows on the x dimension of the grid (no 64K limit), 256 columns per block on y
  const int64_t i = blockIdx.x;
  const int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (i >= a.M || j >= a.M) return;
  double x;
  if (i == j) {
    x = a.dg[i];
  } else {
    T p[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) p[q] = ((const T *)a.planes)[eoff<P>(i, j, q, a.Mp)];
    x = E::dec(p);
  }
  if (a.hole) x = (i == j ? 1.0 : 0.0) - x;
  if (a.dtype == GCP_DTYPE_F64)
    ((double *)a.D)[i * a.ldd + j] = x;
  else
    ((float *)a.D)[i * a.ldd + j] = (float)x;
}

// -------------------------------------------------- encoding conversion
// Re-encodes an iterate from encoding PA to PB (precision schedule): the
// off-diagonal master values dec_A(planes) are encoded in B; the diagonal
// is the exact FP64 vector diag, encoded in B with its residual
// diag - dec_B(enc_B(diag)) written to resid.
template <int P>
__device__ __forceinline__ double dec_at(const void *b, int64_t i, int64_t j, int64_t Mp) {
  using E = Enc<P>;
  typename E::T p[E::NP];
#pragma unroll
  for (int q = 0; q < E::NP; ++q) p[q] = ((const typename E::T *)b)[eoff<P>(i, j, q, Mp)];
  return E::dec(p);
}
template <int P>
__device__ __forceinline__ double enc_at(void *b, int64_t i, int64_t j, int64_t Mp, double x) {
  using E = Enc<P>;
  typename E::T p[E::NP];
  E::enc(x, p);
#pragma unroll
  for (int q = 0; q < E::NP; ++q) ((typename E::T *)b)[eoff<P>(i, j, q, Mp)] = p[q];
  return E::dec(p);
}

__device__ __forceinline__ double enc_any(int pb, void *out, int64_t i, int64_t j, int64_t Mp,
                                            double x) {
  switch (pb) {
    case GCP_FP64: return enc_at<GCP_FP64>(out, i, j, Mp, x);
    case GCP_FP32: return enc_at<GCP_FP32>(out, i, j, Mp, x);
    case GCP_BF16: return enc_at<GCP_BF16>(out, i, j, Mp, x);
    case GCP_FP16: return enc_at<GCP_FP16>(out, i, j, Mp, x);
    case GCP_BF16X3: return enc_at<GCP_BF16X3>(out, i, j, Mp, x);
    case GCP_FP16X3: return enc_at<GCP_FP16X3>(out, i, j, Mp, x);
    default: return enc_at<GCP_BF16X6>(out, i, j, Mp, x);
  }
}

template <int PA>
__global__ __launch_bounds__(256) void k_convert(int pb, const void *in, const double *diag, void *out,
                                                 double *resid, int64_t Mp) {
  // rows on the x dimension of the grid (no 64K limit), 256 columns per block on y
  const int64_t i = blockIdx.x;
  const int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x;
  const double x = (i == j) ? diag[i] : dec_at<PA>(in, i, j, Mp);
  const double xe = enc_any(pb, out, i, j, Mp, x);
  if (i == j) resid[i] = x - xe;
}

hipError_t launch_convert(int pa, int pb, const void *in, const double *diag, void *out,
                          double *resid, int64_t Mp, hipStream_t st) {
  const dim3 grid((unsigned)Mp, (unsigned)(Mp / 256));
  switch (pa) {
    case GCP_FP64: k_convert<GCP_FP64><<<grid, 256, 0, st>>>(pb, in, diag, out, resid, Mp); break;
    case GCP_FP32: k_convert<GCP_FP32><<<grid, 256, 0, st>>>(pb, in, diag, out, resid, Mp); break;
    case GCP_BF16: k_convert<GCP_BF16><<<grid, 256, 0, st>>>(pb, in, diag, out, resid, Mp); break;
    case GCP_FP16: k_convert<GCP_FP16><<<grid, 256, 0, st>>>(pb, in, diag, out, resid, Mp); break;
    case GCP_BF16X3: k_convert<GCP_BF16X3><<<grid, 256, 0, st>>>(pb, in, diag, out, resid, Mp); break;
    case GCP_FP16X3: k_convert<GCP_FP16X3><<<grid, 256, 0, st>>>(pb, in, diag, out, resid, Mp); break;
    case GCP_BF16X6: k_convert<GCP_BF16X6><<<grid, 256, 0, st>>>(pb, in, diag, out, resid, Mp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- dispatch
template <int P>
static hipError_t launch_gemm_p(const GemmArgs &g, int ntiles, hipStream_t st) {
  if constexpr (Enc<P>::KIND >= 2)
    k_gemm16<P><<<gemm16_blocks(g), NTH16, 0, st>>>(g);
  else
    k_gemm<P><<<g.nfull + (ntiles - g.nfull) * g.nsplit, NTH, 0, st>>>(g);
  return hipGetLastError();
}

hipError_t launch_gemm(int prec, const GemmArgs &g, hipStream_t st) {
  const int ntiles = g.nt * (g.nt + 1) / 2;
  switch (prec) {
    case GCP_FP64: return launch_gemm_p<GCP_FP64>(g, ntiles, st);
    case GCP_FP32: return launch_gemm_p<GCP_FP32>(g, ntiles, st);
    case GCP_BF16: return launch_gemm_p<GCP_BF16>(g, ntiles, st);
    case GCP_FP16: return launch_gemm_p<GCP_FP16>(g, ntiles, st);
    case GCP_BF16X3: return launch_gemm_p<GCP_BF16X3>(g, ntiles, st);
    case GCP_FP16X3: return launch_gemm_p<GCP_FP16X3>(g, ntiles, st);
    case GCP_BF16X6: return launch_gemm_p<GCP_BF16X6>(g, ntiles, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_init(int prec, const InitArgs &a, hipStream_t st) {
  const int64_t nt = a.Mp / 64;
  const dim3 grid((unsigned)(nt * (nt + 1) / 2));
  switch (prec) {
    case GCP_FP64: k_init<GCP_FP64><<<grid, 256, 0, st>>>(a); break;
    case GCP_FP32: k_init<GCP_FP32><<<grid, 256, 0, st>>>(a); break;
    case GCP_BF16: k_init<GCP_BF16><<<grid, 256, 0, st>>>(a); break;
    case GCP_FP16: k_init<GCP_FP16><<<grid, 256, 0, st>>>(a); break;
    case GCP_BF16X3: k_init<GCP_BF16X3><<<grid, 256, 0, st>>>(a); break;
    case GCP_FP16X3: k_init<GCP_FP16X3><<<grid, 256, 0, st>>>(a); break;
    case GCP_BF16X6: k_init<GCP_BF16X6><<<grid, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_output(int prec, const OutArgs &a, hipStream_t st) {
  const dim3 grid((unsigned)a.M, (unsigned)((a.M + 255) / 256));
  switch (prec) {
    case GCP_FP64: k_output<GCP_FP64><<<grid, 256, 0, st>>>(a); break;
    case GCP_FP32: k_output<GCP_FP32><<<grid, 256, 0, st>>>(a); break;
    case GCP_BF16: k_output<GCP_BF16><<<grid, 256, 0, st>>>(a); break;
    case GCP_FP16: k_output<GCP_FP16><<<grid, 256, 0, st>>>(a); break;
    case GCP_BF16X3: k_output<GCP_BF16X3><<<grid, 256, 0, st>>>(a); break;
    case GCP_FP16X3: k_output<GCP_FP16X3><<<grid, 256, 0, st>>>(a); break;
    case GCP_BF16X6: k_output<GCP_BF16X6><<<grid, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_hstats(const double *H, int64_t ldh, int64_t M, double *lo, double *hi,
                         double *hd, double *out, hipStream_t st) {
  k_hstats<<<(unsigned)M, 256, 0, st>>>(H, ldh, M, lo, hi, hd);
  k_hfinal<<<1, 256, 0, st>>>(lo, hi, hd, M, out);
  return hipGetLastError();
}

hipError_t launch_hdev(const double *H, int64_t ldh, int64_t M, int64_t Mp, double mu,
                       double *scratch, double *out, hipStream_t st) {
  const unsigned nb = (unsigned)(Mp / 64);
  k_hdev<<<dim3(nb, nb), 256, 0, st>>>(H, ldh, M, mu, scratch);
  k_hdev_sum<<<1, 256, 0, st>>>(scratch, (int)(nb * nb), out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero(uint32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0u;
}

hipError_t launch_zero(void *p, int64_t nwords, hipStream_t st) {
  if (!p || nwords <= 0) return hipSuccess;
  int64_t nb = (nwords + 255) / 256;
  if (nb > 1024) nb = 1024;
  k_zero<<<(unsigned)nb, 256, 0, st>>>((uint32_t *)p, nwords);
  return hipGetLastError();
}

// Traffic yardstick: 64 KiB per block, each wave loading 16 KiB as sixteen
// contiguous wave instructions of 1 KiB (16 bytes per lane) straight into
// LDS, the load type of the 16-bit product kernel's panels.
__global__ __launch_bounds__(256) void k_stream_lds(const uint16_t *buf) {
  __shared__ __attribute__((aligned(16))) uint16_t lds[32768];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint16_t *src = buf + (int64_t)blockIdx.x * 32768 + wave * 8192 + lane * 8;
#pragma unroll
  for (int q = 0; q < 16; ++q)
    __builtin_amdgcn_global_load_lds((const void *)(src + q * 512),
                                     (lds_void *)(lds + wave * 8192 + q * 512), 16, 0, 0);
  __builtin_amdgcn_s_waitcnt(0);
}

hipError_t launch_stream_lds(const void *buf, int64_t bytes, hipStream_t st) {
  k_stream_lds<<<(unsigned)(bytes / 65536), 256, 0, st>>>((const uint16_t *)buf);
  return hipGetLastError();
}

hipError_t launch_reduce(const RedArgs &a, hipStream_t st) {
  k_reduce<<<(unsigned)((a.Mp + 63) / 64), 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace gcp
