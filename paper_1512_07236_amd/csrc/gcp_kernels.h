// gcp_kernels.h -- argument blocks and launchers shared by the host library
// and the device kernels (internal; the public interface is include/gcp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcp {

// Default fold period of the FP32 tile product, in K stages of 32 values:
// with 8 accumulating MFMA steps per stage and n stages, a chunk accumulator
// added into a running total every f stages rounds each term about 8f + n/f
// times; f = sqrt(n / 8) minimises that (one accumulator: 8n).
__host__ __device__ inline int fp32_fold(int64_t Mp) {
  const double f = sqrt((double)(Mp / 32) / 8.0);
  const int r = (int)(f + 0.5);
  return r < 1 ? 1 : r;
}

// D' = a D + b D^2 + e D^3 for the recursion `method` at coefficient c:
// HPCP, eq. (hpcp3) with Dbar = I - D: a = 1 - 2c, b = 2 + 2c, e = -2;
// PMCP, eq. (pm1a) for c <= 1/2: (1 - 2c, 1 + c, -1) / (1 - c),
//       eq. (pm1b) for c > 1/2:  (0, 1 + c, -1) / c.
// Every choice keeps a Tr D + b Tr D^2 + e Tr D^3 = Tr D for this c.
__host__ __device__ inline void update_coefs(int method, double c, double &a, double &b,
                                             double &e) {
  if (method == 0) {
    a = 1.0 - 2.0 * c;
    b = 2.0 + 2.0 * c;
    e = -2.0;
  } else if (c <= 0.5) {
    const double r = 1.0 / (1.0 - c);
    a = (1.0 - 2.0 * c) * r;
    b = (1.0 + c) * r;
    e = -r;
  } else {
    const double r = 1.0 / c;
    a = 0.0;
    b = (1.0 + c) * r;
    e = -r;
  }
}

// Derivatives of (a, b, e) above with respect to c (the adjoint's
// dD'/dc = a' D + b' D^2 + e' D^3).
__host__ __device__ inline void update_coef_derivs(int method, double c, double &da, double &db,
                                                   double &de) {
  if (method == 0) {
    da = -2.0;
    db = 2.0;
    de = 0.0;
  } else if (c <= 0.5) {
    const double r = 1.0 / (1.0 - c);
    da = -r * r;
    db = 2.0 * r * r;
    de = -r * r;
  } else {
    const double r = 1.0 / c;
    da = 0.0;
    db = -r * r;
    de = r * r;
  }
}

// Device-resident scalars of one solve (FP64 traces and the decision).
struct Scalars {
  double t1, t2, t3, omega, c, step;
  int32_t status;   // 0 continue, 1 converged, 2 max_iter reached, 3 breakdown,
                    // 4 stopped at the rounding floor
  int32_t iter;     // update at which status became non-zero
  double hstat[4];  // Gershgorin min, max, Tr H
  double prev_ddbar;   // |Tr(D Dbar)| of the previous iterate (+inf before the first)
  int32_t on_traces;   // 1: the stop was decided from the update's traces, before
                       // the square of the last iterate was formed
  int32_t pad;
};

struct GemmArgs {
  const void *A;       // left operand planes (rows of D or X2)
  const void *B;       // right operand planes (rows of D)
  void *out;           // output planes (X2 in mode 0, D_{n+1} in mode 1)
  int64_t Mp;          // padded size (multiple of 128)
  int64_t pstride;     // elements between planes
  int nt;              // Mp / 128
  int mode;            // 0: X2 = D D, 1: D_{n+1} = (1-2c) D + (2+2c) X2 - 2 X2 D
  int fold;            // fold period of the main accumulator, in K stages
  // Blocks [0, nfull) compute whole units (tile pairs in the 16-bit kernel,
  // tiles in the FP64 / FP32 one); the remaining units are each split over
  // nsplit blocks along K (nsplit = 1: no split), whose partial tiles (FP32,
  // or the accumulator type) meet in ws and are added in FP64, in split
  // order, by the last of them to finish (per-unit arrival counters in cnt,
  // self-resetting)
  int nfull;
  int nsplit;
  int method;          // 0 HPCP, 1 PMCP (update coefficients of mode 1)
  void *ws;
  unsigned *cnt;
  const double *dg;    // diag(D) FP64
  const double *rD;    // diag(D) - dec(enc(diag(D)))
  const double *d2;    // diag(X2) FP64
  double *s2;          // diag(X2) - dec(enc(diag(X2)))   (written in mode 0)
  const double *d3;    // diag(X2 D) FP64                 (mode 1)
  double *dg_new;      // diag(D_{n+1})                   (mode 1)
  double *rD_new;      // its residual                    (mode 1)
  double *part;        // row sums [nt][Mp]
  double *tpart;       // tile sums [ntiles]
  const double *coef;  // coef[0] = c_n (mode 1)
  // non-NULL: the launch does nothing once *status is non-zero (the solve
  // has stopped; later launches of a batch enqueued ahead are void)
  const int32_t *status;
};

struct InitArgs {
  const double *H;
  int64_t ldh, M, Mp, pstride;
  double theta, beta, mu;
  void *out;
  double *dg, *rD, *part;
};

struct RedArgs {
  const double *part;
  int nslots;
  int mode;            // 0 after init, 1 after D^2, 2 after the update
  int64_t Mp;
  double *out;
  const double *extra;
  double *bpart;
  unsigned *counter;
  const double *tpart;
  int ntiles;
  int iter, max_iter;
  int early_stop;      // mode 2: decide the stops that need only T1 and T2 of D_{n+1}
  double tol_ddbar, tol_idem, N;
  double floor_ddbar;  // rounding floor of |Tr(D Dbar)| of the encoding
  int skip_if_stopped; // 1: do nothing once sc->status is non-zero
  int recheck;         // mode 1: the same iterate again (after a change of encoding):
                       // no stall test against, and no update of, prev_ddbar
  Scalars *sc;
  double *hist;
};

struct OutArgs {
  const void *planes;
  const double *dg;
  int64_t M, Mp, pstride, ldd;
  void *D;
  int dtype;
  int hole;            // write I - X instead of X
};

// Adjoint of one update (gcp_backward.hip).  All matrices are Mp x Mp
// row-major in the adjoint's storage type (FP64 or FP32).
struct BwdArgs {
  const void *D;       // D_n
  const void *X2;      // D_n^2                     (modes 1, 2)
  const void *G;       // Gbar_{n+1} = dL/dD_{n+1}
  const void *AT;      // D_n Gbar_{n+1}            (mode 2)
  const void *CT;      // D_n^2 Gbar_{n+1}          (mode 2)
  void *out0;          // mode 0: X2; mode 1: AT; mode 2: Gbar_n
  void *out1;          // mode 1: CT
  int64_t Mp;
  int nt;
  int mode;            // 0: X2 = D D; 1: AT = D G and CT = X2 G; 2: E = D G D + combine
  int need_x3;         // mode 1: also the per-tile sums of X2 o AT (<G, D^3>; e' != 0)
  double a, b, e;      // D_{n+1} = a D + b D^2 + e D^3 at c_n (update_coefs)
  double c, inv_t12;   // c_n, 1 / (T1 - T2)_n
  const double *kappa; // device scalar (mode 2)
  double *tpart;       // per-tile sums: [0, ntri) w_ij G_ij X2_ij and [ntri, 2 ntri)
                       // w_ij G_ij D_ij over upper tiles (mode 0), [2 ntri, 2 ntri + nt^2)
                       // X2 o AT over all tiles (mode 1, need_x3)
};

struct BwdInitArgs {
  const void *G0;      // Gbar_0 (Mp x Mp)
  const void *D0;      // D_0 (Mp x Mp)
  int64_t M, Mp, ldh;
  double beta, dbeta, theta;
  double hdev;         // alpha-searched guess: ||mu I - H||_F^2 (0: alpha fixed)
  double sign;         // -1 for the hole recursion (dL/dDbar = -dL/dD)
  double *rows;        // 2 Mp scratch: row sums of G0 o D0, diag of G0
  double *sums;        // 2 scalars
  void *dH;            // output, M x M with leading dimension ldh
  int dtype;
};

// FP64 verification of a density matrix (gcp_verify.hip).  D and H are the
// symmetric parts of the caller's matrices, Mp x Mp, zero padded.
struct VerifyArgs {
  const double *D, *H;
  double *HD;          // Mp x Mp
  double *tpart;       // upper-tile partials of ||D^2 - D||_F^2
  double *rows;        // 4 Mp row partials
  double *out;         // 5 sums: commutator^2, Tr(DH), ||D||_F^2, Tr D, ||D^2-D||_F^2
  int64_t Mp;
  int nt, ntri;
};
hipError_t launch_verify(const VerifyArgs &a, hipStream_t st);

hipError_t launch_bwd_store(int fprec, int bprec, const void *planes, const double *dg,
                            int64_t Mp, void *out, hipStream_t st);
hipError_t launch_bwd_load(int bprec, const void *g, int64_t ldg, int dtype, int64_t M,
                           int64_t Mp, void *G, hipStream_t st);
hipError_t launch_bwd_gemm(int bprec, const BwdArgs &a, hipStream_t st);
hipError_t launch_bwd_kappa(const double *tpart, int ntri, int nfull, double da, double db,
                            double de, double *kappa, hipStream_t st);
hipError_t launch_bwd_init(int bprec, const BwdInitArgs &a, hipStream_t st);

hipError_t launch_gemm(int prec, const GemmArgs &g, hipStream_t st);
// Blocks of the 16-bit product kernel (pairs of 128 x 128 tiles) for nt tiles per side.
int pair_count(int nt);
// Grid of the 16-bit product kernel: whole pairs plus the K-split tail blocks.
int gemm16_blocks(const GemmArgs &g);
hipError_t launch_init(int prec, const InitArgs &a, hipStream_t st);
hipError_t launch_output(int prec, const OutArgs &a, hipStream_t st);
// Re-encode an Mp x Mp iterate from encoding pa to pb (exact FP64 diagonal
// from diag; the new diagonal residuals go to resid).
hipError_t launch_convert(int pa, int pb, const void *in, const double *diag, void *out,
                          double *resid, int64_t Mp, hipStream_t st);
hipError_t launch_reduce(const RedArgs &a, hipStream_t st);
// Streams `bytes` (a multiple of 64 KiB) of buf into LDS with global_load_lds.
hipError_t launch_stream_lds(const void *buf, int64_t bytes, hipStream_t st);
// n 32-bit words of p set to zero by a kernel (no memset node in a captured graph)
hipError_t launch_zero(void *p, int64_t nwords, hipStream_t st);
hipError_t launch_hstats(const double *H, int64_t ldh, int64_t M, double *lo, double *hi,
                         double *hd, double *out, hipStream_t st);
// out[0] = || (H + H^T)/2 - mu I ||_F^2 over M x M (fixed order); scratch holds
// (Mp/64)^2 block partials.
hipError_t launch_hdev(const double *H, int64_t ldh, int64_t M, int64_t Mp, double mu,
                       double *scratch, double *out, hipStream_t st);

}  // namespace gcp
