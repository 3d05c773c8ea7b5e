// gcp_api.hip -- host side of libgcp: the C ABI declared in include/gcp.h.
//
// Owns the device workspace of one solve and drives the iteration: per
// update two MFMA products (gcp_kernels.hip) and two fixed-order reductions;
// the host reads five FP64 scalars after each D^2 to decide whether to stop
// (the paper's test on Tr(D Dbar) is made before c_n is formed).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gcp.h"
#include "gcp_kernels.h"

using namespace gcp;

namespace {

// Text of the last error, in a fixed buffer: no path of the library that
// runs a solve allocates host memory for its messages.
struct ErrText {
  char buf[320] = {0};
  ErrText &operator=(const char *m) {
    std::snprintf(buf, sizeof(buf), "%s", m);
    return *this;
  }
  void set(const char *a, const char *b) { std::snprintf(buf, sizeof(buf), "%s: %s", a, b); }
  const char *c_str() const { return buf; }
};

thread_local ErrText g_create_error;

int plane_count(int prec) {
  switch (prec) {
    case GCP_BF16X3:
    case GCP_FP16X3: return 2;
    case GCP_BF16X6: return 3;
    default: return 1;
  }
}
int elem_size(int prec) {
  switch (prec) {
    case GCP_FP64: return 8;
    case GCP_FP32: return 4;
    default: return 2;
  }
}
int products(int prec) {
  switch (prec) {
    case GCP_BF16X3:
    case GCP_FP16X3: return 3;
    case GCP_BF16X6: return 6;
    default: return 1;
  }
}

}  // namespace

struct gcp_ctx {
  // a solve of gcp_purify_static: workspace carved from the static array,
  // D_0 built in place in Dp[0], no host-side history kept
  bool one_shot = false;
  int64_t M = 0, Mp = 0;
  int nt = 0, ntiles = 0, ntpart = 0, nred = 0;
  gcp_options opt{};
  hipStream_t stream = nullptr;
  int device = 0;
  // operand planes: D (double-buffered) and X2
  void *Dp[2] = {nullptr, nullptr};
  void *X2p = nullptr;
  int cur = 0;
  // FP64 vectors (length Mp)
  double *dg[2] = {nullptr, nullptr}, *rD[2] = {nullptr, nullptr};
  double *d2[2] = {nullptr, nullptr};
  double *s2 = nullptr, *d3 = nullptr;
  double *part = nullptr, *tpart = nullptr, *bpart = nullptr;
  double *hvec = nullptr;   // 3 Mp scratch for H statistics
  // launch configuration per encoding, one per phase of the schedule
  struct PrecCfg {
    int prec = GCP_FP64;
    int ntpart = 0;   // tile partial sums the reduction adds
    int fold = 1;     // fold period of the product's accumulator (K stages)
    int nfull = 0;    // product units (tile pairs, or tiles for FP64 / FP32) computed whole ...
    int ntail = 0;    // ... and units split along K (0: none) ...
    int nsplit = 1;   // ... over this many blocks each
    double floor_ddbar = 0.0;   // rounding floor of |Tr(D Dbar)| (set by gcp_init)
    double enter_ddbar = 0.0;   // schedule: this encoding from |Tr(D Dbar)| <= enter_ddbar
  } pc[3];                      // the phases of the precision schedule, in order
  int nprec = 1;
  void *Xc = nullptr;       // conversion target of a precision switch
  void *split_ws = nullptr;   // partial tiles of the K-split units
  unsigned *split_cnt = nullptr;   // their arrival counters
  unsigned *counter = nullptr;
  Scalars *sc = nullptr;    // device
  Scalars *sc_host = nullptr;  // pinned
  double *hist = nullptr;   // device, (max_iter + 1) x 9
  std::vector<double> hist_host;
  int hist_rows = 0;
  // init state
  bool inited = false;
  int64_t N = 0;
  double mu = NAN, beta = NAN, emin = NAN, emax = NAN, alpha = 1.0;
  double beta_min = 0.0, beta_max = 0.0;
  bool alpha_searched = false;   // alpha from the search's target (depends on H)
  double hdev = 0.0;             // ||mu I - H||_F^2 when alpha_searched
  double t1_0 = NAN, t2_0 = NAN;
  void *D0p = nullptr;      // copy of the D_0 planes so purify can be re-run
  double *dg0 = nullptr, *rD0 = nullptr, *d20 = nullptr;
  // reverse mode: stored iterates D_0 .. D_{p-1} (adjoint type, Mp x Mp each),
  // or with checkpoint_every = k >= 2 the forward state at every k-th step
  // (operand planes + dg, rD, d2) and k recomputed iterates at a time
  std::vector<void *> slots;
  struct Ckpt {
    void *planes = nullptr;
    double *vec = nullptr;   // dg, rD, d2 (3 Mp)
    int pi = 0;              // encoding index (precision schedule)
  };
  std::vector<Ckpt> ckpts;
  int n_switch[3] = {-1, -1, -1};   // update at which the schedule entered phase k
  int bwd_p = -1;           // updates covered by the stored iterates (-1: none)
  void *bG[2] = {nullptr, nullptr};
  void *bX2 = nullptr, *bAT = nullptr, *bCT = nullptr;
  double *btpart = nullptr; // per-tile partial sums of kappa (2 ntri + nt^2)
  double *bvec = nullptr;   // 2 Mp row scratch + kappa + 2 sums
  // verification workspace (allocated by the first gcp_verify)
  double *vD = nullptr, *vH = nullptr, *vHD = nullptr, *vaux = nullptr;
  // profiling
  std::vector<hipEvent_t> events;
  ErrText err;
};

#define HIPCHK(ctx, expr)                                                          \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      (ctx)->err.set(#expr, hipGetErrorString(e_));                                \
      return GCP_ERR_HIP;                                                          \
    }                                                                              \
  } while (0)

static size_t plane_bytes_of(const gcp_ctx *c, int prec) {
  return (size_t)plane_count(prec) * (size_t)c->Mp * (size_t)c->Mp * (size_t)elem_size(prec);
}
// Operand buffers hold any encoding the context's schedule uses.
static size_t plane_bytes(const gcp_ctx *c) {
  size_t b = 0;
  for (int k = 0; k < c->nprec; ++k) {
    const size_t x = plane_bytes_of(c, c->pc[k].prec);
    if (x > b) b = x;
  }
  return b;
}

static void free_all(gcp_ctx *c) {
  void *ptrs[] = {c->Dp[0], c->Dp[1], c->X2p, c->dg[0], c->dg[1], c->rD[0], c->rD[1],
                  c->d2[0], c->d2[1], c->s2, c->d3, c->part, c->tpart, c->bpart, c->hvec,
                  c->counter, c->sc, c->hist, c->D0p, c->dg0, c->rD0, c->d20};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  void *bptrs[] = {c->bG[0], c->bG[1], c->bX2, c->bAT, c->bCT, c->btpart, c->bvec, c->split_ws,
                   c->split_cnt, c->vD, c->vH, c->vHD, c->vaux, c->Xc};
  for (void *p : bptrs)
    if (p) (void)hipFree(p);
  for (void *p : c->slots)
    if (p) (void)hipFree(p);
  c->slots.clear();
  for (auto &k : c->ckpts) {
    if (k.planes) (void)hipFree(k.planes);
    if (k.vec) (void)hipFree(k.vec);
  }
  c->ckpts.clear();
  if (c->sc_host) (void)hipHostFree(c->sc_host);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  c->events.clear();
}

// Launch configuration of encoding pc[k].prec: tile partial count, fold
// period and the K-split units of the product kernel.
static void PrecCfgInit(gcp_ctx *c, int k) {
  gcp_ctx::PrecCfg &q = c->pc[k];
  const int prec = q.prec;
  const int np = plane_count(prec);
  q.ntpart = elem_size(prec) == 2 ? 2 * pair_count(c->nt) : c->ntiles;
  // fold period of the 16-bit kernel, in K stages: sqrt(stages / products
  // per stage) unless given.  One- and two-plane encodings stage 64 halves
  // per row (64 K values of one plane, or 32 of both); three planes 32 K.
  const int nk = np <= 2 ? (int)(c->Mp * np / 64) : (int)(c->Mp / 32);
  const double per_stage = np == 1 ? 2.0 : (double)products(prec);
  // every pair split along K over `ks` blocks (the ksplit option), each
  // folding its own nk / ks stages
  const int ks = elem_size(prec) == 2 && c->opt.ksplit >= 2 ? std::min(c->opt.ksplit, nk) : 1;
  int f = c->opt.fold_every;
  if (f <= 0)
    f = prec == GCP_FP32 ? fp32_fold(c->Mp)
                         : (int)std::lround(std::sqrt((double)nk / ks / per_stage));
  q.fold = f < 1 ? 1 : f;
  q.nsplit = 1;
  q.ntail = 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (elem_size(prec) != 2) {
    // FP64 / FP32: tiles are equal units of work, two resident blocks per
    // CU.  The tiles of a last partial round (all tiles when there are fewer
    // than one round) would leave most slots idle, so each is split along K
    // over up to 8 blocks of at least 64 (FP64) or 256 (FP32) K values.  At
    // most 128 split blocks in all for M <= GCP_STATIC_MAX_M (16 MB of
    // partial tiles, within the static workspace of gcp_purify_static), 512
    // above.  Measured per product (FP64 / FP32): M = 1024 0.19 -> 0.13 /
    // 0.11 -> 0.09 ms, M = 4096 1.69 -> 1.40 / 0.91 -> 0.70 ms, M = 8192
    // 9.54 -> 9.53 / 5.03 -> 4.57 ms.
    const int slots = 2 * cus;
    const int nkt = (int)(c->Mp / (128 / elem_size(prec)));
    const int tail = c->ntiles % slots;
    const int cap = c->M <= GCP_STATIC_MAX_M ? 128 : 512;
    int S = tail > 0 ? slots / tail : 1;
    S = std::min(S, 8);
    S = std::min(S, nkt / (prec == GCP_FP32 ? 8 : 4));
    if (tail > 0 && tail * S > cap) S = cap / tail;
    q.nfull = c->ntiles;
    if (tail > 0 && S >= 2) {
      q.nfull = c->ntiles - tail;
      q.ntail = tail;
      q.nsplit = S;
    }
    return;
  }
  const int npairs = pair_count(c->nt);
  q.nfull = npairs;
  if (ks >= 2) {
    q.nfull = 0;
    q.ntail = npairs;
    q.nsplit = ks;
    return;
  }
  // Pairs are equal units of work, one resident block per CU: the last
  // partial round of np % CUs pairs would leave most CUs idle, so each of
  // those pairs is split along K over up to min(CUs / tail, 4) blocks (at
  // least 8 K stages each) and finished by the last of its splits.  At
  // M = 8192 (32 tail pairs) 2, 4 and 8 splits measured 1.63, 1.63 and
  // 1.62 ms per product (FP16X3), 3.16, 3.01 and 3.02 ms (BF16X6); each
  // split re-pays the pipeline fill and writes a 128 KB partial.
  const int tail = npairs % cus;
  int S = tail > 0 ? cus / tail : 1;
  if (S > nk / 8) S = nk / 8;
  if (S > 4) S = 4;
  if (tail > 0 && S >= 2) {
    q.nfull = npairs - tail;
    q.ntail = tail;
    q.nsplit = S;
  }
}

extern "C" int gcp_options_default(gcp_options *opt) {
  if (!opt) return GCP_ERR_INVALID_ARG;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = GCP_FP64;
  opt->max_iter = 100;
  opt->tol_ddbar = 1e-6;
  opt->tol_idem = 0.0;
  opt->fold_every = 0;
  opt->profile = 0;
  opt->keep_iterates = 0;
  opt->bwd_precision = GCP_FP64;
  opt->late_precision = -1;
  opt->switch_ddbar = 0.0;
  opt->final_precision = -1;
  opt->final_ddbar = 0.0;
  opt->method = GCP_METHOD_HPCP;
  opt->init_mode = GCP_INIT_PMCP;
  opt->alpha = 0.5;
  opt->delta = 2.0 / 3.0;
  opt->hole = 0;
  opt->checkpoint_every = 0;
  opt->sync_every = 4;
  opt->floor_ddbar = NAN;
  return GCP_OK;
}

// Checks the options and the size; the message goes to err.
static int check_options(const gcp_options &o, int64_t M, ErrText &err) {
  if (M <= 0 || M > (int64_t)1 << 20) {
    err = "gcp_create: M must be in [1, 2^20]";
    return GCP_ERR_INVALID_ARG;
  }
  if (o.precision < GCP_FP64 || o.precision > GCP_BF16X6) {
    err = "gcp_create: unknown precision";
    return GCP_ERR_INVALID_ARG;
  }
  if (o.max_iter < 0 || o.max_iter > 100000 || !(o.tol_ddbar >= 0.0) || !(o.tol_idem >= 0.0) ||
      o.fold_every < 0) {
    err = "gcp_create: max_iter, tolerances and fold_every must be non-negative";
    return GCP_ERR_INVALID_ARG;
  }
  if ((o.keep_iterates != 0 && o.keep_iterates != 1) ||
      (o.bwd_precision != GCP_FP64 && o.bwd_precision != GCP_FP32)) {
    err = "gcp_create: keep_iterates must be 0 or 1 and bwd_precision FP64 or FP32";
    return GCP_ERR_INVALID_ARG;
  }
  if (o.late_precision < -1 || o.late_precision > GCP_BF16X6 || !(o.switch_ddbar >= 0.0) ||
      o.final_precision < -1 || o.final_precision > GCP_BF16X6 || !(o.final_ddbar >= 0.0) ||
      (o.late_precision >= 0 && o.final_precision >= 0 && o.final_ddbar > o.switch_ddbar)) {
    err = "gcp_create: late_precision and final_precision must be -1 or a precision, "
          "switch_ddbar and final_ddbar >= 0, final_ddbar <= switch_ddbar";
    return GCP_ERR_INVALID_ARG;
  }
  if (o.sync_every < 1 || !(std::isnan(o.floor_ddbar) || o.floor_ddbar >= 0.0) ||
      o.ksplit < 0 || o.ksplit > 64) {
    err = "gcp_create: sync_every must be >= 1, ksplit in [0, 64] and floor_ddbar NaN or >= 0";
    return GCP_ERR_INVALID_ARG;
  }
  if (o.method < GCP_METHOD_HPCP || o.method > GCP_METHOD_PMCP || o.init_mode < GCP_INIT_PMCP ||
      o.init_mode > GCP_INIT_HP_SEARCH || !(o.alpha >= 0.0 && o.alpha <= 1.0) ||
      !(o.delta > 0.5 && o.delta < 1.0) || (o.hole != 0 && o.hole != 1) ||
      o.checkpoint_every < 0) {
    err = "gcp_create: method, init_mode, alpha in [0,1], delta in (1/2,1), hole or "
          "checkpoint_every invalid";
    return GCP_ERR_INVALID_ARG;
  }
  return GCP_OK;
}

// Sizes and launch configuration of a context for M x M problems.
static void setup_ctx(gcp_ctx *c, int64_t M, const gcp_options &o, void *stream) {
  c->M = M;
  c->Mp = (M + 255) / 256 * 256;   // whole pairs of 128-wide tiles
  c->nt = (int)(c->Mp / 128);
  c->ntiles = c->nt * (c->nt + 1) / 2;
  c->nred = (int)((c->Mp + 63) / 64);   // k_reduce blocks (64 rows each)
  c->opt = o;
  c->stream = (hipStream_t)stream;
  (void)hipGetDevice(&c->device);
  // the schedule's phases: an encoding that repeats the previous one adds none
  c->pc[0].prec = o.precision;
  c->pc[0].enter_ddbar = INFINITY;
  c->nprec = 1;
  const int later[2] = {o.late_precision, o.final_precision};
  const double enter[2] = {o.switch_ddbar, o.final_ddbar};
  for (int q = 0; q < 2; ++q)
    if (later[q] >= 0 && later[q] != c->pc[c->nprec - 1].prec) {
      c->pc[c->nprec].prec = later[q];
      c->pc[c->nprec].enter_ddbar = enter[q];
      ++c->nprec;
    }
  // tile partial sums: one per upper tile (FP64/FP32 kernel) or two per
  // tile pair (16-bit kernel, zero for the half of a pair below the diagonal)
  c->ntpart = 0;
  for (int k = 0; k < c->nprec; ++k) {
    PrecCfgInit(c, k);
    if (c->pc[k].ntpart > c->ntpart) c->ntpart = c->pc[k].ntpart;
  }
}

// K-split units of the product launches of any phase: the most units
// (arrival counters) and the most split blocks (partial tiles of 128 KB).
static void split_tail(const gcp_ctx *c, int &tail, int &blocks) {
  tail = 0;
  blocks = 0;
  for (int k = 0; k < c->nprec; ++k)
    if (c->pc[k].ntail > 0) {
      tail = std::max(tail, c->pc[k].ntail);
      blocks = std::max(blocks, c->pc[k].ntail * c->pc[k].nsplit);
    }
}

// Every device buffer of the context with its size, in a fixed order.
// one_shot: a solve that is neither re-run from its D_0 nor differentiated,
// whose D_0 is built in place in the first D buffer.
template <class F>
static void for_each_buffer(gcp_ctx *c, bool one_shot, F &&f) {
  const size_t Mp = (size_t)c->Mp;
  const size_t vec = Mp * sizeof(double);
  const size_t nslots_max = Mp / 64;   // the initial guess uses 64-wide column slots
  const size_t pb = plane_bytes(c);
  f(&c->Dp[0], pb);
  f(&c->Dp[1], pb);
  f(&c->X2p, pb);
  if (!one_shot) f(&c->D0p, pb);
  for (int k = 0; k < 2; ++k) {
    f((void **)&c->dg[k], vec);
    f((void **)&c->rD[k], vec);
    f((void **)&c->d2[k], vec);
  }
  f((void **)&c->s2, vec);
  f((void **)&c->d3, vec);
  if (!one_shot) {
    f((void **)&c->dg0, vec);
    f((void **)&c->rD0, vec);
    f((void **)&c->d20, vec);
  }
  f((void **)&c->part, nslots_max * vec);
  f((void **)&c->tpart, (size_t)c->ntpart * sizeof(double));
  f((void **)&c->bpart, (size_t)2 * c->nred * sizeof(double));
  f((void **)&c->hvec, 3 * vec);
  f((void **)&c->counter, sizeof(unsigned));
  f((void **)&c->sc, sizeof(Scalars));
  f((void **)&c->hist, (size_t)(c->opt.max_iter + 1) * GCP_HIST_COLS * sizeof(double));
  int tail, blocks;
  split_tail(c, tail, blocks);
  if (tail > 0) {
    // one partial tile of 128 KB per split block (FP32 128 x 256 of the
    // 16-bit kernel, FP64 128 x 128 of the FP64 one)
    f(&c->split_ws, (size_t)blocks * 128 * 1024);
    f((void **)&c->split_cnt, (size_t)tail * sizeof(unsigned));
  }
  if (c->nprec > 1) f(&c->Xc, pb);
  if (!one_shot && c->opt.keep_iterates) {
    const size_t bb = Mp * Mp * (size_t)elem_size(c->opt.bwd_precision);
    f(&c->bG[0], bb);
    f(&c->bG[1], bb);
    f(&c->bX2, bb);
    f(&c->bAT, bb);
    f(&c->bCT, bb);
    f((void **)&c->btpart, ((size_t)c->nt * (c->nt + 1) + (size_t)c->nt * c->nt) * sizeof(double));
    f((void **)&c->bvec, (2 * Mp + 8) * sizeof(double));
  }
}

extern "C" int gcp_create(gcp_ctx **out, int64_t M, const gcp_options *opt, void *stream) {
  if (!out) {
    g_create_error = "gcp_create: ctx pointer is NULL";
    return GCP_ERR_INVALID_ARG;
  }
  *out = nullptr;
  gcp_options o;
  if (opt) o = *opt; else gcp_options_default(&o);
  int st = check_options(o, M, g_create_error);
  if (st != GCP_OK) return st;
  gcp_ctx *c = new (std::nothrow) gcp_ctx();
  if (!c) {
    g_create_error = "gcp_create: out of host memory";
    return GCP_ERR_NO_MEMORY;
  }
  setup_ctx(c, M, o, stream);
  bool ok = true;
  for_each_buffer(c, false, [&](void **p, size_t bytes) {
    if (!ok) return;
    if (hipMalloc(p, bytes) != hipSuccess) {
      ok = false;
      *p = nullptr;
    }
  });
  if (ok && hipHostMalloc((void **)&c->sc_host, sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
    ok = false;
  if (!ok) {
    free_all(c);
    delete c;
    g_create_error = "gcp_create: device allocation failed";
    return GCP_ERR_NO_MEMORY;
  }
  int ntail, nblk;
  split_tail(c, ntail, nblk);
  const size_t vec = (size_t)c->Mp * sizeof(double);
  if ((c->split_cnt && hipMemsetAsync(c->split_cnt, 0, (size_t)ntail * sizeof(unsigned),
                                     c->stream) != hipSuccess) ||
      hipMemsetAsync(c->counter, 0, sizeof(unsigned), c->stream) != hipSuccess ||
      hipMemsetAsync(c->s2, 0, vec, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    free_all(c);
    delete c;
    g_create_error = "gcp_create: initialisation of the workspace failed";
    return GCP_ERR_HIP;
  }
  *out = c;
  return GCP_OK;
}

extern "C" void gcp_destroy(gcp_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

extern "C" const char *gcp_last_error(const gcp_ctx *c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

static int reduce(gcp_ctx *c, const double *part, int nslots, int mode, double *out,
                  const double *extra, const double *tpart, int ntp, int iter,
                  bool skip_if_stopped = false, double floor_ddbar = 0.0,
                  bool early_stop = false, bool recheck = false) {
  RedArgs a{};
  a.part = part;
  a.nslots = nslots;
  a.mode = mode;
  a.Mp = c->Mp;
  a.out = out;
  a.extra = extra;
  a.bpart = c->bpart;
  a.counter = c->counter;
  a.tpart = tpart;
  a.ntiles = ntp;
  a.iter = iter;
  a.max_iter = c->opt.max_iter;
  a.tol_ddbar = c->opt.tol_ddbar;
  a.tol_idem = c->opt.tol_idem;
  a.N = (double)(c->opt.hole ? c->M - c->N : c->N);   // trace of the purified matrix
  a.floor_ddbar = floor_ddbar;
  a.skip_if_stopped = skip_if_stopped ? 1 : 0;
  a.early_stop = early_stop ? 1 : 0;
  a.recheck = recheck ? 1 : 0;
  a.sc = c->sc;
  a.hist = c->hist;
  HIPCHK(c, launch_reduce(a, c->stream));
  return GCP_OK;
}

static int build_guess(gcp_ctx *c, const double *H, int64_t ldh, double theta, double beta,
                       double mu);
static int first_traces(gcp_ctx *c);

// Rounding floor of |Tr(D Dbar)| for encoding pc[k] (unless the caller gave
// one).  One update leaves an off-diagonal error of relative size
// rho = u_enc + 2 u_acc sqrt(kappa) (encoding of the result, and the
// accumulation of the product over kappa rounding steps, statistically)
// on elements of typical size sqrt(N)/M.  The diagonal is exact, so near a
// projector P the error E moves Tr(D Dbar) by Tr(E (I - 2P)) = -2 Tr(E P),
// a sum with standard deviation 2 rho sqrt(N)/M ||P||_F = 2 rho N / M.  The
// floor is ten times that.
static double rounding_floor(const gcp_ctx *c, int k) {
  if (!std::isnan(c->opt.floor_ddbar)) return c->opt.floor_ddbar;
  const int prec = c->pc[k].prec;
  double u_enc = 0.0;
  switch (prec) {
    case GCP_FP32: u_enc = std::ldexp(1.0, -24); break;
    case GCP_BF16: u_enc = std::ldexp(1.0, -8); break;     // 8-bit significand
    case GCP_FP16: u_enc = std::ldexp(1.0, -11); break;    // 11-bit significand
    case GCP_BF16X3: u_enc = std::ldexp(1.0, -16); break;
    case GCP_FP16X3: u_enc = std::ldexp(1.0, -22); break;
    case GCP_BF16X6: u_enc = std::ldexp(1.0, -24); break;
    default: break;
  }
  const double u_acc = std::ldexp(1.0, prec == GCP_FP64 ? -53 : -24);
  double kappa = (double)c->Mp + 1.0;   // one accumulator over K
  if (prec == GCP_FP32) {                // chunks of fold stages of 32 K values
    const double f = (double)c->pc[k].fold;
    kappa = 32.0 * f + (double)(c->Mp / 32) / f;
  } else if (elem_size(prec) == 2) {
    const int np = plane_count(prec);
    const double stages = np <= 2 ? (double)c->Mp * np / 64.0 : (double)c->Mp / 32.0;
    const double per_stage = np == 1 ? 2.0 : (double)products(prec);
    const double f = (double)c->pc[k].fold;
    const double ks = c->pc[k].nfull == 0 ? (double)c->pc[k].nsplit : 1.0;   // ksplit
    kappa = 32.0 * per_stage * f + stages / ks / f;
  }
  const double rho = u_enc + 2.0 * u_acc * std::sqrt(kappa);
  const double n_eff = (double)(c->opt.hole ? c->M - c->N : c->N);
  return 20.0 * rho * n_eff / (double)c->M;
}

// Fields of the product launch that do not change within a solve.
static void setup_gemm(gcp_ctx *c, GemmArgs &g, int pi) {
  const gcp_ctx::PrecCfg &q = c->pc[pi];
  g.Mp = c->Mp;
  g.pstride = c->Mp * c->Mp;
  g.nt = c->nt;
  g.fold = q.fold;
  g.nfull = q.nfull;
  g.nsplit = q.nsplit;
  g.method = c->opt.method;
  g.ws = c->split_ws;
  g.cnt = c->split_cnt;
  g.part = c->part;
  g.tpart = c->tpart;
  g.s2 = c->s2;
  g.d3 = c->d3;
  g.coef = &c->sc->c;
  g.status = nullptr;   // set by gcp_purify's loop
}

extern "C" int gcp_init(gcp_ctx *c, const double *H, int64_t ldh, int64_t N, double emin,
                        double emax) {
  if (!c) return GCP_ERR_INVALID_ARG;
  c->inited = false;
  c->bwd_p = -1;
  if (!H || ldh < c->M || N < 0 || N > c->M) {
    c->err = "gcp_init: need H != NULL, ldh >= M and 0 <= N <= M";
    return GCP_ERR_INVALID_ARG;
  }
  const bool given = !std::isnan(emin) && !std::isnan(emax);
  if (given && !(emin < emax)) {
    c->err = "gcp_init: emin must be < emax";
    return GCP_ERR_INVALID_ARG;
  }
  const size_t vec = (size_t)c->Mp * sizeof(double);
  double *lo = c->hvec, *hi = c->hvec + c->Mp, *hd = c->hvec + 2 * c->Mp;
  HIPCHK(c, launch_hstats(H, ldh, c->M, lo, hi, hd, c->sc->hstat, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double g_lo = c->sc_host->hstat[0], g_hi = c->sc_host->hstat[1];
  const double trH = c->sc_host->hstat[2];
  if (!given) {
    emin = g_lo;
    emax = g_hi;
  }
  const double M = (double)c->M;
  const double theta = (double)N / M;
  const double mu = trH / M;
  double beta = 0.0, bmin = 0.0, bmax = 0.0, alpha = 1.0;
  bool searched = false;
  if (N > 0 && N < c->M) {
    if (!(emin < mu && mu < emax)) {
      c->err = "gcp_init: mu = Tr(H)/M must lie strictly inside (emin, emax)";
      return GCP_ERR_INVALID_ARG;
    }
    const double bt = theta / (emax - mu), bb = (1.0 - theta) / (mu - emin);
    bmin = bt < bb ? bt : bb;
    bmax = bt < bb ? bb : bt;
    beta = bmin;
    if (c->opt.init_mode == GCP_INIT_HP) {
      alpha = c->opt.alpha;
    } else if (c->opt.init_mode == GCP_INIT_HP_SEARCH) {
      // Tr(D0^2) = N theta + beta^2 ||H - mu I||_F^2 for D0 = theta I + beta (mu I - H):
      // the target fixes beta, and beta = alpha beta_min + (1 - alpha) beta_max fixes alpha
      const double delta = c->opt.delta;
      double target = NAN;
      if (theta < 1.0 - delta) target = (double)N - delta * (double)N;
      else if (theta > delta) target = (double)N - delta * (double)(c->M - N);
      if (std::isnan(target)) {
        alpha = 0.5;
      } else {
        HIPCHK(c, launch_hdev(H, ldh, c->M, c->Mp, mu, c->part, &c->sc->hstat[3], c->stream));
        HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const double S = c->sc_host->hstat[3];
        c->hdev = S;
        const double b2 = (target - (double)N * theta) / S;
        if (!(b2 > 0.0) || !(S > 0.0)) {
          alpha = 1.0;
        } else if (bmax > bmin) {
          alpha = (bmax - std::sqrt(b2)) / (bmax - bmin);
          searched = alpha > 0.0 && alpha < 1.0;
          alpha = alpha < 0.0 ? 0.0 : (alpha > 1.0 ? 1.0 : alpha);
        }
      }
    }
    beta = alpha * bmin + (1.0 - alpha) * bmax;
  }
  c->N = N;
  c->mu = mu;
  c->emin = emin;
  c->emax = emax;
  c->beta_min = bmin;
  c->beta_max = bmax;

  for (int attempt = 0; attempt < 2; ++attempt) {
    // the hole recursion starts from I - D_0 = (1 - theta) I - beta (mu I - H)
    int st = c->opt.hole ? build_guess(c, H, ldh, 1.0 - theta, -beta, mu)
                         : build_guess(c, H, ldh, theta, beta, mu);
    if (st != GCP_OK) return st;
    if (c->opt.init_mode == GCP_INIT_PMCP || !(N > 0 && N < c->M) || attempt == 1) break;
    // hole-particle guess: one product gives c_0; Tr(D0 Dbar0) <= 0 or c_0
    // outside [0, 1] means the recursion would run away: use alpha = 1
    st = first_traces(c);
    if (st != GCP_OK) return st;
    const double t1 = c->sc_host->t1, t2 = c->sc_host->t2, t3 = c->sc_host->t3;
    const double c0 = (t2 - t3) / (t1 - t2);
    if (t1 - t2 > 0.0 && c0 >= 0.0 && c0 <= 1.0) break;
    alpha = 1.0;
    beta = bmin;
    searched = false;
  }
  c->alpha = alpha;
  c->alpha_searched = searched;
  c->beta = beta;
  for (int k = 0; k < c->nprec; ++k) c->pc[k].floor_ddbar = rounding_floor(c, k);
  (void)vec;
  c->inited = true;
  return GCP_OK;
}

// D_0 = theta I + beta (mu I - H) in the main encoding, its FP64 diagonal and
// the traces T1, T2 (kept in t1_0, t2_0).
static int build_guess(gcp_ctx *c, const double *H, int64_t ldh, double theta, double beta,
                       double mu) {
  InitArgs a{};
  a.H = H;
  a.ldh = ldh;
  a.M = c->M;
  a.Mp = c->Mp;
  a.pstride = c->Mp * c->Mp;
  a.theta = theta;
  a.beta = beta;
  a.mu = mu;
  a.out = c->D0p;
  a.dg = c->dg0;
  a.rD = c->rD0;
  a.part = c->part;
  HIPCHK(c, launch_init(c->opt.precision, a, c->stream));
  int st = reduce(c, c->part, (int)(c->Mp / 64), 0, c->d20, c->dg0, nullptr, 0, 0);
  if (st != GCP_OK) return st;
  HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->t1_0 = c->sc_host->t1;
  c->t2_0 = c->sc_host->t2;
  return GCP_OK;
}

// T1, T2, T3 of D_0 (one D^2 product, as the first step of gcp_purify) into
// c->sc_host.
static int first_traces(gcp_ctx *c) {
  GemmArgs g{};
  setup_gemm(c, g, 0);
  g.mode = 0;
  g.A = c->D0p;
  g.B = c->D0p;
  g.out = c->X2p;
  g.dg = c->dg0;
  g.rD = c->rD0;
  g.d2 = c->d20;
  HIPCHK(c, launch_gemm(c->pc[0].prec, g, c->stream));
  int st = reduce(c, c->part, c->nt, 1, c->d3, nullptr, c->tpart, c->pc[0].ntpart, 0);
  if (st != GCP_OK) return st;
  HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GCP_OK;
}

extern "C" int gcp_get_init_scalars(const gcp_ctx *c, double *mu, double *beta, double *emin,
                                    double *emax, double *alpha) {
  if (!c) return GCP_ERR_INVALID_ARG;
  if (!c->inited) return GCP_ERR_STATE;
  if (mu) *mu = c->mu;
  if (beta) *beta = c->beta;
  if (emin) *emin = c->emin;
  if (emax) *emax = c->emax;
  if (alpha) *alpha = c->alpha;
  return GCP_OK;
}

// Keeps iterate D_n (forward planes Dp[k] plus its FP64 diagonal) as slot n.
static int store_iterate(gcp_ctx *c, int n, int k, int prec) {
  const size_t bytes = (size_t)c->Mp * (size_t)c->Mp * (size_t)elem_size(c->opt.bwd_precision);
  while ((int)c->slots.size() <= n) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      c->err = "gcp_purify: out of device memory for the iterates kept for gcp_backward";
      return GCP_ERR_NO_MEMORY;
    }
    c->slots.push_back(p);
  }
  HIPCHK(c, launch_bwd_store(prec, c->opt.bwd_precision, c->Dp[k], c->dg[k], c->Mp,
                             c->slots[n], c->stream));
  return GCP_OK;
}

// Launch accounting of one solve (events when profiling, issued MFMA flops).
struct LaunchLog {
  bool prof = false;
  int n = 0;
  int phase[3] = {0, 0, 0};   // launches in each phase of the schedule
  int reruns = 0;             // second K1 of an update after a change of encoding
};

// One product launch in encoding pc[pi].
static int run_product(gcp_ctx *c, GemmArgs &g, int pi, LaunchLog *log) {
  const gcp_ctx::PrecCfg &q = c->pc[pi];
  g.fold = q.fold;
  g.nfull = q.nfull;
  g.nsplit = q.nsplit;
  const bool ev = log && log->prof && 2 * log->n + 1 < (int)c->events.size();
  if (ev) HIPCHK(c, hipEventRecord(c->events[2 * log->n], c->stream));
  HIPCHK(c, launch_gemm(q.prec, g, c->stream));
  if (ev) HIPCHK(c, hipEventRecord(c->events[2 * log->n + 1], c->stream));
  if (log) {
    ++log->n;
    ++log->phase[pi];
  }
  return GCP_OK;
}

// K1 of update n on the iterate in buffer k: X2 = D D and the scalar step.
// recheck: the same iterate once more, in a new encoding (after a switch).
static int step_k1(gcp_ctx *c, GemmArgs &g, int pi, int k, int n, LaunchLog *log,
                   bool recheck = false) {
  g.mode = 0;
  g.A = c->Dp[k];
  g.B = c->Dp[k];
  g.out = c->X2p;
  g.dg = c->dg[k];
  g.rD = c->rD[k];
  g.d2 = c->d2[k];
  int st = run_product(c, g, pi, log);
  if (st != GCP_OK) return st;
  return reduce(c, c->part, c->nt, 1, c->d3, nullptr, c->tpart, c->pc[pi].ntpart, n,
                g.status != nullptr, c->pc[pi].floor_ddbar, false, recheck);
}

// K2 of update n: D_{n+1} into buffer 1 - k.
static int step_k2(gcp_ctx *c, GemmArgs &g, int pi, int k, int n, LaunchLog *log) {
  g.mode = 1;
  g.A = c->X2p;
  g.B = c->Dp[k];
  g.out = c->Dp[1 - k];
  g.dg_new = c->dg[1 - k];
  g.rD_new = c->rD[1 - k];
  int st = run_product(c, g, pi, log);
  if (st != GCP_OK) return st;
  // In the solve (not when a segment is recomputed for the adjoint) the
  // stops that need only the new traces are decided here, unless the
  // idempotency test, which needs the next square, is on.
  const bool solve = g.status != nullptr;
  return reduce(c, c->part, c->nt, 2, c->d2[1 - k], c->dg[1 - k], c->tpart, c->pc[pi].ntpart, n,
                solve, c->pc[pi].floor_ddbar, solve && !(c->opt.tol_idem > 0.0));
}

// Precision schedule: re-encode D_n (buffer k) from phase `from` into phase
// `to`'s encoding, the FP64 diagonal kept and the new encoding's residual in
// rD.  D_n^2 is then formed again, in the new encoding, by a second K1 of
// the same update (recheck): c_n and the next iterate then carry none of the
// old encoding's rounding of D^2 (with it, the first update of a precise
// phase inherits the old encoding's noise in Tr(D Dbar), which can be
// negative far above the new encoding's rounding floor).
static int switch_precision(gcp_ctx *c, int k, int from, int to) {
  const int pa = c->pc[from].prec, pb = c->pc[to].prec;
  HIPCHK(c, launch_convert(pa, pb, c->Dp[k], c->dg[k], c->Xc, c->rD[k], c->Mp, c->stream));
  std::swap(c->Dp[k], c->Xc);
  return GCP_OK;
}

// Checkpoint j: the forward state that K1 of update j * checkpoint_every reads.
static int save_checkpoint(gcp_ctx *c, int j, int k, int pi) {
  const size_t vec = (size_t)c->Mp * sizeof(double);
  while ((int)c->ckpts.size() <= j) {
    gcp_ctx::Ckpt q;
    if (hipMalloc(&q.planes, plane_bytes(c)) != hipSuccess ||
        hipMalloc((void **)&q.vec, 3 * vec) != hipSuccess) {
      if (q.planes) (void)hipFree(q.planes);
      c->err = "gcp_purify: out of device memory for the checkpoints kept for gcp_backward";
      return GCP_ERR_NO_MEMORY;
    }
    c->ckpts.push_back(q);
  }
  gcp_ctx::Ckpt &q = c->ckpts[j];
  q.pi = pi;
  HIPCHK(c, hipMemcpyAsync(q.planes, c->Dp[k], plane_bytes(c), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(q.vec, c->dg[k], vec, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(q.vec + c->Mp, c->rD[k], vec, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(q.vec + 2 * c->Mp, c->d2[k], vec, hipMemcpyDeviceToDevice, c->stream));
  return GCP_OK;
}

// Recompute updates [n0, n1) from checkpoint n0 / checkpoint_every, keeping
// D_n as slot n - n0 (the forward's kernels, launch configuration and
// decisions: bitwise the iterates of gcp_purify).
static int recompute_segment(gcp_ctx *c, int n0, int n1) {
  const size_t vec = (size_t)c->Mp * sizeof(double);
  const gcp_ctx::Ckpt &q = c->ckpts[n0 / c->opt.checkpoint_every];
  HIPCHK(c, hipMemcpyAsync(c->Dp[0], q.planes, plane_bytes(c), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->dg[0], q.vec, vec, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->rD[0], q.vec + c->Mp, vec, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d2[0], q.vec + 2 * c->Mp, vec, hipMemcpyDeviceToDevice, c->stream));
  Scalars s0{};   // traces of D_{n0}, as K1's reduction expects them
  s0.t1 = c->hist_host[(size_t)n0 * GCP_HIST_COLS + 1];
  s0.t2 = c->hist_host[(size_t)n0 * GCP_HIST_COLS + 2];
  s0.prev_ddbar = INFINITY;
  *c->sc_host = s0;
  HIPCHK(c, hipMemcpyAsync(c->sc, c->sc_host, sizeof(Scalars), hipMemcpyHostToDevice, c->stream));
  int pi = q.pi, k = 0;
  if (n0 == n1) {   // no update applied (p = 0): keep D_{n0} itself
    int st = store_iterate(c, 0, 0, c->pc[pi].prec);
    if (st != GCP_OK) return st;
  }
  GemmArgs g{};
  setup_gemm(c, g, pi);
  for (int n = n0; n < n1; ++n) {
    int st = step_k1(c, g, pi, k, n, nullptr);
    if (st != GCP_OK) return st;
    int to = pi;
    while (to + 1 < c->nprec && n == c->n_switch[to + 1]) ++to;
    if (to != pi) {
      st = switch_precision(c, k, pi, to);
      if (st != GCP_OK) return st;
      pi = to;
      st = step_k1(c, g, pi, k, n, nullptr, true);
      if (st != GCP_OK) return st;
    }
    st = store_iterate(c, n - n0, k, c->pc[pi].prec);
    if (st != GCP_OK) return st;
    st = step_k2(c, g, pi, k, n, nullptr);
    if (st != GCP_OK) return st;
    k = 1 - k;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));   // the host copy of the scalars is reused
  return GCP_OK;
}

extern "C" int gcp_purify(gcp_ctx *c, void *D, int32_t dtype, int64_t ldd, gcp_result *res) {
  if (!c) return GCP_ERR_INVALID_ARG;
  if (!c->inited) {
    c->err = "gcp_purify: call gcp_init first";
    return GCP_ERR_STATE;
  }
  if (!D || ldd < c->M || (dtype != GCP_DTYPE_F64 && dtype != GCP_DTYPE_F32)) {
    c->err = "gcp_purify: need D != NULL, ldd >= M and dtype F64 or F32";
    return GCP_ERR_INVALID_ARG;
  }
  const auto t_start = std::chrono::steady_clock::now();
  int pi = 0;                         // index of the current encoding in c->pc
  int prec = c->pc[0].prec;
  const size_t vec = (size_t)c->Mp * sizeof(double);
  const int64_t PS = c->Mp * c->Mp;
  const int max_iter = c->opt.max_iter;

  // start from D_0
  c->cur = 0;
  if (c->D0p != c->Dp[0]) {   // (a one-shot solve builds D_0 in place)
    HIPCHK(c, hipMemcpyAsync(c->Dp[0], c->D0p, plane_bytes(c), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dg[0], c->dg0, vec, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->rD[0], c->rD0, vec, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d2[0], c->d20, vec, hipMemcpyDeviceToDevice, c->stream));
  }
  Scalars s0{};
  s0.t1 = c->t1_0;
  s0.t2 = c->t2_0;
  s0.prev_ddbar = INFINITY;
  *c->sc_host = s0;
  HIPCHK(c, hipMemcpyAsync(c->sc, c->sc_host, sizeof(Scalars), hipMemcpyHostToDevice, c->stream));

  const bool keep = c->opt.keep_iterates != 0;
  c->bwd_p = -1;

  const bool prof = c->opt.profile != 0;
  // launches: K1 of updates 0..max_iter, K2 of 0..max_iter-1, plus at most
  // sync_every - 1 void launches of each past the stop
  const int max_launch = 2 * max_iter + 2 * c->opt.sync_every + 2;
  if (prof && (int)c->events.size() < 2 * max_launch) {
    for (int k = (int)c->events.size(); k < 2 * max_launch; ++k) {
      hipEvent_t e;
      HIPCHK(c, hipEventCreate(&e));
      c->events.push_back(e);
    }
  }
  LaunchLog lg;
  lg.prof = prof;
  GemmArgs g{};
  setup_gemm(c, g, 0);
  g.status = &c->sc->status;   // launches past the device's stop do nothing
  const int ck = keep && c->opt.checkpoint_every >= 2 ? c->opt.checkpoint_every : 0;
  for (int q = 0; q < 3; ++q) c->n_switch[q] = -1;

  // Update n reads D_n from buffer n % 2 and writes D_{n+1} to the other.
  // The decision to stop is taken on the device (k_reduce, before c_n is
  // formed); the host enqueues sync_every updates at a time and reads the
  // decision after each batch.  Until a precision schedule has switched, the
  // host checks after every D^2, because the switch is decided there.
  int status = 0, n = 0, syncs = 0;
  for (;;) {
    const bool per_step = pi + 1 < c->nprec;
    const int nb = per_step ? 1 : c->opt.sync_every;
    bool stopped = false;
    for (int q = 0; q < nb && n <= max_iter; ++q, ++n) {
      const int k = n & 1;
      if (ck && n % ck == 0) {
        int st = save_checkpoint(c, n / ck, k, pi);
        if (st != GCP_OK) return st;
      }
      int st = step_k1(c, g, pi, k, n, &lg);
      if (st != GCP_OK) return st;
      if (per_step) {
        HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        ++syncs;
        if (c->sc_host->status != 0) {
          stopped = true;
          break;
        }
        int to = pi;
        while (to + 1 < c->nprec &&
               std::fabs(c->sc_host->t1 - c->sc_host->t2) <= c->pc[to + 1].enter_ddbar) {
          ++to;
          c->n_switch[to] = n;
        }
        if (to != pi) {
          st = switch_precision(c, k, pi, to);
          if (st != GCP_OK) return st;
          pi = to;
          prec = c->pc[pi].prec;
          st = step_k1(c, g, pi, k, n, &lg, true);
          if (st != GCP_OK) return st;
          ++lg.reruns;
          HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                                   c->stream));
          HIPCHK(c, hipStreamSynchronize(c->stream));
          ++syncs;
          if (c->sc_host->status != 0) {
            stopped = true;
            break;
          }
        }
      }
      // the iterate K2 reads, in the encoding it reads it (after a switch)
      if (keep && !ck) {
        st = store_iterate(c, n, k, prec);
        if (st != GCP_OK) return st;
      }
      st = step_k2(c, g, pi, k, n, &lg);
      if (st != GCP_OK) return st;
    }
    if (!stopped) {
      HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                               c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      ++syncs;
    }
    if (c->sc_host->status != 0) break;
  }
  status = c->sc_host->status;
  n = c->sc_host->iter;
  c->cur = n & 1;
  const int iters = n;
  if (keep) c->bwd_p = iters;
  // output D_p
  OutArgs oa{};
  oa.planes = c->Dp[c->cur];
  oa.dg = c->dg[c->cur];
  oa.M = c->M;
  oa.Mp = c->Mp;
  oa.pstride = PS;
  oa.ldd = ldd;
  oa.D = D;
  oa.dtype = dtype;
  oa.hole = c->opt.hole;
  HIPCHK(c, launch_output(prec, oa, c->stream));
  c->hist_rows = iters + 1;
  double c_last = NAN;
  if (!c->one_shot) {
    c->hist_host.assign((size_t)c->hist_rows * GCP_HIST_COLS, NAN);
    HIPCHK(c, hipMemcpyAsync(c->hist_host.data(), c->hist, c->hist_host.size() * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  } else if (iters > 0) {   // only c of the last update
    HIPCHK(c, hipMemcpyAsync(&c_last, c->hist + (size_t)(iters - 1) * GCP_HIST_COLS + 4,
                             sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (!c->one_shot && iters > 0) c_last = c->hist_host[(size_t)(iters - 1) * GCP_HIST_COLS + 4];
  const auto t_end = std::chrono::steady_clock::now();

  int rc = GCP_OK;
  if (status == 2) rc = GCP_ERR_NOT_CONVERGED;
  if (status == 3) rc = GCP_ERR_BREAKDOWN;
  if (status == 4) rc = GCP_STOPPED_AT_FLOOR;
  // launches that did work: K1 of updates 0..p (0..p-1 when the stop was
  // decided from the traces of D_p), K2 of 0..p-1 and the second K1 after
  // each change of encoding (any after them were enqueued past the stop and
  // returned at once; they all fall in the last phase)
  const int worked = 2 * iters + (c->sc_host->on_traces ? 0 : 1) + lg.reruns;
  const int real = worked < lg.n ? worked : lg.n;
  if (res) {
    std::memset(res, 0, sizeof(*res));
    res->status = rc;
    res->iters = iters;
    res->t1 = c->sc_host->t1;
    res->t2 = c->sc_host->t2;
    if (c->opt.hole) {   // Tr D = M - Tr Dbar, Tr D^2 = M - 2 Tr Dbar + Tr Dbar^2
      res->t1 = (double)c->M - c->sc_host->t1;
      res->t2 = (double)c->M - 2.0 * c->sc_host->t1 + c->sc_host->t2;
    }
    res->c_last = c_last;
    res->idem = std::sqrt(c->sc_host->omega);
    res->ms_total = std::chrono::duration<double, std::milli>(t_end - t_start).count();
    res->gemm_launches = real;
    res->host_syncs = syncs;
    const double Md = (double)c->M;
    res->gemm_flops = (double)real * Md * Md * (Md + 1.0);
    // issued MFMA flops: whole 128 x 128 tiles of the padded size times the
    // split products, launch by launch in each phase's encoding
    const double tile_fl = (double)c->ntiles * 2.0 * 128.0 * 128.0 * (double)c->Mp;
    double mf = 0.0;
    for (int q = 0; q < c->nprec; ++q) {
      int nq = lg.phase[q];
      if (q == pi) nq -= lg.n - real;   // the void launches past the stop
      mf += (double)nq * products(c->pc[q].prec);
    }
    res->mfma_flops = tile_fl * mf;
    double ms = 0.0;
    if (prof) {
      for (int k = 0; k < real; ++k) {
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, c->events[2 * k], c->events[2 * k + 1]));
        ms += t;
      }
    }
    res->gemm_ms = ms;
  }
  if (rc == GCP_ERR_NOT_CONVERGED) c->err = "gcp_purify: max_iter reached before the tolerance";
  if (rc == GCP_ERR_BREAKDOWN)
    c->err = "gcp_purify: breakdown (c outside [0,1], Tr(D Dbar) <= 0 above the rounding floor, "
             "or a non-finite value)";
  if (rc == GCP_STOPPED_AT_FLOOR)
    c->err = "gcp_purify: stopped at the rounding floor of the encoding above tol_ddbar";
  return rc;
}

extern "C" int gcp_backward(gcp_ctx *c, const void *dLdD, int64_t ldg, void *dLdH, int64_t ldh,
                            int32_t dtype, gcp_result *res) {
  if (!c) return GCP_ERR_INVALID_ARG;
  if (c->bwd_p < 0 || !c->inited) {
    c->err = "gcp_backward: needs a gcp_purify with keep_iterates = 1 after the last gcp_init";
    return GCP_ERR_STATE;
  }
  if (!dLdD || !dLdH || ldg < c->M || ldh < c->M ||
      (dtype != GCP_DTYPE_F64 && dtype != GCP_DTYPE_F32)) {
    c->err = "gcp_backward: need non-NULL buffers, ldg >= M, ldh >= M and dtype F64 or F32";
    return GCP_ERR_INVALID_ARG;
  }
  const auto t_start = std::chrono::steady_clock::now();
  const int bprec = c->opt.bwd_precision;
  const int p = c->bwd_p;
  const bool prof = c->opt.profile != 0;
  const int nlaunch_max = 3 * p;
  if (prof && (int)c->events.size() < 2 * nlaunch_max) {
    for (int k = (int)c->events.size(); k < 2 * nlaunch_max; ++k) {
      hipEvent_t e;
      HIPCHK(c, hipEventCreate(&e));
      c->events.push_back(e);
    }
  }
  int nlaunch = 0;
  double flops = 0.0, mflops = 0.0;
  const double Md = (double)c->M, tile_fl = 2.0 * 128.0 * 128.0 * (double)c->Mp;
  const int ntri = c->nt * (c->nt + 1) / 2;
  auto gemm = [&](BwdArgs &a) -> int {
    if (prof) HIPCHK(c, hipEventRecord(c->events[2 * nlaunch], c->stream));
    HIPCHK(c, launch_bwd_gemm(bprec, a, c->stream));
    if (prof) HIPCHK(c, hipEventRecord(c->events[2 * nlaunch + 1], c->stream));
    ++nlaunch;
    if (a.mode == 1) {
      flops += 4.0 * Md * Md * Md;
      mflops += 2.0 * c->nt * c->nt * tile_fl;
    } else {
      flops += Md * Md * (Md + 1.0);
      mflops += ntri * tile_fl;
    }
    return GCP_OK;
  };

  HIPCHK(c, launch_bwd_load(bprec, dLdD, ldg, dtype, c->M, c->Mp, c->bG[0], c->stream));
  int cur = 0;
  double *kappa = c->bvec + 2 * c->Mp;
  BwdArgs a{};
  a.Mp = c->Mp;
  a.nt = c->nt;
  a.X2 = c->bX2;
  a.AT = c->bAT;
  a.CT = c->bCT;
  a.kappa = kappa;
  a.tpart = c->btpart;
  // iterates: all kept (slot n = D_n), or recomputed segment by segment from
  // the checkpoints (slot n - n0 = D_n), last segment first
  const int ck = c->opt.checkpoint_every >= 2 ? c->opt.checkpoint_every : 0;
  int n0 = ck ? (p > 0 ? (p - 1) / ck * ck : 0) : 0;
  if (ck) {
    int st = recompute_segment(c, n0, p);
    if (st != GCP_OK) return st;
  }
  for (int n = p - 1; n >= 0; --n) {
    if (ck && n < n0) {
      n0 -= ck;
      int st = recompute_segment(c, n0, n0 + ck);
      if (st != GCP_OK) return st;
    }
    const double *h = c->hist_host.data() + (size_t)n * GCP_HIST_COLS;
    const double cn = h[4], t12 = h[1] - h[2];
    double da, db, de;
    update_coefs(c->opt.method, cn, a.a, a.b, a.e);
    update_coef_derivs(c->opt.method, cn, da, db, de);
    a.D = c->slots[n - n0];
    a.G = c->bG[cur];
    a.c = cn;
    a.inv_t12 = 1.0 / t12;
    a.need_x3 = de != 0.0;
    // X2 = D D and the partial sums of <G, D^2> and <G, D>
    a.mode = 0;
    a.out0 = c->bX2;
    int st = gemm(a);
    if (st != GCP_OK) return st;
    // AT = D G, CT = X2 G (and the partial sums of <G, D^3> = <X2, AT>)
    a.mode = 1;
    a.out0 = c->bAT;
    a.out1 = c->bCT;
    st = gemm(a);
    if (st != GCP_OK) return st;
    HIPCHK(c, launch_bwd_kappa(c->btpart, ntri, c->nt * c->nt, da, db, de, kappa, c->stream));
    // Gbar_n
    a.mode = 2;
    a.out0 = c->bG[1 - cur];
    st = gemm(a);
    if (st != GCP_OK) return st;
    cur = 1 - cur;
  }
  BwdInitArgs ia{};
  ia.G0 = c->bG[cur];
  ia.D0 = c->slots[0];
  ia.M = c->M;
  ia.Mp = c->Mp;
  ia.ldh = ldh;
  ia.theta = (double)c->N / (double)c->M;
  ia.beta = c->beta;
  ia.dbeta = 0.0;
  ia.hdev = c->alpha_searched ? c->hdev : 0.0;
  if (c->N > 0 && c->N < c->M && !c->alpha_searched) {
    // beta = alpha beta_min + (1 - alpha) beta_max with alpha fixed; each
    // branch differentiated through mu with the bounds held fixed
    const double bt = ia.theta / (c->emax - c->mu), bb = (1.0 - ia.theta) / (c->mu - c->emin);
    const double dbt = ia.theta / ((c->emax - c->mu) * (c->emax - c->mu));
    const double dbb = -(1.0 - ia.theta) / ((c->mu - c->emin) * (c->mu - c->emin));
    const double dmin = bt <= bb ? dbt : dbb, dmax = bt <= bb ? dbb : dbt;
    ia.dbeta = c->alpha * dmin + (1.0 - c->alpha) * dmax;
  }
  ia.sign = 1.0;
  if (c->opt.hole) {   // Dbar_0 = (1 - theta) I - beta (mu I - H), dL/dDbar = -dL/dD
    ia.theta = 1.0 - ia.theta;
    ia.beta = -ia.beta;
    ia.dbeta = -ia.dbeta;
    ia.sign = -1.0;
  }
  ia.rows = c->bvec;
  ia.sums = c->bvec + 2 * c->Mp + 1;
  ia.dH = dLdH;
  ia.dtype = dtype;
  HIPCHK(c, launch_bwd_init(bprec, ia, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const auto t_end = std::chrono::steady_clock::now();
  if (res) {
    std::memset(res, 0, sizeof(*res));
    res->status = GCP_OK;
    res->iters = p;
    res->t1 = res->t2 = res->c_last = res->idem = NAN;
    res->ms_total = std::chrono::duration<double, std::milli>(t_end - t_start).count();
    res->gemm_launches = nlaunch;
    res->gemm_flops = flops;
    res->mfma_flops = mflops;
    double ms = 0.0;
    if (prof) {
      for (int k = 0; k < nlaunch; ++k) {
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, c->events[2 * k], c->events[2 * k + 1]));
        ms += t;
      }
    }
    res->gemm_ms = ms;
  }
  return GCP_OK;
}

extern "C" int gcp_verify(gcp_ctx *c, const void *D, int32_t dtype, int64_t ldd, const double *H,
                          int64_t ldh, gcp_verify_result *res) {
  if (!c) return GCP_ERR_INVALID_ARG;
  if (!D || !H || ldd < c->M || ldh < c->M || (dtype != GCP_DTYPE_F64 && dtype != GCP_DTYPE_F32)) {
    c->err = "gcp_verify: need non-NULL D and H, ldd >= M, ldh >= M and dtype F64 or F32";
    return GCP_ERR_INVALID_ARG;
  }
  const auto t_start = std::chrono::steady_clock::now();
  const size_t Mp = (size_t)c->Mp, mat = Mp * Mp * sizeof(double);
  const int ntri = c->nt * (c->nt + 1) / 2;
  if (!c->vD) {
    void *p[4] = {nullptr, nullptr, nullptr, nullptr};
    const size_t sz[4] = {mat, mat, mat, (4 * Mp + (size_t)ntri + 8) * sizeof(double)};
    for (int k = 0; k < 4; ++k) {
      if (hipMalloc(&p[k], sz[k]) != hipSuccess) {
        for (int q = 0; q < k; ++q) (void)hipFree(p[q]);
        c->err = "gcp_verify: device allocation of the workspace failed";
        return GCP_ERR_NO_MEMORY;
      }
    }
    c->vD = (double *)p[0];
    c->vH = (double *)p[1];
    c->vHD = (double *)p[2];
    c->vaux = (double *)p[3];
  }
  HIPCHK(c, launch_bwd_load(GCP_FP64, D, ldd, dtype, c->M, c->Mp, c->vD, c->stream));
  HIPCHK(c, launch_bwd_load(GCP_FP64, H, ldh, GCP_DTYPE_F64, c->M, c->Mp, c->vH, c->stream));
  VerifyArgs a{};
  a.D = c->vD;
  a.H = c->vH;
  a.HD = c->vHD;
  a.rows = c->vaux;
  a.tpart = c->vaux + 4 * Mp;
  a.out = c->vaux + 4 * Mp + ntri;
  a.Mp = c->Mp;
  a.nt = c->nt;
  a.ntri = ntri;
  HIPCHK(c, launch_verify(a, c->stream));
  double out[5];
  HIPCHK(c, hipMemcpyAsync(out, a.out, sizeof(out), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const auto t_end = std::chrono::steady_clock::now();
  if (res) {
    res->comm = std::sqrt(2.0 * out[0]);   // each off-diagonal pair counted once
    res->energy = out[1];
    res->fro2 = out[2];
    res->trace = out[3];
    res->idem = std::sqrt(out[4]);
    res->ms = std::chrono::duration<double, std::milli>(t_end - t_start).count();
  }
  return GCP_OK;
}

extern "C" int gcp_get_history(const gcp_ctx *c, double *rows, int32_t max_rows,
                               int32_t *n_rows) {
  if (!c || !n_rows) return GCP_ERR_INVALID_ARG;
  *n_rows = c->hist_rows;
  if (rows) {
    const int n = max_rows < c->hist_rows ? max_rows : c->hist_rows;
    if (n > 0) std::memcpy(rows, c->hist_host.data(), (size_t)n * GCP_HIST_COLS * sizeof(double));
  }
  return GCP_OK;
}

extern "C" int gcp_stream_lds(const void *buf, int64_t bytes, void *stream) {
  if (!buf || bytes <= 0 || bytes % 65536 != 0 || bytes / 65536 > 0x7fffffff) {
    g_create_error = "gcp_stream_lds: need buf != NULL and bytes a positive multiple of 65536";
    return GCP_ERR_INVALID_ARG;
  }
  const hipError_t e = launch_stream_lds(buf, bytes, (hipStream_t)stream);
  if (e != hipSuccess) {
    g_create_error.set("gcp_stream_lds", hipGetErrorString(e));
    return GCP_ERR_HIP;
  }
  return GCP_OK;
}

// ------------------------------------------------ solve without allocation
// Workspace of gcp_purify_static: one copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in; its device
// address on each GPU comes from hipGetSymbolAddress (kept per device) and is
// the only form in which host code uses it.
static __device__ __align__(256) unsigned char scratch[GCP_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this GPU's scratch array (the device must be current).
int scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) {
    g_create_error = "gcp_purify_static: device index out of range";
    return GCP_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      g_create_error.set("gcp_purify_static: hipGetSymbolAddress(scratch)", hipGetErrorString(e));
      return GCP_ERR_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GCP_OK;
}
}  // namespace

extern "C" int gcp_purify_static(const double *H, int64_t ldh, int64_t M, int64_t N, double emin,
                                 double emax, const gcp_options *opt, void *D, int32_t dtype,
                                 int64_t ldd, void *stream, gcp_result *out) {
  gcp_options o;
  if (opt) o = *opt; else gcp_options_default(&o);
  int st = check_options(o, M, g_create_error);
  if (st != GCP_OK) return st;
  if (M > GCP_STATIC_MAX_M) {
    std::snprintf(g_create_error.buf, sizeof(g_create_error.buf),
                  "gcp_purify_static: M = %lld exceeds GCP_STATIC_MAX_M = %d", (long long)M,
                  GCP_STATIC_MAX_M);
    return GCP_ERR_INVALID_ARG;
  }
  if (o.keep_iterates || o.profile) {
    g_create_error = "gcp_purify_static: keep_iterates and profile need allocations; use gcp_create";
    return GCP_ERR_INVALID_ARG;
  }
  gcp_ctx c;   // on the stack; its host containers stay empty
  c.one_shot = true;
  setup_ctx(&c, M, o, stream);
  void *base = nullptr;
  st = scratch_address(c.device, &base);
  if (st != GCP_OK) return st;
  size_t off = 0;
  for_each_buffer(&c, true, [&](void **p, size_t bytes) {
    off = (off + 255) / 256 * 256;
    *p = (off + bytes <= GCP_STATIC_SCRATCH_BYTES) ? (void *)((char *)base + off) : nullptr;
    off += bytes;
  });
  if (off > GCP_STATIC_SCRATCH_BYTES) {
    std::snprintf(g_create_error.buf, sizeof(g_create_error.buf),
                  "gcp_purify_static: the workspace of M = %lld needs %zu bytes, more than the "
                  "static %u (lower max_iter)", (long long)M, off, GCP_STATIC_SCRATCH_BYTES);
    return GCP_ERR_INVALID_ARG;
  }
  c.D0p = c.Dp[0];
  c.dg0 = c.dg[0];
  c.rD0 = c.rD[0];
  c.d20 = c.d2[0];
  Scalars host_sc{};
  c.sc_host = &host_sc;
  // the array keeps the previous call's contents: the arrival counters and
  // the X2 diagonal residuals must start at zero
  int ntail, nblk;
  split_tail(&c, ntail, nblk);
  if (launch_zero(c.split_cnt, ntail, c.stream) != hipSuccess ||
      launch_zero(c.counter, 1, c.stream) != hipSuccess ||
      launch_zero(c.s2, 2 * c.Mp, c.stream) != hipSuccess) {
    g_create_error = "gcp_purify_static: clearing the workspace failed";
    return GCP_ERR_HIP;
  }
  st = gcp_init(&c, H, ldh, N, emin, emax);
  if (st == GCP_OK) st = gcp_purify(&c, D, dtype, ldd, out);
  if (st != GCP_OK) g_create_error = c.err.c_str();
  return st;
}
