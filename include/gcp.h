/*
 * gcp.h -- C ABI of libgcp: generalized canonical purification on one
 * AMD Instinct MI355X (gfx950).
 *
 * The library computes the ground-state one-particle density matrix D of a
 * real symmetric Hamiltonian H (M states, N occupied) without
 * diagonalisation, by the hole-particle canonical purification (HPCP) of
 * Truflandier, Dianzinga & Bowler, arXiv:1512.07236:
 *
 *   D_0     = theta I + beta (mu I - H)                          eqs. (dmguess),(pmcpguess)
 *             theta = N/M, mu = Tr(H)/M,
 *             beta  = min(theta/(emax - mu), (1-theta)/(mu - emin))
 *   D_{n+1} = D_n + 2 (D_n^2 Dbar_n - c_n D_n Dbar_n),  Dbar = I - D      eq. (hpcp3)
 *   c_n     = Tr(D_n^2 Dbar_n) / Tr(D_n Dbar_n)
 *
 * iterated until Tr(D_n Dbar_n) (the paper's criterion) or ||D_n^2 - D_n||_F
 * falls below a tolerance.  Tr D_n = N holds at every step by construction
 * (no a-posteriori trace correction).  Each iteration costs two symmetric
 * matrix products (D^2 and D^2 D), the paper's "two matrix multiplications".
 *
 * Conventions for every entry point
 *  - Matrices are dense, row-major, with a leading dimension (elements)
 *    >= M.  All matrix pointers are DEVICE pointers on the GPU that was
 *    current when the context was created, owned by the caller.
 *  - Work is enqueued on the stream given to gcp_create (a hipStream_t passed
 *    as void*; NULL = the default stream).  Entry points that must decide on
 *    the host (gcp_init, gcp_purify, gcp_backward) synchronise that stream.
 *  - Every function returns a gcp_status; nothing throws across the ABI.
 *    gcp_last_error() gives a text description of the last failure.
 *  - A context is not thread-safe; use one context per stream.
 */
#ifndef GCP_H
#define GCP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gcp_ctx gcp_ctx;

typedef enum {
    GCP_STOPPED_AT_FLOOR = 1,   /* not an error: |Tr(D Dbar)| stopped decreasing, or turned
                                   negative, while already within the rounding floor of the
                                   encoding (see floor_ddbar): the returned iterate is as
                                   idempotent as the arithmetic allows, above tol_ddbar */
    GCP_OK = 0,
    GCP_ERR_INVALID_ARG = -1,   /* bad size, pointer, dtype, tolerance or bounds */
    GCP_ERR_HIP = -2,           /* a HIP runtime call failed (text in gcp_last_error) */
    GCP_ERR_NO_MEMORY = -3,     /* device or pinned-host allocation failed */
    GCP_ERR_NOT_CONVERGED = -4, /* max_iter updates applied without meeting a tolerance */
    GCP_ERR_BREAKDOWN = -5,     /* c_n outside [0,1], Tr(D Dbar) <= 0 above the rounding
                                   floor, or a non-finite value before convergence (the
                                   paper's runaway case) */
    GCP_ERR_STATE = -6,         /* call out of order (purify before init, ...) */
    GCP_ERR_UNSUPPORTED = -7    /* option combination not available */
} gcp_status;

/* Arithmetic of the two matrix products per iteration.  Traces, the
 * coefficient c_n, the diagonal of D, D^2 and D^3 and the termination test
 * are FP64 in every mode; off-diagonal iterates are stored in the product's
 * operand encoding.
 *   FP64     FP64 MFMA, FP64 storage.
 *   FP32     FP32 MFMA, FP32 storage.
 *   BF16     one bfloat16 operand, FP32 accumulate.
 *   FP16     one float16 operand (scaled by 2^10), FP32 accumulate.
 *   BF16X3   bfloat16 hi+lo split, 3 products (hi*hi, hi*lo, lo*hi).
 *   FP16X3   float16 hi+lo split of 2^10 x, 3 products (about 22 bits).
 *   BF16X6   bfloat16 hi+mid+lo split, 6 products (about 24 bits).        */
typedef enum {
    GCP_FP64 = 0,
    GCP_FP32 = 1,
    GCP_BF16 = 2,
    GCP_FP16 = 3,
    GCP_BF16X3 = 4,
    GCP_FP16X3 = 5,
    GCP_BF16X6 = 6
} gcp_precision;

/* Element types of caller buffers. */
typedef enum { GCP_DTYPE_F64 = 0, GCP_DTYPE_F32 = 1 } gcp_dtype;

typedef struct {
    int32_t precision;   /* gcp_precision */
    int32_t max_iter;    /* maximum number of updates (default 100) */
    double tol_ddbar;    /* stop when |Tr(D Dbar)| <= tol_ddbar (default 1e-6, the paper's) */
    double tol_idem;     /* stop when ||D^2 - D||_F <= tol_idem (default 0 = off) */
    int32_t fold_every;  /* FP32 and 16-bit encodings: add the FP32 chunk accumulator
                            into a second FP32 total every fold_every K stages (32
                            values of K per stage; 16-bit one- and two-plane
                            encodings: 64 halves of a row).  0 (default) = sqrt(stages /
                            accumulations per stage), which minimises the accumulated
                            rounding, the dominant error of the split encodings and
                            of FP32 at large M; a value >= the stage count never
                            folds.  FP64 keeps one accumulator. */
    int32_t profile;     /* 1: time every matrix-product launch with HIP events */
    int32_t keep_iterates; /* 1: gcp_purify keeps D_0 .. D_{p-1} for gcp_backward, one
                              M x M matrix of the adjoint's type per update (default 0) */
    int32_t bwd_precision; /* arithmetic of gcp_backward: GCP_FP64 (default) or GCP_FP32
                              (FP32 MFMA and storage; kappa and the traces stay FP64) */
    int32_t late_precision; /* precision schedule: -1 (default) = none; otherwise the
                               encoding of every product once |Tr(D Dbar)| <= switch_ddbar.
                               The switch re-encodes D and D^2 (the FP64 diagonal is
                               kept), so Tr D stays exact.  Rounding already made in the
                               occupied-virtual block is not undone by a later, more
                               precise encoding: a late FP64 phase makes the result
                               idempotent to FP64 level and lets it reach tolerances
                               below the early encoding's rounding floor. */
    int32_t final_precision; /* a third phase: -1 (default) = none; otherwise the encoding
                               of every product once |Tr(D Dbar)| <= final_ddbar (after
                               late_precision's phase, or directly from the first one when
                               late_precision is -1); final_ddbar <= switch_ddbar when
                               both are given.  E.g. FP16X3 -> BF16X6 -> FP64. */
    double switch_ddbar;   /* see late_precision (default 0) */
    int32_t method;        /* GCP_METHOD_HPCP (default): eq. (hpcp3); GCP_METHOD_PMCP: the
                              Palser-Manolopoulos canonical purification of the
                              appendix, eqs. (pm1a) (c <= 1/2) and (pm1b) (c > 1/2) */
    int32_t init_mode;     /* GCP_INIT_PMCP (default): eq. (pmcpguess), beta = min;
                              GCP_INIT_HP: the hole-particle guess of eq. (hpcpguess),
                              alpha D0 + (1 - alpha)(I - Dbar0) = theta I
                              + (alpha beta_min + (1 - alpha) beta_max)(mu I - H);
                              GCP_INIT_HP_SEARCH: alpha chosen so that Tr(D0^2) = N - delta N
                              (theta < 1 - delta) or N - delta (M - N) (theta > delta), else
                              alpha = 1/2 (eq. (hpcpguessalpha); closed form through
                              ||H - mu I||_F^2).  Both hole-particle guesses cost one extra
                              product in gcp_init, which checks c_0 and falls back to
                              alpha = 1 (the PMCP guess) when Tr(D0 Dbar0) <= 0 or c_0 is
                              outside [0, 1] (the runaway the paper reports for alpha = 1/2
                              at extreme fillings). */
    double alpha;          /* GCP_INIT_HP mixing coefficient, in [0, 1] (default 0.5) */
    double delta;          /* GCP_INIT_HP_SEARCH constant, in (1/2, 1) (default 2/3) */
    int32_t hole;          /* 1: purify the hole matrix Dbar = I - D instead (the alternative
                              the paper gives before eq. (hpcpguess)): Dbar_0 = I - D_0 of
                              the selected guess, trace M - N, and D = I - Dbar_p is returned.
                              HPCP is hole-particle symmetric (the same iterates up to
                              rounding); PMCP is not.  History rows and gcp_backward's
                              kept iterates are those of Dbar; result t1/t2 are of D. */
    int32_t checkpoint_every; /* with keep_iterates: 0 or 1 (default) keeps every iterate;
                              k >= 2 keeps only the state of every k-th iterate (operand
                              planes and FP64 diagonals) and gcp_backward recomputes each
                              segment of k updates from it with the forward kernels
                              (bitwise the same iterates), storing k iterates at a time:
                              memory p/k + k matrices instead of p, for two extra
                              products per update in the backward. */
    int32_t sync_every;    /* gcp_purify enqueues this many updates between host checks of
                              the termination decision (default 4; 1 = check after every
                              D^2).  Each update's decision is taken on the device before c_n
                              is formed, and launches enqueued past the stop do nothing, so
                              the iterates and the history do not depend on it.  A precision
                              schedule checks after every update until it has switched. */
    int32_t ksplit;        /* 16-bit encodings: split the K range of every tile pair over
                              ksplit blocks (2..64), whose FP32 totals the last of them
                              adds in FP64, in split order: the chunked accumulation is
                              then combined in FP64 across K.  Each block accumulates
                              K/ksplit, so a term passes through about 3 fold +
                              stages/(ksplit fold) FP32 roundings instead of 3 fold +
                              stages/fold, at the price of one 128 KB FP32 partial tile
                              written and read per block.  0 or 1 (default): only the last
                              partial round of pairs is split (for load balance). */
    double floor_ddbar;    /* rounding floor of |Tr(D Dbar)|: NaN (default) = derived by the
                              library from the encoding's unit roundoff and its accumulation
                              scheme, 20 rho N / M with rho = u_enc + 2 u_acc sqrt(kappa) (kappa:
                              rounding steps of a product element); 0 = none (every negative
                              Tr(D Dbar) or c outside [0,1] is a breakdown).  Within the floor a
                              stalled or negative Tr(D Dbar) stops the solve with
                              GCP_STOPPED_AT_FLOOR instead of GCP_ERR_BREAKDOWN. */
    double final_ddbar;    /* see final_precision (default 0) */
} gcp_options;

enum { GCP_METHOD_HPCP = 0, GCP_METHOD_PMCP = 1 };
enum { GCP_INIT_PMCP = 0, GCP_INIT_HP = 1, GCP_INIT_HP_SEARCH = 2 };

typedef struct {
    int32_t status;      /* gcp_status of the solve */
    int32_t iters;       /* updates applied (p) */
    double t1;           /* Tr D of the returned matrix (FP64) */
    double t2;           /* Tr D^2 (FP64) */
    double c_last;       /* last coefficient c_n used */
    double idem;         /* ||D^2 - D||_F of the returned matrix, when its square was
                            formed: with tol_idem = 0 (default) a stop on Tr(D Dbar)
                            (tolerance or rounding floor) is decided from the traces
                            of the last update, the last square is never formed and
                            idem is NaN (gcp_verify measures it in FP64) */
    double ms_total;     /* wall time of gcp_purify on the host clock (ms) */
    double gemm_ms;      /* summed device time of the matrix-product launches (profile=1) */
    int32_t gemm_launches; /* number of matrix-product launches that did work: 2p, or
                              2p + 1 when the stop needed the square of D_p */
    int32_t host_syncs;  /* host synchronisations of the iteration loop (gcp_purify) */
    double gemm_flops;   /* algorithmic flops of those launches (M^3 per product,
                            upper-triangle output; split products not counted) */
    double mfma_flops;   /* flops issued to the matrix cores (whole 128x128 tiles of the
                            padded size, times the number of split products) */
} gcp_result;

/* Fills *opt with the defaults listed above (precision FP64). */
int gcp_options_default(gcp_options *opt);

/* Creates a context for M x M problems on the current device and the given
 * stream and allocates its device workspace (four copies of the operand
 * encoding of an M x M matrix, O(M^2 / 64) FP64 partial sums, and 128 KB per
 * block of a product whose tiles are split along K: at most 16 MB for
 * M <= GCP_STATIC_MAX_M and 64 MB above, more with the ksplit option).  M >= 1;
 * M is padded internally to a multiple of 256 with zero rows/columns (exact:
 * the padding is an invariant zero block).  *ctx is set to NULL on failure. */
int gcp_create(gcp_ctx **ctx, int64_t M, const gcp_options *opt, void *stream);

/* Releases the context and its workspace (NULL is accepted). */
void gcp_destroy(gcp_ctx *ctx);

/* Builds D_0 from H (device FP64, M x M, leading dimension ldh >= M) and N,
 * eqs. (dmguess)+(pmcpguess).  emin/emax must bound the spectrum of H; if
 * either is NaN the Gershgorin bounds (section on the initial guess) are
 * used.  H is read as (H + H^T)/2.  H is not retained after the call.
 * Errors: INVALID_ARG for N outside [0, M], ldh < M, NULL H, emin >= emax, or
 * mu = Tr(H)/M outside (emin, emax) when 0 < N < M. */
int gcp_init(gcp_ctx *ctx, const double *H, int64_t ldh, int64_t N, double emin,
             double emax);

/* Runs the recursion of eq. (hpcp3) from the current D_0 and writes the
 * converged density matrix to D (device, M x M, leading dimension ldd,
 * dtype gcp_dtype).  D is valid once the context's stream is synchronised.
 * Returns OK on convergence, STOPPED_AT_FLOOR (a positive status, not an
 * error) when the rounding floor of the encoding was reached above tol_ddbar,
 * NOT_CONVERGED or BREAKDOWN otherwise (D then holds the last iterate and
 * *out is filled in every case; out may be NULL).
 * Calling it again re-runs the solve from the D_0 of the last gcp_init. */
int gcp_purify(gcp_ctx *ctx, void *D, int32_t dtype, int64_t ldd, gcp_result *out);

/* Reverse mode of the last gcp_purify (which must have run with keep_iterates = 1,
 * after the last gcp_init): given dL/dD of the returned matrix D_p (device,
 * M x M, leading dimension ldg, dtype gcp_dtype; read as its symmetric part),
 * writes dL/dH (device, M x M, leading dimension ldh, same dtype), the
 * gradient with respect to symmetric perturbations of H, for the p updates
 * that gcp_purify applied, whatever its status.  Every recursion, initial
 * guess and hole option is supported.
 *   - Each update, D' = a D + b D^2 + e D^3 with (a, b, e) functions of
 *     c = (T2 - T3)/(T1 - T2) (eq. (hpcp3), or eqs. (pm1a)/(pm1b) for PMCP),
 *     is differentiated including the dependence of c on D; this costs two
 *     symmetric and two general M x M products per update (about three
 *     times the forward).
 *   - The initial guess is differentiated through mu = Tr(H)/M and the
 *     slope beta: beta(mu) of eqs. (dmguess),(pmcpguess) or of the
 *     fixed-alpha guess of eq. (hpcpguess), with emin/emax held fixed (also
 *     when they were Gershgorin bounds derived from H); for the alpha
 *     search of eq. (hpcpguessalpha) (alpha strictly inside (0, 1)), beta
 *     through ||mu I - H||_F.  A searched alpha that fell back to 1 or was
 *     clamped to 0 or 1 is differentiated as that fixed alpha.
 *   - N = 0 or N = M gives dL/dH = 0 (D_0 does not depend on H).
 * The stored iterates stay valid for repeated calls (several loss gradients).
 * out may be NULL; out->iters = p, out->gemm_* count the adjoint products and
 * out->ms_total is the host wall time.  Errors: STATE without a purify that
 * kept its iterates, INVALID_ARG for NULL pointers, ld < M or a bad dtype. */
int gcp_backward(gcp_ctx *ctx, const void *dL_dD, int64_t ldg, void *dL_dH, int64_t ldh,
                 int32_t dtype, gcp_result *out);

/* Checks of a density matrix D against H, all in FP64 (MFMA products and
 * fixed-order sums); neither matrix needs to come from this context.
 * D (M x M, leading dimension ldd, dtype gcp_dtype) and H (FP64, M x M,
 * leading dimension ldh) are device pointers on the context's GPU, read as
 * their symmetric parts.  The values are those the paper uses to accept a
 * converged density matrix (the tests after the convergence discussion):
 *   trace     Tr D (N for the ground-state projector)
 *   fro2      ||D||_F^2 (also N for a projector)
 *   idem      ||D^2 - D||_F
 *   energy    Tr(D H) (the sum of the N lowest eigenvalues at the ground state)
 *   comm      ||H D - D H||_F
 * Work: two M^3-class FP64 products (D^2 on upper tiles, H D on all tiles).
 * The first call allocates three M x M FP64 matrices of workspace, kept by
 * the context.  Errors: INVALID_ARG for NULL pointers, ld < M or a bad dtype;
 * NO_MEMORY if the workspace cannot be allocated. */
typedef struct {
    double trace, fro2, idem, energy, comm;
    double ms;           /* host wall time of the call */
} gcp_verify_result;
int gcp_verify(gcp_ctx *ctx, const void *D, int32_t dtype, int64_t ldd, const double *H,
               int64_t ldh, gcp_verify_result *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the whole
 * solve of gcp_create + gcp_init + gcp_purify in one call that allocates
 * nothing.  Its workspace is a static device array of
 * GCP_STATIC_SCRATCH_BYTES, one per GPU, held by the library from its first
 * use on that GPU until the process ends; M is limited to GCP_STATIC_MAX_M.
 *   H, ldh, N, emin, emax   as for gcp_init (device FP64 H, NaN bounds ->
 *                           Gershgorin);
 *   opt                     as for gcp_create (NULL = defaults); keep_iterates
 *                           and profile must be 0 (they would allocate);
 *   D, dtype, ldd, out      as for gcp_purify (D device, out may be NULL);
 *   stream                  a hipStream_t as void* (NULL = default stream).
 * Returns the status gcp_purify would (OK, STOPPED_AT_FLOOR, NOT_CONVERGED,
 * BREAKDOWN), INVALID_ARG for M > GCP_STATIC_MAX_M or the options above, or
 * the errors of gcp_init; the text is in gcp_last_error(NULL).  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * host threads, other streams) race and must be serialised by the caller.
 * The iterates and D are bitwise those of gcp_create + gcp_init +
 * gcp_purify with the same options on the same GPU (the same kernels and
 * launch configuration). */
#define GCP_STATIC_MAX_M 1024
#define GCP_STATIC_SCRATCH_BYTES (48u << 20)
int gcp_purify_static(const double *H, int64_t ldh, int64_t M, int64_t N, double emin,
                      double emax, const gcp_options *opt, void *D, int32_t dtype, int64_t ldd,
                      void *stream, gcp_result *out);

/* Measurement support (not part of the method): reads `bytes` bytes of the
 * device buffer buf (a multiple of 65536) with the same loads the 16-bit
 * product kernel uses for its panels (global memory straight to LDS, 16 bytes
 * per lane, 128-byte row segments) and writes nothing, on the given stream.
 * A memory-traffic counter read over this kernel gives the factor that turns
 * that counter into bytes for the product kernel's loads.  Returns OK,
 * INVALID_ARG (NULL buf, bytes not a positive multiple of 65536) or HIP. */
int gcp_stream_lds(const void *buf, int64_t bytes, void *stream);

/* Per-iterate history of the last gcp_purify: GCP_HIST_COLS doubles per row,
 *   [n, Tr D, Tr D^2, Tr D^3, c_n, Omega = ||D^2-D||_F^2, gamma_n = (1-2c_n)/3,
 *    L_n = Omega - gamma_n (3 Tr D^2 - 2 Tr D^3 - N) (eq. mcw4b), ||D_{n+1} - D_n||_F]
 * for n = 0..iters (the last row has NaN where no update followed).
 * rows may be NULL to query *n_rows. */
#define GCP_HIST_COLS 9
int gcp_get_history(const gcp_ctx *ctx, double *rows, int32_t max_rows, int32_t *n_rows);

/* Scalars of the last gcp_init: mu, the slope beta of D_0 = theta I + beta (mu I - H),
 * emin, emax (bounds actually used) and alpha (1 for the PMCP guess or after the
 * fall-back).  Any output pointer may be NULL. */
int gcp_get_init_scalars(const gcp_ctx *ctx, double *mu, double *beta, double *emin,
                         double *emax, double *alpha);

/* Text of the last error on this context (or of the last failed gcp_create
 * when ctx is NULL).  The pointer stays valid until the next call. */
const char *gcp_last_error(const gcp_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GCP_H */
