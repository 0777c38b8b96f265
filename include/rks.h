/*
 * rks.h -- C-ABI of the MI355X randomized Krylov-Schur (rKS) eigensolver.
 *
 * The solver computes k eigenpairs of a large sparse non-symmetric matrix A
 * (Section 1, eq. "evp") with randomized Krylov-Schur: Algorithm 1 (rKS)
 * driving Algorithm 2 (extension of an rKS factorisation), residual
 * monitoring (Section 4.1), locking of converged Schur vectors (Sections
 * 4.2-4.4) and whitening re-orthogonalisation (Section 3.3).
 *
 * Conventions for every entry point:
 *   * Dense matrices are column-major.  "Host" pointers are ordinary CPU
 *     memory; "device" pointers are HIP device memory of the current device.
 *   * A call returns RKS_OK (0), RKS_ENOTCONV (1, results still valid for
 *     the converged pairs) or a negative error code; rks_last_error() then
 *     describes the failure.  No call aborts the process.
 *   * The context owns every device buffer it allocates; caller buffers are
 *     never retained after a call returns.  Calls on one context must not
 *     overlap; distinct contexts are independent.
 *   * All work is enqueued on the stream given in rks_opts (NULL = the
 *     default stream); calls that return host data synchronise that stream.
 */
#ifndef RKS_H
#define RKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define RKS_OK 0
#define RKS_ENOTCONV 1       /* max_restarts reached before every estimate <= tol */
#define RKS_EINVAL (-1)      /* invalid argument or malformed CSR */
#define RKS_ENOMEM (-2)      /* device or host allocation failed */
#define RKS_EHIP (-3)        /* a HIP runtime call failed */
#define RKS_ENAN (-4)        /* NaN/Inf in A, in u0 or in the iteration */
#define RKS_ESTATE (-5)      /* call order violated (e.g. eigpairs before solve) */
#define RKS_EBREAKDOWN (-6)  /* an exact invariant subspace that could not be continued past */
#define RKS_EDENSE (-7)      /* small dense step failed (QR iteration / reordering) */

/* Which part of the spectrum (Section 5: largest / smallest modulus; also
 * largest / smallest real part).  Ties are broken by larger imaginary part. */
typedef enum { RKS_LM = 0, RKS_SM = 1, RKS_LR = 2, RKS_SR = 3 } rks_which;

/* Oblivious subspace embedding Omega (Section 2, "Preliminaries"):
 *  GAUSS  -- dense, entries N(0, 1/d);
 *  SPARSE -- zeta nonzeros +-1/sqrt(zeta) per column in distinct rows
 *            (Section 5 uses zeta = 8).
 * Omega is never stored: its entries are regenerated from Philox4x32-10
 * counters (column index, slot) keyed by sketch_seed. */
typedef enum { RKS_SKETCH_GAUSS = 0, RKS_SKETCH_SPARSE = 1 } rks_sketch_kind;

/* Storage precision of the n-dimensional basis U (mixed precision is the
 * paper's future-work direction of Section 6; sketch-space quantities, the
 * Rayleigh quotient and all small dense steps stay FP64).  V32 and VBF16
 * store binary32 or bfloat16 columns and multiply them with binary32 copies
 * of A's values.  V32_FX16 stores each element x as a pair, 6 bytes: hi, its
 * binary32 rounding, and lo, a 16-bit signed integer, the remainder x - hi in
 * units of 2^-15 ulp(hi) rounded to nearest even (ulp(hi) = 2^(max(e,1) - 150)
 * for the biased binary32 exponent e of hi); the value hi + lo 2^-15 ulp(hi)
 * is within 2^-39 of x relative to it.  Arithmetic stays FP64, the products
 * with A read an FP64 copy of the column last written (n doubles more device
 * memory). */
typedef enum { RKS_PREC_FP64 = 0, RKS_PREC_V32 = 1, RKS_PREC_VBF16 = 2, RKS_PREC_V32_FX16 = 3 } rks_precision;

/* SpMV layout.  ROWS: wave tiles of consecutive rows.  COLUMN_BLOCKS: for
 * rows that gather x from everywhere, with x larger than an XCD's L2: the
 * columns split into 8 contiguous blocks and the rows into panels, one
 * workgroup per panel, which multiplies its rows block after block (all
 * workgroups on the same block at about the same time, so the gathered part
 * of x stays in L2) and keeps the row sums in LDS until w is written (it
 * stores a second copy of A, reordered by panel and block, with 16-bit row
 * offsets).  SLICED: slices of 64 consecutive rows, one row per lane of a
 * wave, each slice's nonzeros stored k-th of every row together (a sliced
 * ELLPACK layout, SELL-C with C = 64 as in Kreutzer et al., SIAM J. Sci.
 * Comput. 2014, rows padded to the longest row of their slice): a wave's
 * loads of the k-th nonzeros are contiguous, and on a banded matrix so are
 * its gathers of x; a lane adds its row's products in order in a register.
 * It stores a second copy of A in that order.  AUTO picks COLUMN_BLOCKS when
 * n >= 2^20 and the median column span of a row tile exceeds n/4, else
 * SLICED when the padding adds at most 1/8 to the nonzeros, else ROWS. */
typedef enum {
  RKS_SPMV_AUTO = 0,
  RKS_SPMV_ROWS = 1,
  RKS_SPMV_COLUMN_BLOCKS = 2,
  RKS_SPMV_SLICED = 3
} rks_spmv_layout;

/* RKS: randomized Krylov-Schur (Algorithm 1 with Algorithm 2).  KS_CGS2:
 * deterministic Krylov-Schur, the paper's point of comparison (Section 5):
 * the same restart on the same kernels, with the Euclidean inner product
 * and classical Gram-Schmidt applied twice in each Arnoldi step (four
 * passes over the basis instead of one); FP64 basis only; d and the sketch
 * options are ignored. */
typedef enum { RKS_METHOD_RKS = 0, RKS_METHOD_KS_CGS2 = 1 } rks_method;

/* Storage of A's values for the FP64 product (FP64 and pair bases, and the
 * FP64 residual checks) in the row-tile and sliced layouts.  AUTO: when A has at most
 * 256 distinct values (compared bit for bit), each nonzero stores a one-byte
 * index into the table of those values instead of the 8-byte value (a
 * value-indexed CSR, as in Kourtis, Goumas and Koziris, "Optimizing sparse
 * matrix-vector multiplication using index and value compression", 2008);
 * the SpMV looks the values up in a copy of the table in LDS and forms the
 * same FP64 products, so results are identical to the bit.  Constant-
 * coefficient stencils have a handful of values; matrices with more than 256
 * keep FP64 values.  FP64: always 8-byte values.  The FP32 and BF16 bases'
 * binary32 product and the column-blocked layout always store values. */
typedef enum { RKS_AVALUES_AUTO = 0, RKS_AVALUES_FP64 = 1 } rks_a_values;

/* rks_opts.keep: restart size chosen from k and m (see the field). */
#define RKS_KEEP_AUTO (-1)

/* Square CSR matrix: row_ptr[n+1] (monotone, row_ptr[0] = 0), col[nnz]
 * (in [0, n), strictly increasing inside a row), val[nnz] FP64.
 * on_device = 0: host arrays; 1: device arrays.  Copied by rks_create. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t* row_ptr;
  const int32_t* col;
  const double* val;
  int32_t on_device;
} rks_csr;

typedef struct {
  int32_t sketch_kind;   /* rks_sketch_kind, default SPARSE */
  int32_t zeta;          /* nonzeros per sparse-sign column, 1..8, default 8 */
  uint64_t sketch_seed;  /* default 0 */
  uint64_t start_seed;   /* seed of the N(0,1) start vector, default 1 */
  int32_t precision;     /* rks_precision, default FP64 */
  int32_t max_restarts;  /* contraction/extension cycles after the first extension, default 300 */
  int32_t lock;          /* 1: lock converged leading Schur vectors (Section 4.4), default;
                            2: before that, move every converged block of the wanted set to
                            the front (aggressive deflation, the reordering remark of
                            Section 4.4); 0: no locking */
  int32_t profile;       /* P > 0: time every P-th Arnoldi step on the solver's stream,
                            alternately per kernel (HIP events attached to the launches,
                            which take the dispatches' own start and end times) and as a
                            whole (one event pair recorded around the step, which adds a
                            few microseconds), and every rotation; 0 = off (default) */
  double whiten_tol;     /* whiten when ||S_k^T S_k - I||_F exceeds this, default 1e-12 */
  void* stream;          /* hipStream_t, NULL = default stream */
  double resid_tol;      /* > 0: also stop once every pair's FP64 residual
                            ||A x - lambda x|| / (||A||_1 ||x||) is verified on the
                            device to be <= resid_tol (checked only when the
                            estimates predict it; after a failed check, when they
                            do so scaled by the true/estimated ratio seen there,
                            or have halved); default 0 = off */
  int32_t refine;        /* V32 and VBF16 bases only: 1 = after the low-precision
                            phase reaches refine_tol, continue in FP64 from a
                            combination of its Schur vectors; default 1 */
  double refine_tol;     /* verified-residual target of the low-precision phase
                            (it also stops when its estimates reach it);
                            0 = 1e-6 for an FP32 basis, 1e-3 for BF16 */
  int32_t spmv_layout;   /* rks_spmv_layout, default AUTO */
  int32_t method;        /* rks_method, default RKS */
  int32_t keep;          /* restart size: Schur vectors kept at each contraction,
                            k <= keep <= min(m - 2, 127) (keep + 1 when a conjugate
                            pair would be split); 0 = k, the truncation of
                            Algorithm 1; RKS_KEEP_AUTO (-1) = k + (m - k) / 4,
                            clamped to that range.  Any leading truncation of an
                            rKS decomposition is again one (Section 3.1), so
                            keeping the keep most wanted vectors instead of k is
                            valid; convergence, locking and the returned pairs
                            still concern only the leading k (k + 1 for a pair).
                            Default 0. */
  int32_t graphs;        /* 1: an extension (all Arnoldi steps of one restart
                            cycle) whose start column, pending column and basis
                            precision occurred before is recorded once as a HIP
                            graph on a private stream and then replayed on the
                            solver's stream (same kernels, same arguments, same
                            results to the last bit); 0: launch every kernel.
                            Not used when profile > 0 or for deterministic KS.
                            Default 0: on the measured workloads the host stays
                            ahead of the GPU, so replays save no time; they
                            save host launch work. */
  int32_t stall_restarts; /* S > 0: stop (RKS_ENOTCONV, stop_reason 3) when the largest
                            estimate |b^T y| / |lambda| has not fallen below half of its
                            level S restarts earlier (stagnation, as on operators whose
                            wanted eigenvalues are packed together); 0 = off (default) */
  int32_t a_values;      /* rks_a_values: storage of A's values for the FP64 product,
                            default AUTO (value-indexed when A has at most 256
                            distinct values) */
} rks_opts;

/* Fills *o with the defaults listed above. */
void rks_opts_default(rks_opts* o);

/* Per-solve statistics (filled by rks_solve when st != NULL). */
typedef struct {
  int32_t converged;     /* 1 if every estimate <= tol */
  int32_t restarts;      /* contraction/extension cycles performed */
  int64_t matvecs;       /* products with A */
  int32_t locked;        /* locked (deflated) leading Schur vectors at exit */
  int32_t keff;          /* effective number of pairs (k or k+1, Section 3.1) */
  int32_t whitenings;    /* whitening steps applied */
  int32_t breakdowns;    /* invariant subspaces met and continued past (Section 2.1) */
  int32_t dense_fail;    /* reorderings that had to stop early */
  double max_est;        /* max |b^T y| / |lambda| at exit (eq. "rks_reserror_bound") */
  int32_t stop_reason;   /* 0 restart cap, 1 estimates <= tol, 2 verified residuals <= resid_tol,
                            3 stagnation (opts.stall_restarts) */
  int32_t resid_checks;  /* device residual verifications performed */
  double max_resid;      /* largest verified residual at exit (0 if never verified) */
  int32_t restarts_lo;   /* restarts of the low-precision phase (mixed precision) */
  int32_t refined;       /* 1 if an FP64 refinement phase ran */
  double t_lo;           /* seconds of the low-precision phase */
  double max_resid_lo;   /* largest FP64 residual verified at the end of the low-precision phase */
  double t_total;        /* seconds, host wall clock of the solve */
  double t_host;         /* seconds spent in the host small dense steps */
  /* kernel timings (only when opts.profile > 0), seconds summed over the timed launches */
  double t_spmv, t_reduce, t_ls, t_update, t_rotate;  /* the randomized step runs its least squares
                                                          inside the update launch, so t_update
                                                          covers both and t_ls stays 0 there */
  int64_t n_spmv, n_update, n_rotate;     /* launches */
  double bytes_spmv, bytes_update, bytes_rotate;  /* algorithmic HBM bytes moved, all launches */
  int64_t n_timed_steps, n_timed_rotate;  /* Arnoldi steps timed per kernel, and rotations */
  double bytes_timed_spmv, bytes_timed_update, bytes_timed_rotate;  /* algorithmic bytes of the timed launches */
  int64_t n_timed_whole;     /* sampled Arnoldi steps timed as a whole (the other half of the sample) */
  double t_step;             /* seconds summed over those steps (one event pair around each) */
  double bytes_timed_whole;  /* their algorithmic bytes (SpMV + update) */
  int32_t spmv_layout;       /* rks_spmv_layout in use (ROWS or COLUMN_BLOCKS) */
  int32_t keep;              /* restart size in use */
  double hist_est[512];  /* max estimate after contraction r (r < 512) */
  int32_t a_distinct;    /* distinct values of A in the value table of the FP64
                            product (value-indexed storage), 0 when it reads
                            FP64 values */
} rks_stats;

/* Create a solver for k eigenpairs of A with Krylov dimension m and sketch
 * size d, targeting `which`, with tolerance tol on the estimates
 * |b^T y| / |lambda| (Section 4.1).  Requires 1 <= k, k + 2 <= m <= 255,
 * m + 1 <= d <= min(n, 1024) (Omega must embed the (m+1)-dimensional Krylov
 * space, Algorithm 1 input), k + 1 <= 128 and keep + 1 <= 128 (the
 * rotation writes at most 128 columns), tol > 0, a valid CSR.  opts may be
 * NULL (defaults).
 * Allocates the basis U (n x (m+1)), the sketch S (d x (m+1)), the Rayleigh
 * quotient B ((m+1) x m) and scratch on the device.
 * Errors: RKS_EINVAL, RKS_ENAN (non-finite value in A), RKS_ENOMEM, RKS_EHIP. */
int rks_create(const rks_csr* A, int32_t k, int32_t m, int32_t d, int32_t which, double tol,
               const rks_opts* opts, struct rks_ctx** out);

/* Run Algorithm 1 from the start vector u0 (n FP64 values, host or device
 * per u0_on_device; NULL = the seeded N(0,1) start), scaled so that
 * ||Omega u1|| = 1.  Stops when every estimate is <= tol (the paper's test,
 * Section 5), when opts.resid_tol > 0 and every FP64 residual is verified to
 * be <= resid_tol, or after max_restarts cycles (RKS_ENOTCONV).  Synchronises
 * with the host once per restart.
 * An exact invariant subspace (a vanishing remainder in the extension,
 * Section 2.1) is continued past: the column is replaced by a seeded random
 * vector sketch-orthogonalised against the basis, with a zero subdiagonal
 * entry in B, so the exact pairs stay in the decomposition; RKS_EBREAKDOWN
 * only when that fails (the product with A of the replacement vanishes too,
 * as for the zero operator).  Deterministic Krylov-Schur does not continue.
 * Errors: RKS_EINVAL, RKS_ENAN, RKS_EBREAKDOWN, RKS_EDENSE, RKS_EHIP. */
int rks_solve(struct rks_ctx* ctx, const double* u0, int32_t u0_on_device, rks_stats* st);

/* Number of pairs rks_eigpairs returns (k, or k+1 to keep a conjugate pair). */
int32_t rks_num_pairs(const struct rks_ctx* ctx);

/* Eigenpairs after rks_solve, sorted by `which`: lam_re/lam_im[keff] (host),
 * X (n x keff, column-major; real Ritz vectors of unit 2-norm, a conjugate
 * pair packed as real part then imaginary part of the member with positive
 * imaginary part, that complex vector of unit 2-norm; NULL to skip),
 * resid[keff] (host, NULL to skip) with
 * resid = ||A x - lambda x||_2 / (||A||_1 ||x||_2) computed in FP64 on the
 * device (eq. "RitzError" side).  X_on_device selects where X lives.
 * Errors: RKS_ESTATE before a solve, RKS_EHIP. */
int rks_eigpairs(struct rks_ctx* ctx, double* lam_re, double* lam_im, double* X,
                 int32_t X_on_device, double* resid);

/* Free everything the context owns.  NULL is ignored. */
void rks_destroy(struct rks_ctx* ctx);

/* Static description of an error code. */
const char* rks_strerror(int code);

/* Description of the last failure on ctx (empty string if none). */
const char* rks_last_error(const struct rks_ctx* ctx);

/* ---- lower-level entry points (kernel-level checks and tools) ----------
 * They run single steps of the hot path on the context's matrix and sketch. */

/* z = Omega x for a device FP64 vector x (n) -> device z (d). */
int rks_sketch(struct rks_ctx* ctx, const double* x_dev, double* z_dev);

/* z = Omega x as rks_sketch, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context; the embedding is given by d, sketch_kind, zeta and
 * sketch_seed as in rks_opts, x (n FP64) and z (d FP64) are device buffers
 * of the caller, and the work is enqueued on `stream` (hipStream_t, NULL =
 * default) without synchronising it.  The call allocates nothing: its
 * partial sums go to a fixed device array of the library (512 x 1024 FP64,
 * 4 MiB per GPU, held until the process ends), so d <= 1024.  Every call on
 * one GPU uses that one array: calls in stream order are fine, calls that
 * overlap on one GPU (other streams, other host threads) race.  Results are
 * those of rks_sketch on a context with the same embedding, to the bit.
 * Errors (rks_last_error(NULL) describes them): RKS_EINVAL (NULL pointer,
 * n < 1, d outside 1..1024, sketch_kind, zeta outside 1..min(8, d)),
 * RKS_EHIP. */
int rks_sketch_noalloc(int64_t n, int32_t d, int32_t sketch_kind, int32_t zeta, uint64_t sketch_seed,
                       const double* x_dev, double* z_dev, void* stream);

/* w = A x and z = Omega w (Algorithm 2, apply A and sketch) for device FP64
 * x (n) -> device w (n), device z (d); the fused SpMV + sketch kernel. */
int rks_spmv_sketch(struct rks_ctx* ctx, const double* x_dev, double* w_dev, double* z_dev);

/* Start from u0 (as in rks_solve) and run Algorithm 2 from one to m+1 basis
 * columns, leaving the extended sketch-orthonormal Krylov decomposition
 * A U_m = U_{m+1} B in the context (no contraction); breakdowns are
 * continued past as in rks_solve. */
int rks_arnoldi(struct rks_ctx* ctx, const double* u0, int32_t u0_on_device);

/* Copy the current decomposition to the host: *ncols basis columns
 * (j + 1), B ((m+1) x m, leading dimension m+1), S (d x (m+1), leading
 * dimension d), U (n x (m+1), leading dimension n, normalised FP64 values;
 * may be NULL).  Any output may be NULL. */
int rks_get_state(struct rks_ctx* ctx, int32_t* ncols, double* B, double* S, double* U);

/* Restart rotation U[:, out0:out0+kout] <- U[:, in0:in0+min] * Y on the
 * device basis (Algorithm 1, truncation line), with Y (min x kout, host,
 * column-major), kout <= 128.  Output columns may overlap input columns. */
int rks_rotate(struct rks_ctx* ctx, int32_t in0, int32_t min, int32_t out0, int32_t kout,
               const double* Y);

/* Bandwidth reference: copies nbytes (multiple of 16) from src to dst
 * (device) iters times with a plain streaming kernel and returns the
 * achieved GB/s (bytes read + written) in *gbs. */
int rks_copy_probe(const void* src, void* dst, int64_t nbytes, int32_t iters, double* gbs, void* stream);

/* Bandwidth reference for read-dominated kernels: streams nbytes (multiple
 * of 16) of src (device, only read) iters times and returns the achieved
 * GB/s (bytes read) in *gbs. */
int rks_read_probe(const void* src, int64_t nbytes, int32_t iters, double* gbs, void* stream);

/* Host small dense FP64 helpers used by the contraction step (no device
 * work): real Schur form of A (n x n, in place, lda = n) with Schur vectors
 * Z; reordering of the `which`-wanted kw eigenvalues to the front
 * (*p = kw or kw+1).  Return 0 on success. */
int rks_host_schur(int32_t n, double* A, double* Z);
int rks_host_order(int32_t n, double* T, double* Z, int32_t which, int32_t kw, int32_t* p);

/* ---- learned start (FP32 network kernels, device pointers, stream may be NULL) ----
 * The start vector u1 of Algorithm 1 is a free input (Section 2.1 takes it
 * random).  These entry points train and run a small network that proposes
 * it from the operator's coarse velocity field.  Tensors are row-major:
 * activations B x C x H x W, weights O x C x 3 x 3.  Return RKS_OK,
 * RKS_EINVAL (bad sizes or NULL) or RKS_EHIP. */

/* y = conv3x3(x; w, b, dilation dil), zero padding, optional ReLU. */
int rks_net_conv3x3_forward(const float* x, const float* w, const float* b, float* y, int32_t B, int32_t Cin,
                            int32_t Cout, int32_t H, int32_t W, int32_t dil, int32_t relu, void* stream);

/* Gradients of a layer: dy is the gradient at the layer output y (masked by
 * y > 0 when relu), giving dw, db and, if dx != NULL, the input gradient. */
int rks_net_conv3x3_backward(const float* x, const float* w, const float* y, const float* dy, float* dx, float* dw,
                             float* db, int32_t B, int32_t Cin, int32_t Cout, int32_t H, int32_t W, int32_t dil,
                             int32_t relu, void* stream);

/* loss[b] = 1 - ||V_b^T u_b||^2 / ||u_b||^2 (V_b: P x K orthonormal, K <= 32)
 * and du = gradient of the batch mean of loss with respect to u. */
int rks_net_subspace_loss(const float* u, const float* V, float* loss, float* du, int32_t B, int32_t P, int32_t K,
                          void* stream);

/* One Adam step (bias-corrected, step index t >= 1) on n parameters. */
int rks_net_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int32_t t, void* stream);

/* Bilinear resampling (half-pixel centres) of u (h x w, FP32) to out (H x W, FP64). */
int rks_net_upsample(const float* u, int32_t h, int32_t w, double* out, int32_t H, int32_t W, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RKS_H */
