/*
 * rnmf.h -- randomized HALS for nonnegative matrix factorisation on AMD
 * MI355X (gfx950).  C ABI of librnmf.so.
 *
 * Method: N. B. Erichson, A. Mendible, S. Wihlborn, J. N. Kutz,
 * "Randomized Nonnegative Matrix Factorization", arXiv:1711.02037.
 *   X (m x n, X >= 0) ~ W H with W (m x k) >= 0 and H (k x n) >= 0,
 *   minimising ||X - W H||_F^2 (Sec. 2.2, Eq. nmf_opt).
 *   rnmf_sketch    : randomized range finder, Sec. 2.3 and Algorithm 1
 *                    (sketch X Omega, q subspace iterations, QR).
 *   rnmf_compress  : B = Q^T X, Sec. 2.3 and Algorithm 1.
 *   rnmf_hals_step : compressed HALS sweeps, Sec. 3.2 and Algorithm 1, with
 *                    the projected-gradient stop of Sec. 3.3.
 *   rnmf_factorize : all of Algorithm 1 plus the relative error of Sec. 4.
 *   rnmf_hals      : deterministic HALS sweeps on X itself (Sec. 3.1), the
 *                    baseline that randomized HALS accelerates.
 *
 * Conventions (every entry point):
 *   - Matrices are dense and row-major.  X has a leading dimension ldx >= n
 *     (elements); every other matrix is packed (leading dimension = columns).
 *   - Every array pointer is DEVICE memory owned by the caller.  The library
 *     never allocates device memory: scratch space is the caller's workspace
 *     `ws` of at least rnmf_workspace_bytes(...) bytes, 256-byte aligned.
 *     The workspace may be reused between calls once the previous call's work
 *     on the stream has finished (stream order guarantees this).
 *   - `stream` is a hipStream_t (cast to void*); NULL means the default
 *     stream.  Every call only enqueues work on it, except rnmf_factorize,
 *     which synchronises the stream to fill its report.
 *   - Argument and shape errors are detected on the host before anything is
 *     enqueued and return an error status; rnmf_last_error() then gives a
 *     message (thread-local).  No function throws, exits or aborts.
 *   - Conditions found on the device (non-finite or negative input, Cholesky
 *     breakdown, a sweep that hit its spin limit) are written to a status word
 *     at the start of the workspace, which every entry point clears when it
 *     starts; rnmf_factorize reports them, and rnmf_read_status() fetches them
 *     after an asynchronous call.
 *   - Dtypes: in RNMF_PREC_F64 every array is double; in RNMF_PREC_F32 and
 *     RNMF_PREC_BF16 every array is float, except X, which may also be given
 *     as bfloat16 (RNMF_BF16) for RNMF_PREC_BF16.
 */
#ifndef RNMF_H
#define RNMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rnmf_status {
  RNMF_OK = 0,
  RNMF_ERR_ARG = 1,            /* invalid scalar argument (k, p, q, flags ...)   */
  RNMF_ERR_SHAPE = 2,          /* inconsistent or unsupported shape              */
  RNMF_ERR_DTYPE = 3,          /* dtype not valid for the precision mode         */
  RNMF_ERR_WORKSPACE = 4,      /* workspace NULL, too small or misaligned        */
  RNMF_ERR_NONFINITE = 5,      /* NaN or Inf found in X or produced on device    */
  RNMF_ERR_NEGATIVE_INPUT = 6, /* X has a negative entry (NMF needs X >= 0)      */
  RNMF_ERR_NOT_SPD = 7,        /* Cholesky QR broke down even after the shift    */
  RNMF_ERR_HIP = 8,            /* a HIP runtime call or kernel launch failed     */
  RNMF_ERR_DEVICE_TIMEOUT = 9, /* a device-wide wait hit its spin limit          */
  RNMF_NOT_CONVERGED = 10      /* informational: tol > 0 and max_iter was hit    */
} rnmf_status;

typedef enum rnmf_dtype { RNMF_F64 = 0, RNMF_F32 = 1, RNMF_BF16 = 2 } rnmf_dtype;

/* Arithmetic of the passes over X.  F64 and F32 compute in that type.  BF16
 * stores X as bfloat16 (cast once, round to nearest even) and runs the X
 * passes on bf16 matrix cores with FP32 accumulation.  In the compression
 * B = Q^T X the small operand Q is split into two bfloat16 terms, so only X
 * is rounded; in the passes that only steer the subspace (Y = X Omega,
 * Z = X^T Q and Y = X Z of the subspace iterations) the operand is rounded
 * to bfloat16 too.
 * The orthonormalisation (Gram and Cholesky in FP64), the sweeps (FP32) and
 * the final error (FP64 accumulation) are the same as in F32. */
typedef enum rnmf_prec { RNMF_PREC_F64 = 0, RNMF_PREC_F32 = 1, RNMF_PREC_BF16 = 2 } rnmf_prec;

/* Gram matrix used by the H update (Sec. 3.2).  FULL: S = W^T W for both the
 * numerator and the scale, as in Algorithm 1 (default).  LOWDIM: S = W~^T W~
 * for both, as in the printed rHALS H rule.  MIXED: W~^T W~ in the numerator
 * with (W^T W)_jj as the scale, as the note after that rule suggests. */
enum { RNMF_GRAM_FULL = 0, RNMF_GRAM_LOWDIM = 1, RNMF_GRAM_MIXED = 2 };
/* Block order inside a sweep (Sec. 3.2, cyclic orders): H_FIRST updates all
 * rows of H and then all columns of W, as Algorithm 1 (default); W_FIRST is the
 * other blocked order. */
enum { RNMF_ORDER_H_FIRST = 0, RNMF_ORDER_W_FIRST = 1 };
/* Test matrix distribution when Omega is generated (Sec. 2.3 / Remark on the
 * random test matrix): standard normal (default) or uniform on [0, 1).
 * GAUSS_CLIPPED (standard normal with the negative entries set to zero) is the
 * distribution of the Gaussian start (RNMF_FLAG_GAUSS_INIT); rnmf_random takes
 * all three. */
enum { RNMF_OMEGA_GAUSSIAN = 0, RNMF_OMEGA_UNIFORM = 1, RNMF_DIST_GAUSS_CLIPPED = 2 };

/* opts.flags */
#define RNMF_FLAG_CHECK_INPUT 0x1u      /* scan X for NaN/Inf/negative values  */
#define RNMF_FLAG_NO_SHIFT 0x2u         /* no shifted Cholesky QR fallback     */
#define RNMF_FLAG_EXACT_Q 0x4u          /* BF16: do not add one power iteration */
#define RNMF_FLAG_TRACE 0x8u            /* rnmf_hals_step: record phase timestamps */
#define RNMF_FLAG_SVD_INIT 0x20u        /* rnmf_factorize: W0, H0 by the SVD-based
                                           initialization (rnmf_svd_init)      */
#define RNMF_FLAG_GAUSS_INIT 0x40u       /* rnmf_factorize: W0, H0 drawn from the seed
                                           as standard normal entries with the
                                           negative ones set to zero (the Remark
                                           on initialization after Algorithm 1),
                                           instead of uniform on [0, 1)          */
#define RNMF_FLAG_SHIFTED_QR3 0x10u     /* every QR: shifted Cholesky QR pass first, then
                                           two plain passes (shifted CholeskyQR3)   */

/* Regularization (Sec. 3.4 and its appendix): the cost becomes
 *   1/2 ||X - W H||_F^2 + alpha_w/2 ||W||_F^2 + beta_w sum(W)
 *                       + alpha_h/2 ||H||_F^2 + beta_h sum(H),
 * whose exact block minimisers are the printed rules: the ridge weight alpha
 * is added to the scale (S_jj + alpha_h for a row of H, V_jj + alpha_w for a
 * column of W) and the LASSO weight beta is subtracted from the cross product;
 * both nonzero is the elastic net.  In the compressed sweep the ridge part acts
 * on W~ and the LASSO shift beta_w / (V_jj + alpha_w) is subtracted from the
 * lifted column Q W~(:,j) before the clip.  The stop test uses the gradient of
 * this cost.  All four zero (the default) is plain HALS, bit for bit. */
typedef struct rnmf_opts {
  int32_t k;          /* target rank, 1 <= k < min(m, n)                        */
  int32_t p;          /* oversampling (paper default 20); l = min(k+p, m, n)    */
  int32_t q;          /* subspace iterations (paper default 2); BF16 adds one    */
  int32_t max_iter;   /* sweep cap                                               */
  double tol;         /* projected-gradient ratio tolerance; <= 0: run max_iter */
  uint64_t seed;      /* Philox key for Omega / W0 / H0 when they are NULL       */
  int32_t prec;       /* rnmf_prec                                               */
  int32_t omega_dist; /* RNMF_OMEGA_*                                            */
  int32_t gram_mode;  /* RNMF_GRAM_*                                             */
  int32_t order;      /* RNMF_ORDER_*                                            */
  uint32_t flags;     /* RNMF_FLAG_*                                             */
  int32_t reserved;   /* must be 0                                               */
  double alpha_w;     /* ridge weight on W, >= 0 (0: none)                       */
  double alpha_h;     /* ridge weight on H, >= 0                                 */
  double beta_w;      /* LASSO weight on W, >= 0 (0: none)                       */
  double beta_h;      /* LASSO weight on H, >= 0                                 */
} rnmf_opts;

typedef struct rnmf_report {
  int32_t iters;      /* sweeps performed                                        */
  int32_t l_eff;      /* sketch width actually used                              */
  int32_t q_eff;      /* subspace iterations actually used                       */
  int32_t qr_path;    /* bit0: a shifted Cholesky QR pass was needed             */
  int32_t status;     /* rnmf_status of the run                                  */
  int32_t reserved;
  double rel_err;     /* ||X - W H||_F / ||X||_F, FP64 accumulation              */
  double pg_ratio;    /* ||grad^P||^2 at the end / at the start (on Q B)         */
  double ms_qb;       /* stream time of cast, sketch, compression and init (ms)  */
  double ms_sweeps;   /* stream time of the sweep launch (ms)                    */
  double ms_error;    /* stream time of the final error (ms)                     */
  double comp_err;    /* ||B - W~ H||_F / ||B||_F on the compressed data, FP64   */
                      /* accumulation (the error the sweeps minimise, Sec. 3.2)  */
} rnmf_report;

/* Operation selector for rnmf_workspace_bytes. */
enum { RNMF_OP_SKETCH = 0, RNMF_OP_COMPRESS = 1, RNMF_OP_HALS_STEP = 2,
       RNMF_OP_FACTORIZE = 3, RNMF_OP_REL_ERROR = 4, RNMF_OP_HALS = 5,
       RNMF_OP_SVD_INIT = 6 };

/* Fills opts with the paper's defaults: p = 20, q = 2 (Sec. 4, experimental
 * setup), max_iter = 200, tol = 0, prec F32, Gaussian Omega, FULL Gram,
 * H-first order, CHECK_INPUT set.  k is left 0 and must be set. */
void rnmf_default_opts(rnmf_opts* opts);

/* Bytes of workspace the operation needs for an m x n input (for
 * RNMF_OP_HALS_STEP, m and n are the sizes of W's rows and H's columns).
 * Returns 0 if the arguments are invalid (rnmf_last_error() says why). */
size_t rnmf_workspace_bytes(int op, int64_t m, int64_t n, const rnmf_opts* opts);

/* Static string for a status code (never NULL). */
const char* rnmf_status_string(int status);

/* Message for the last error returned on this thread ("" if none). */
const char* rnmf_last_error(void);

/* Sketch width used for (k, p, m, n): min(k + p, m, n). */
int32_t rnmf_sketch_width(int32_t k, int32_t p, int64_t m, int64_t n);

/* Randomized range finder (Sec. 2.3; Algorithm 1 up to the final QR):
 *   Y = X Omega; q times { Q = qr(Y); Q = qr(X^T Q); Y = X Q }; Q = qr(Y).
 * X: m x n (ldx), dtype xt.  Omega: n x l test matrix in the factor dtype, or
 * NULL to draw it from opts->seed (Philox4x32-10; normal by Box-Muller or
 * uniform).  Q (out): m x l, orthonormal columns; qr is Cholesky QR repeated
 * twice with the Gram and Cholesky factor in FP64, which yields the thin QR
 * with positive diag(R); a shifted pass is prepended if the Gram is not
 * numerically positive definite (unless RNMF_FLAG_NO_SHIFT).
 * l_out (host, may be NULL) receives l.  Asynchronous. */
rnmf_status rnmf_sketch(const void* X, int xt, int64_t m, int64_t n, int64_t ldx,
                        const void* Omega, const rnmf_opts* opts, void* Q,
                        int32_t* l_out, void* ws, size_t ws_bytes, void* stream);

/* Compression B = Q^T X (Sec. 2.3; Algorithm 1).  Q: m x l; B (out): l x n.
 * Any n >= 1 is accepted (with X = W0 it also forms W~ = Q^T W0).  Only
 * opts->prec is read.  The workspace query for RNMF_OP_COMPRESS sizes
 * l = min(k + p, m).  Asynchronous. */
rnmf_status rnmf_compress(const void* X, int xt, int64_t m, int64_t n, int64_t ldx,
                          const void* Q, int32_t l, const rnmf_opts* opts, void* B,
                          void* ws, size_t ws_bytes, void* stream);

/* nsweeps sweeps of compressed HALS (Sec. 3.2; Algorithm 1), in place:
 *   H phase: R = B^T W~, S (see gram_mode), rows j of H in turn:
 *            H(j,:) <- max(0, H(j,:) + (R(:,j) - H^T S(:,j)) / S_jj)
 *   W phase: T = B H^T, V = H H^T, columns j of W in turn:
 *            W~(:,j) <- W~(:,j) + (T(:,j) - W~ V(:,j)) / V_jj
 *            W(:,j)  <- max(0, Q W~(:,j));  W~(:,j) <- Q^T W(:,j)
 * A block whose scale S_jj or V_jj is exactly zero is skipped.
 * Q: m x l; B: l x n; W: m x k (in/out); Wt: l x k (in/out, the compressed
 * factor W~, normally Q^T W); H: k x n (in/out).  If opts->tol > 0 the sweeps
 * stop once ||grad^P f||^2 on Q B falls below tol times its value at entry
 * (Sec. 3.3).  dev_stats (device, optional): 3 doubles = {sweeps done,
 * ||grad^P||^2 at entry, at exit}; the device status word stays in ws
 * (rnmf_read_status).  Requires k <= 64 and
 * l <= 128.  With RNMF_FLAG_TRACE, workgroup 0 writes 10 + 2k timestamps of
 * the device's 100 MHz real-time counter for the first sweep (entry, Q slab
 * loaded, prologue, H phase, T/V exchange, each W column before and after its
 * exchange, W phase, local S, S exchange, sweep end, kernel end) as uint64 at
 * byte offset 1024 of ws; entries 120 to 125 mark steps inside the phases for
 * the register-slab kernel: 120 the end of the local T/V products (before
 * their exchange), 124 and 125 the start and end of their arithmetic; 121,
 * 122 and 123 the H phase of wavefront 0 after R = B^T W~, after the S terms
 * and after the row updates.  Asynchronous. */
/* Launch plan of rnmf_hals_step for this shape on the current device (host
 * only; nothing is launched).  out: 8 int32 = {workgroups, W rows per
 * workgroup, H columns per workgroup, 1 if the Q slab is held in registers,
 * 1 if (with the register slab) the W rows stay in global memory instead of
 * LDS, dedicated exchange-owner workgroups, LDS bytes per workgroup, rows of
 * Q staged in LDS (LDS-slab path)}.  opts: prec and tol are used.  Errors:
 * RNMF_ERR_ARG / ERR_SHAPE for bad arguments, RNMF_ERR_HIP without a device. */
rnmf_status rnmf_sweep_plan(int64_t m, int64_t n, int32_t l, int32_t k, const rnmf_opts* opts, int32_t* out);

rnmf_status rnmf_hals_step(const void* Q, const void* B, int64_t m, int64_t n,
                           int32_t l, int32_t k, void* W, void* Wt, void* H,
                           int32_t nsweeps, const rnmf_opts* opts, double* dev_stats,
                           void* ws, size_t ws_bytes, void* stream);

/* rnmf_hals_step without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  It runs the same sweep kernel; its scratch memory (the
 * status word, the statistics and the exchange buffers) is a fixed array of
 * RNMF_NOALLOC_SCRATCH_BYTES in the library's device code, one per GPU, held
 * until the process ends.  The call allocates nothing: no hipMalloc, no
 * hipFree, no allocating library routine.  Arguments as for rnmf_hals_step,
 * plus dev_status (device, optional): one uint32 that receives the device
 * status bits of the sweeps (0 = fine; nonzero: rnmf_status_string of
 * rnmf_read_status's mapping - a non-finite value or a wait that hit its spin
 * limit); dev_stats as for rnmf_hals_step.  RNMF_FLAG_TRACE is rejected (the
 * trace would land in the hidden scratch).  The scratch holds 4 KiB plus the
 * sweep's exchange buffers, which at 256 workgroups take
 * 8 (262,144 + 512 c + 2,048 ceil(c / 16)) bytes for c = l k + k^2: any
 * c <= 7,781 fits (k = 50 with l <= 105, k = 64 with l <= 57; k = 50, l = 70
 * takes 32.8 MB).  A larger problem returns RNMF_ERR_WORKSPACE before any
 * launch, naming the bytes it needs.  Every call on
 * one GPU shares that GPU's scratch: calls that overlap in time on one GPU
 * (on different streams or host threads) race and must be serialised by the
 * caller.  Each call clears what must start at zero.  Asynchronous. */
#define RNMF_NOALLOC_SCRATCH_BYTES (40u << 20)
rnmf_status rnmf_hals_step_noalloc(const void* Q, const void* B, int64_t m, int64_t n,
                                   int32_t l, int32_t k, void* W, void* Wt, void* H,
                                   int32_t nsweeps, const rnmf_opts* opts, double* dev_stats,
                                   uint32_t* dev_status, void* stream);

/* Relative error ||X - W H||_F / ||X||_F (reading of the "error" of Sec. 4),
 * with FP64 accumulation.  W: m x k, H: k x n in the factor dtype.  out
 * (device): 2 doubles = {||X - W H||_F^2, ||X||_F^2}.  Asynchronous. */
rnmf_status rnmf_rel_error(const void* X, int xt, int64_t m, int64_t n, int64_t ldx,
                           const void* W, const void* H, int32_t k, const rnmf_opts* opts,
                           double* out, void* ws, size_t ws_bytes, void* stream);

/* Algorithm 1 end to end: sketch, compression, W~ = Q^T W0, sweeps until the
 * stop test or max_iter, then the relative error.  Omega (n x l), W0 (m x k),
 * H0 (k x n) are optional device inputs in the factor dtype; NULL draws them
 * from opts->seed (W0, H0 uniform on [0, 1), or clipped standard normal with
 * RNMF_FLAG_GAUSS_INIT); with RNMF_FLAG_SVD_INIT, W0 and
 * H0 must be NULL and come from rnmf_svd_init on this call's Q and B (needs
 * l <= 96).  W (out, m x k), H (out, k x n).
 * report (host, may be NULL) is filled after the stream is synchronised.
 * Returns the run's status (RNMF_NOT_CONVERGED only when tol > 0). */
rnmf_status rnmf_factorize(const void* X, int xt, int64_t m, int64_t n, int64_t ldx,
                           const rnmf_opts* opts, const void* Omega, const void* W0,
                           const void* H0, void* W, void* H, rnmf_report* report,
                           void* ws, size_t ws_bytes, void* stream);

/* SVD-based initialization (the Remark on initialization after Algorithm 1):
 * the nonnegative double SVD of Boutsidis and Gallopoulos (2008) of the k
 * leading singular triplets of the randomized SVD from the QB decomposition
 * (Sec. 2.3): B = U_B S V^T, U = Q U_B.  Component 1 is sqrt(s_1) |u_1|,
 * sqrt(s_1) |v_1|; component j > 1 keeps the positive parts of (u_j, v_j) if
 * ||u+|| ||v+|| > ||u-|| ||v-||, else the negative parts, scaled so that the
 * product of its two factors is s_j times the larger product; a component
 * whose two products vanish is zero.  The SVD of B comes from FP64 Jacobi on
 * B B^T.
 * Q: m x l orthonormal, B: l x n, both packed, in the factor dtype of
 * opts->prec (RNMF_F64 for RNMF_PREC_F64, else RNMF_F32); 1 <= k <= min(l, 64),
 * l <= 96, k = opts->k.  W (out, m x k) and H (out, k x n), packed.
 * Workspace: RNMF_OP_SVD_INIT.  Asynchronous; no device status is set. */
rnmf_status rnmf_svd_init(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k,
                          void* W, void* H, const rnmf_opts* opts, void* ws, size_t ws_bytes,
                          void* stream);

/* ---- Sweeps with an explicit order of block updates --------------------------
 * Sec. 3.2 allows different orders of the block updates: the interleaved
 * cyclic order W(:,1) -> H(1,:) -> ... -> W(:,k) -> H(k,:), the blocked
 * orders (all columns of W, then all rows of H, or the reverse), and a
 * shuffled order that takes the components in a random order per sweep.
 * This entry point runs nsweeps compressed-HALS sweeps (plain rules,
 * S = W^T W) on W, Wt, H in place, with the block updates of sweep s in the
 * order order[s*2k .. s*2k + 2k - 1]: entry e < k updates column e of W
 * (update, lift, clip and map-back), entry e >= k updates row e - k of H.
 * Every block update takes the products of the factors as they are at that
 * moment.  Each sweep's list must be a permutation of 0..2k-1
 * (RNMF_ERR_ARG otherwise); order is host memory (nsweeps*2k int32), drawn
 * by the caller for a shuffled order.  Blocks with a zero scale are skipped.
 * Arguments as for rnmf_hals_step; gram_mode must be RNMF_GRAM_FULL and the
 * regularization weights zero.  A few launches per block update: the
 * blocked orders run much faster in rnmf_hals_step.  Workspace:
 * rnmf_hals_ordered_workspace_bytes.  Asynchronous. */
size_t rnmf_hals_ordered_workspace_bytes(int64_t m, int64_t n, int32_t l, int32_t k);
rnmf_status rnmf_hals_ordered(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k, void* W,
                              void* Wt, void* H, int32_t nsweeps, const int32_t* order, const rnmf_opts* opts,
                              void* ws, size_t ws_bytes, void* stream);

/* ---- Reverse mode through unrolled sweeps ---------------------------------
 * T sweeps, one launch each, with every state recorded: the forward that
 * rnmf_backward differentiates without recomputation.  Runs T sweeps of
 * Algorithm 1's sweep (Sec. 3.2) on W, Wt, H in place, exactly as T calls of
 * rnmf_hals_step with nsweeps = 1 (one launch of T sweeps carries sums across
 * sweeps and matches this to rounding only).  If states is not NULL, the
 * state after sweep i (i = 0..T-1) is written at
 *   states + i * (m*k + l*k + k*n) * es,  es = 8 (RNMF_PREC_F64) or 4,
 * as W (m x k), then Wt (l x k), then H (k x n), packed.  Arguments as for
 * rnmf_hals_step; workspace: RNMF_OP_HALS_STEP.  Asynchronous. */
rnmf_status rnmf_unroll(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k, void* W, void* Wt,
                        void* H, int32_t T, void* states, const rnmf_opts* opts, void* ws, size_t ws_bytes,
                        void* stream);

/* Gradients through T compressed-HALS sweeps (Algorithm 1's sweep, Sec. 3.2,
 * S = W^T W, rows of H first, plain rules) with the basis Q held fixed.  The
 * derivative of max(0, x) is taken as 0 at 0; a block whose scale is zero is
 * skipped, as in the forward.  Given the upstream gradients gW_T, gH_T of the
 * sweeps' outputs (W_T, H_T), returns the gradients of
 * <gW_T, W_T> + <gH_T, H_T> with respect to B, W0 (including the path through
 * Wt0 = Q^T W0) and H0, and optionally gX = Q gB (the path of X through
 * B = Q^T X).
 * The states of the forward come either from rnmf_unroll's record (states
 * not NULL, ckpt_every = 0: nothing is recomputed) or are recomputed inside
 * the call (states NULL, ckpt_every >= 1): the sweep kernel runs one sweep
 * per launch from Wt0, a checkpoint is kept every ckpt_every sweeps, and one
 * segment is recomputed at a time.  Either way the gradients describe the
 * one-sweep-per-launch forward of rnmf_unroll.
 * Q (m x l), B (l x n), W0 (m x k), Wt0 (l x k), H0 (k x n): packed, in the
 * factor dtype of opts->prec (RNMF_F64 for RNMF_PREC_F64, else RNMF_F32).
 * gW_T (m x k), gH_T (k x n) in; gB (l x n), gW0 (m x k), gH0 (k x n) and gX
 * (m x n, may be NULL) out; all FP64, packed, device memory.  gW0 may be
 * gW_T and gH0 may be gH_T (updated in place).  Requires gram_mode
 * RNMF_GRAM_FULL, order RNMF_ORDER_H_FIRST and zero regularization weights;
 * 1 <= k <= min(64, l), l <= min(128, m); T >= 0.
 * Workspace: rnmf_backward_workspace_bytes with the same ckpt_every.  A
 * device-wide wait that passes its spin limit sets RNMF_ERR_DEVICE_TIMEOUT in
 * the status word (rnmf_read_status).  Asynchronous. */
size_t rnmf_backward_workspace_bytes(int64_t m, int64_t n, int32_t l, int32_t k, int32_t T, int32_t ckpt_every,
                                     const rnmf_opts* opts);
rnmf_status rnmf_backward(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k,
                          const void* W0, const void* Wt0, const void* H0, int32_t T, int32_t ckpt_every,
                          const void* states, const double* gW_T, const double* gH_T, double* gB, double* gW0,
                          double* gH0, double* gX, const rnmf_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* ---- Batched randomized HALS ------------------------------------------------
 * Many independent problems of uneven shapes (Algorithm 1 for each, with the
 * plain FP32 rules, Gram mode RNMF_GRAM_FULL and order RNMF_ORDER_H_FIRST) in
 * one persistent launch.  Each workgroup takes whole problems from a work
 * queue, largest first, and runs sketch, q subspace iterations with
 * CholeskyQR2, compression, W~ = Q^T W0, nsweeps sweeps and the relative
 * error on its own, so no workgroup ever waits for another.  FP32 storage
 * and arithmetic, FP64 Grams, Cholesky factors and error sums.
 * One problem: all pointers are caller-owned device memory, FP32, row-major
 * and packed except X.  Requirements: 1 <= k <= min(32, l), 1 <= l <= 64,
 * l <= min(m, n); ldx >= n. */
typedef struct rnmf_problem {
  const float* X;      /* m x n, leading dimension ldx                        */
  const float* Omega;  /* n x l test matrix                                   */
  const float* W0;     /* m x k initial W                                     */
  const float* H0;     /* k x n initial H                                     */
  float* W;            /* out: m x k                                          */
  float* H;            /* out: k x n                                          */
  float* Q;            /* out: m x l orthonormal basis                        */
  float* B;            /* out: l x n compressed matrix Q^T X                  */
  float* Z;            /* scratch: n l + k ceil(m / 32) 32 + 32 floats (B^T,
                          n x l, then W held by columns during the sweeps:
                          k columns of m rounded up to 32 floats, from the
                          next 128-byte boundary)                           */
  int64_t m, n, ldx;
  int32_t k, l;
  int32_t prec;        /* RNMF_PREC_F32, or RNMF_PREC_BF16: the passes over X
                          on bf16 matrix cores (X rounded to bfloat16 as it is
                          staged, the small operand split hi + lo, FP32
                          accumulation) with one more subspace iteration     */
  int32_t reserved;    /* must be 0                                           */
} rnmf_problem;

/* Workspace bytes for a batch of nprob problems (descriptors, queue counter,
 * per-problem error sums and status). */
size_t rnmf_batch_workspace_bytes(int32_t nprob);

/* Checks every problem (host array), orders them by estimated cost (largest
 * first), picks each problem's X-pass tiling from the autotune table and
 * copies the descriptors into ws (asynchronous copy on stream; the host array
 * may be reused when the call returns).  Errors: RNMF_ERR_ARG / ERR_SHAPE
 * name the first bad problem in rnmf_last_error(). */
rnmf_status rnmf_batch_plan(const rnmf_problem* probs, int32_t nprob, void* ws, size_t ws_bytes,
                            void* stream);

/* Runs a planned batch: q subspace iterations and nsweeps sweeps per problem.
 * Launches one small fill kernel and the persistent kernel and nothing else
 * (no allocation, no memset, no host synchronisation), so it may be captured
 * in a HIP graph and replayed.  Asynchronous. */
rnmf_status rnmf_batch_run(int32_t nprob, int32_t q, int32_t nsweeps, void* ws, size_t ws_bytes,
                           void* stream);

/* Synchronises stream and copies the results of the last run to host arrays
 * in the caller's problem order: rel_err[i] = ||X - W H||_F / ||X||_F (FP64
 * sums) and status[i] (an rnmf_status; RNMF_OK, RNMF_ERR_NOT_SPD when a
 * Cholesky QR pass failed even with a shift).  Either pointer may be NULL. */
rnmf_status rnmf_batch_results(int32_t nprob, void* ws, size_t ws_bytes, double* rel_err, int32_t* status,
                               void* stream);

/* Tunes the batch per sketch-width class (l <= 16, <= 32, <= 48, <= 64), on
 * that class's own problems: times each X-pass tiling (q subspace
 * iterations and compression, no sweeps), then, with the chosen tiling, each
 * H-phase tile width that fits (64, 128 or 256 columns of B^T staged per
 * tile; 8 sweeps).  Keeps the fastest in the library's autotune table (the
 * only library-global state) and re-plans the batch with it.  tiling_out
 * (host, 8 entries, may be NULL) receives the table: column groups for the
 * four classes, then the H-phase tile widths.  Synchronises the stream. */
rnmf_status rnmf_batch_autotune(const rnmf_problem* probs, int32_t nprob, int32_t q, void* ws,
                                size_t ws_bytes, int32_t* tiling_out, void* stream);

/* The autotune table (8 int32, the layout rnmf_batch_autotune reports):
 * read it, or set it, for instance from an earlier tuning run.  Set checks
 * every entry (column groups 4, 8 or 16; tile widths 64, 128 or 256) and
 * changes nothing on error (RNMF_ERR_ARG).  rnmf_batch_plan uses the table
 * current at its call; a problem whose sketch is wider than an entry allows
 * takes the next wider tiling or narrower tile.  Host only. */
rnmf_status rnmf_batch_set_tuning(const int32_t* table);
rnmf_status rnmf_batch_get_tuning(int32_t* table);

/* nsweeps sweeps of deterministic HALS (Sec. 3.1, residual-free block rules)
 * on X itself, in place; randomized HALS is this algorithm run on the
 * compressed B with the lift through Q:
 *   H phase: R = X^T W, S = W^T W, rows j of H in turn:
 *            H(j,:) <- max(0, H(j,:) + (R(:,j) - H^T S(:,j)) / S_jj)
 *   W phase: T = X H^T, V = H H^T, columns j of W in turn:
 *            W(:,j) <- max(0, W(:,j) + (T(:,j) - W V(:,j)) / V_jj)
 * in the order opts->order; a block whose scale is exactly zero is skipped.
 * X: m x n (ldx) in RNMF_F32 (opts->prec RNMF_PREC_F32) or RNMF_F64
 * (RNMF_PREC_F64); W: m x k and H: k x n (in/out, packed, same dtype).
 * k = opts->k with 1 <= k <= min(64, m, n).  opts->tol must be <= 0 (a fixed
 * number of sweeps); gram_mode is not used.  Each sweep streams X twice
 * (one TN and one NN pass); S and V are formed with FP64 accumulation and
 * both Gauss-Seidel sweeps accumulate in FP64.  Workspace: RNMF_OP_HALS.
 * Asynchronous. */
rnmf_status rnmf_hals(const void* X, int xt, int64_t m, int64_t n, int64_t ldx, void* W, void* H,
                      int32_t nsweeps, const rnmf_opts* opts, void* ws, size_t ws_bytes, void* stream);

/* Cast an m x n FP32 matrix (ldx) to packed bfloat16 (round to nearest even),
 * for callers that keep a BF16 copy of X for RNMF_PREC_BF16.  Asynchronous. */
rnmf_status rnmf_cast_bf16(const float* X, int64_t m, int64_t n, int64_t ldx,
                           void* Xb, void* stream);

/* The library's seeded random matrices (Algorithm 1, step 2, and the Remark on
 * the random test matrix after it): fills `out` (device, rows x cols, packed
 * row-major, RNMF_F64 or RNMF_F32) with the stream that rnmf_sketch and
 * rnmf_factorize draw when a pointer is NULL.  Element e = r * cols + c is
 * computed from one Philox4x32-10 block (Salmon et al., SC 2011) with counter
 * (e mod 2^32, e div 2^32, stream_id, 0x524E4D46) and key (seed mod 2^32,
 * seed div 2^32); with output words (c0, c1, c2, c3) and
 * u(a, b) = ((b << 21) xor (a >> 11)) / 2^53:
 *   RNMF_OMEGA_UNIFORM:      u(c0, c1), in [0, 1);
 *   RNMF_OMEGA_GAUSSIAN:     sqrt(-2 log(u(c0, c1) + 2^-53)) cos(2 pi u(c2, c3))
 *                            (Box-Muller, cosine branch);
 *   RNMF_DIST_GAUSS_CLIPPED: the Gaussian value with negative values set to 0;
 * computed in FP64 and rounded once to the output type.  Stream ids used by
 * the library: 3 Omega, 4 W0, 5 H0.  Asynchronous. */
rnmf_status rnmf_random(void* out, int dt, int64_t rows, int64_t cols, uint64_t seed, uint32_t stream_id,
                        int32_t dist, void* stream);

/* The Philox4x32-10 block function behind rnmf_random, on caller-given inputs
 * (all device arrays): out[4i..4i+3] = philox4x32_10(ctr[4i..4i+3],
 * key[2i..2i+1]) for i < count; ten rounds with multipliers 0xD2511F53 and
 * 0xCD9E8D57 and key increments 0x9E3779B9 and 0xBB67AE85 (Salmon et al.,
 * SC 2011).  It lets a caller reproduce or verify the generator's stream.
 * count = 0 is a no-op.  Asynchronous. */
rnmf_status rnmf_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count,
                               void* stream);

/* Synchronises `stream` and returns the device status word recorded in `ws`
 * by the most recent asynchronous call that used `ws` (each entry point clears
 * the word when it starts), then clears it. */
rnmf_status rnmf_read_status(void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RNMF_H */
