/*
 * ntf.h - C ABI of the MI355X (gfx950) library for nonnegative CP tensor factorization
 * (NTF) by block-coordinate descent with A-HALS block updates, accelerated by heuristic
 * extrapolation with restarts (HER).
 *
 * Method: A. M. S. Ang, J. E. Cohen, L. T. K. Hien, N. Gillis, "Accelerating block
 * coordinate descent for nonnegative tensor factorization", arXiv 2001.04321. Citations
 * below name the paper's sections, equations (by their labels) and algorithms.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Modes are 0-based here (1-based in the paper). 2 <= order <= NTF_MAX_ORDER.
 *  - A tensor is dense and C-contiguous: the last mode is the fastest-varying index. Its
 *    size must stay below 2 GiB (NTF_EUNSUPPORTED otherwise).
 *  - A factor A^(n) is an I_n x r float32 matrix, row-major (row j holds the r entries
 *    a_1^(n)[j] .. a_r^(n)[j] contiguously). 1 <= r <= NTF_MAX_RANK.
 *  - Every data pointer is a DEVICE pointer on the handle's device unless stated
 *    otherwise. Arrays of pointers (`const float* const* A`) are HOST arrays holding
 *    device pointers. The caller allocates and owns all buffers; the library never frees
 *    caller memory. Buffers must stay valid until the enqueued work has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream). All
 *    calls enqueue work asynchronously and return; results are valid after the stream
 *    has been synchronized.
 *  - Errors: a call returns NTF_OK or an error status. On an argument error nothing is
 *    enqueued and no caller buffer is written. C++ exceptions never cross this ABI.
 *    ntf_last_error() returns a thread-local message describing the last error.
 *  - A handle is bound to one device, owns the library's workspace (MTTKRP split
 *    partials, Gram partials, inner-solver synchronization slots, captured graphs) and
 *    is not thread-safe: one host thread at a time, calls on one handle must not overlap
 *    on different streams.
 *  - Kernels report rare runtime conditions (a bounded wait that timed out, a non-finite
 *    objective) in a device-side flag word; read it with ntf_device_flags().
 */
#ifndef NTF_H
#define NTF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NTF_MAX_ORDER 8
#define NTF_MAX_RANK 256

typedef enum ntf_status {
  NTF_OK = 0,
  NTF_EINVAL = 1,         /* invalid argument (null pointer, bad size/mode/rank/dtype) */
  NTF_ENOMEM = 2,         /* device allocation of the handle's workspace failed */
  NTF_EDEVICE = 3,        /* a HIP runtime call failed */
  NTF_EUNSUPPORTED = 4,   /* valid but outside what the kernels implement */
  NTF_ENUMERIC = 5        /* non-finite value where a finite one is required */
} ntf_status;

typedef enum ntf_dtype {
  NTF_F32 = 0,            /* IEEE float32 */
  NTF_BF16 = 1            /* bfloat16 (upper 16 bits of a float32) */
} ntf_dtype;

/* Device flag bits reported by ntf_device_flags(). */
#define NTF_FLAG_WAIT_TIMEOUT 0x1u   /* a cross-workgroup wait gave up; results invalid */
#define NTF_FLAG_NONFINITE 0x2u      /* a restart surrogate F-hat was NaN or infinite */

/* Dense tensor descriptor (paper Sec. 1: T in R^{I_1 x ... x I_N}). */
typedef struct ntf_tensor {
  int32_t order;                 /* N, 2..NTF_MAX_ORDER */
  int32_t dtype;                 /* ntf_dtype of the elements */
  int64_t dims[NTF_MAX_ORDER];   /* I_1..I_N, each >= 1; entries past `order` ignored */
  const void* data;              /* device pointer, C-contiguous, 16-byte aligned */
} ntf_tensor;

typedef struct ntf_handle ntf_handle;

/* Data given in Tucker format (Appendix A): T = (U^(1) (x) ... (x) U^(N)) G with a core G
 * (float32, order N, dims r_1..r_N, C-contiguous device tensor) and bases U^(p) (n_p x r_p
 * float32, row-major device matrices). dims: n_1..n_N, the sizes of T (never formed). */
typedef struct ntf_tucker {
  ntf_tensor core;
  const float* U[NTF_MAX_ORDER];
  int64_t dims[NTF_MAX_ORDER];
} ntf_tucker;

/* HER parameters (Sec. 3.1.4, table of HER parameters; defaults of Sec. 4.1) and the
 * inner stopping rule of Sec. 4.1. Validation: 0 <= beta0 < 1 (beta0 = 0 gives plain
 * Algorithm 1), 1 <= gamma_bar <= gamma <= eta, 1 <= max_inner <= 1000, inner_tol >= 0. */
typedef struct ntf_her_params {
  double beta0;        /* initial extrapolation weight, default 0.5 */
  double gamma;        /* growth rate of beta, default 1.05 */
  double gamma_bar;    /* growth rate of beta_bar, default 1.01 */
  double eta;          /* decay rate of beta, default 1.5 */
  int32_t max_inner;   /* inner steps per block at most (A-HALS sweeps), default 50 */
  int32_t inner_solver; /* block solver: 0 A-HALS (Sec. 2.1.4, default), 1 projected gradient,
                           2 accelerated (Nesterov) projected gradient (Sec. 2.2; the
                           HER-PGD50 / HER-Nesterov50 runs of Sec. 3.1.4: they take exactly
                           max_inner steps and need inner_tol = 0), 3 ADMM (Sec. 2.1.2,
                           HER-ADMM; the stopping rule applies, max_inner <= 64) */
  double inner_tol;    /* stop when ||W_s - W_{s-1}||_F <= inner_tol ||W_1 - W_0||_F, default 1e-2 */
  int32_t scheme;      /* extrapolation between block updates: 0 HER (Algorithm 2, default);
                          1 Bro's sequence in the block-wise form of Sec. 3.3: the same
                          structure (each block extrapolated right after its update, the
                          extrapolated sequence abandoned when F-hat increases) with
                          beta_k = omega_k = k^(1/h) - 1 (0 for k < 5), h = 3 raised by one
                          every fifth increase, and no projection of the extrapolated
                          point; beta0, gamma, gamma_bar and eta are then unused */
  int32_t reserved;    /* 0 */
} ntf_her_params;

/* HER scalar state, kept in DEVICE memory (Algorithm 2: beta_k, beta_bar_k, F-hat_k). */
typedef struct ntf_her_state {
  double beta;         /* extrapolation weight used by the next extrapolation step */
  double beta_bar;     /* upper bound of beta */
  double fhat_prev;    /* F-hat of the last completed iteration (F(A_0) after INIT); a
                          non-finite F-hat restarts and leaves the last finite value here */
  double fhat;         /* F-hat_k of the last DECIDE */
  int64_t k;           /* completed outer iterations since INIT */
  int32_t restart;     /* 1 if the last DECIDE restarted, else 0 */
  int32_t nrestarts;   /* restarts since INIT */
  int64_t it;          /* iterations completed in the current ntf_solve call (trace index) */
} ntf_her_state;

/* Per-iteration record written by ntf_solve (device arrays, each may be NULL; each
 * array has room for `iters` entries, `sweeps` for iters * order). */
typedef struct ntf_trace {
  double* fhat;        /* F-hat_k */
  double* beta;        /* beta after iteration k's update */
  double* beta_bar;    /* beta_bar after iteration k's update */
  int32_t* restart;    /* 1 if iteration k restarted */
  int32_t* sweeps;     /* A-HALS sweeps of block n at iteration k: [k * order + n] */
} ntf_trace;

typedef enum ntf_her_op {
  NTF_HER_INIT = 0,         /* state <- (beta0, beta_bar = 1, fhat_prev = *fhat, k = 0) */
  NTF_HER_EXTRAPOLATE = 1,  /* A_hat[b] <- max(0, A_new[b] + beta (A_new[b] - A[b])) */
  NTF_HER_DECIDE = 2        /* restart test on *fhat, beta update, A[l] <- survivor */
} ntf_her_op;

/* ---------------------------------------------------------------- handle, errors --- */

/* Create a handle on HIP device `device`. */
ntf_status ntf_handle_create(ntf_handle** out, int device);
/* Release the handle's workspace (synchronizes the device first). NULL is a no-op. */
void ntf_handle_destroy(ntf_handle* h);
/* Thread-local message of the last failed call on this thread ("" if none). */
const char* ntf_last_error(void);
/* Static name of a status code. */
const char* ntf_status_string(ntf_status s);
/* Library version string. */
const char* ntf_version(void);
/* Synchronize `stream`, then read and clear the handle's device flag word (NTF_FLAG_*).
 * The calls below are asynchronous and return NTF_OK once enqueued; conditions found on
 * the device while they run (a bounded wait that gave up, a non-finite F-hat) are
 * reported here, never by the enqueueing call. */
ntf_status ntf_device_flags(ntf_handle* h, void* stream, uint32_t* flags_out);
/* Time after which a bounded cross-workgroup wait of the A-HALS kernel (its stopping rule,
 * Sec. 4.1, is decided across workgroups) gives up: the kernel then finishes its sweep
 * loop at once, writes its current iterate and raises NTF_FLAG_WAIT_TIMEOUT. Default 2 s,
 * far above any legitimate wait; seconds in [0, 60]. 0 makes every wait that is not
 * already satisfied give up, which lets tests force the time-out path from the host.
 * Takes effect for later calls (a cached solver graph is rebuilt). */
ntf_status ntf_handle_set_wait_limit(ntf_handle* h, double seconds);

/* ------------------------------------------------------------------ hot-path steps --- */

/* ||T||_F^2 accumulated in float64 (needed by the restart surrogate F-hat, Sec. 3.1.3).
 * out: one device double. Deterministic (fixed reduction order). */
ntf_status ntf_norm2(ntf_handle* h, const ntf_tensor* T, double* out, void* stream);

/* bfloat16 copy of a float32 array, round to nearest even (the stored-tensor form).
 * src: n floats; dst: n uint16 bit patterns. Finite inputs round exactly like the
 * IEEE-style rule; NaN inputs give a quiet NaN. */
ntf_status ntf_cast_bf16(ntf_handle* h, const float* src, uint16_t* dst, int64_t n,
                         void* stream);

/* MTTKRP of mode `mode` (Sec. 2, eq. def:grad, data term T_[n] B^(n) with B^(n) of eq.
 * def:B): P[j, p] = sum over all indices but j_n of T[j_1..j_N] * prod_{l != n} A_l[j_l, p].
 * A: host array of `order` device pointers (A[mode] is ignored and may be NULL).
 * P: I_mode x r float32, row-major, overwritten. float32 tensors use float32 matrix
 * cores, bfloat16 tensors use bfloat16 matrix cores; both accumulate in float32. The
 * Khatri-Rao rows are formed on chip and never written to memory. Deterministic. */
ntf_status ntf_mttkrp(ntf_handle* h, const ntf_tensor* T, const float* const* A, int32_t r,
                      int32_t mode, float* P, void* stream);

/* ntf_mttkrp for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): same arguments, same
 * kernels, same launch shapes and the same bits in P. The split partials live in a static
 * device array of 16 MiB per device (resolved when the handle is created) instead of the
 * handle's workspace; no call allocates. A mode whose partials would exceed it (splits x
 * I_mode x r floats, e.g. beyond 4M floats) returns NTF_EUNSUPPORTED with nothing written;
 * ntf_mttkrp covers it. Calls on one device share the array: calls that overlap on one
 * GPU (different streams, or different handles of the same device) race; calls ordered on
 * one stream do not (each writes every partial it reads). */
ntf_status ntf_mttkrp_noalloc(ntf_handle* h, const ntf_tensor* T, const float* const* A,
                              int32_t r, int32_t mode, float* P, void* stream);

/* The MTTKRPs of every mode n with bit n of `mask` set, all with the same factors (the
 * partial derivatives of the objective for every block at one point, Sec. 2, eq.
 * def:grad), in as few passes over T as the shapes allow: for a 3-way tensor the first
 * two modes share one pass that forms Y = T x_3 A_3 (I_1 x I_2 x r, kept in the handle's
 * workspace when it is smaller than T) and two folds of Y. A: `order` device pointers (a
 * factor may be NULL only if its mode is the only one requested); P: host array of
 * `order` device pointers, P[n] (I_n x r float32) written for the requested modes, others
 * ignored. A 4-way bfloat16 tensor whose last two modes have 128 indices, with r <= 64 and
 * all four modes asked, takes a fused kernel that reads T once: per slab T(i, j, :, :) two
 * matrix-core products (with A_4 and with A_3) give the last two MTTKRPs and an
 * I_1 x I_2 x r array that two folds turn into the first two. Results equal
 * ntf_mttkrp's up to the order of float32 summation. */
ntf_status ntf_mttkrp_multi(ntf_handle* h, const ntf_tensor* T, const float* const* A,
                            int32_t r, int32_t mask, float* const* P, void* stream);

/* MTTKRP autotuner. Times every kernel shape the planner can take for mode `mode` of a
 * tensor of T's shape, dtype and rank r (row tiles of 32, 64 or 128 rows; the row-slab
 * kernel where it applies), `reps` calls each after one warm-up, with HIP events on
 * `stream`, on the caller's T and A; records the fastest in the handle's tuning table
 * (the planner's default shape is kept unless another is faster by more than 3 %),
 * which later ntf_mttkrp and ntf_solve calls on the same shape, dtype, mode and rank use
 * (a cached solver graph is rebuilt). P (I_mode x r) receives the MTTKRP from the chosen
 * shape. Synchronizes `stream` (not for use under stream capture). kernel_out (1 row
 * tiles, 2 row slab), wm_out (row-tile waves along rows) and ms_out (milliseconds per call
 * of the chosen shape) are host pointers and may be NULL. reps outside [1, 1000]:
 * NTF_EINVAL. */
ntf_status ntf_mttkrp_autotune(ntf_handle* h, const ntf_tensor* T, const float* const* A,
                               int32_t r, int32_t mode, float* P, int32_t reps,
                               int32_t* kernel_out, int32_t* wm_out, float* ms_out,
                               void* stream);

/* The handle's tuning table as text, one entry per line: "<key> <kernel> <wm>", where key
 * names dtype, shape, mode and rank (e.g. "bf16:400x400x400:mode2:r32"). Returns the bytes
 * needed including the terminating NUL and copies the text into buf if cap is at least
 * that (buf may be NULL to ask for the size); -1 for a NULL handle. */
int64_t ntf_tune_export(ntf_handle* h, char* buf, int64_t cap);

/* Adds the entries of a text in ntf_tune_export's format to the handle's tuning table
 * (replacing entries with the same key). Blank lines are skipped; a malformed line returns
 * NTF_EINVAL and adds nothing. A choice that does not apply to a shape is ignored by the
 * planner (it falls back to its default). */
ntf_status ntf_tune_import(ntf_handle* h, const char* text);

/* Hadamard product of factor Grams, G = (*)_{l != exclude} A_l^T A_l (r x r, row-major);
 * with exclude = n this is (B^(n))^T B^(n) (Appendix A gradient; Sec. 2.2 Lipschitz
 * matrix). rows: host array of the I_l. exclude = -1 multiplies all `nfac` Grams.
 * Grams accumulate in float64. G32 (float) and/or G64 (double) may be NULL, not both. */
ntf_status ntf_gram(ntf_handle* h, const float* const* A, const int64_t* rows, int32_t nfac,
                    int32_t r, int32_t exclude, float* G32, double* G64, void* stream);

/* A-HALS on one block (Sec. 2.1.4): repeated cyclic sweeps over the columns j = 1..r,
 * W[:, j] <- max(0, P[:, j] - sum_{l != j} W[:, l] G[l, j]) / G[j, j], stopping after
 * max_sweeps sweeps or after the first sweep s with ||W_s - W_{s-1}||_F <= tol *
 * ||W_1 - W_0||_F (Sec. 4.1; norms in float64). tol = 0 runs until a sweep changes
 * nothing or max_sweeps is reached. A column with G[j, j] = 0 is set to 0.
 * W: rows x r, in place (input = warm start). P: rows x r. G: r x r float32, symmetric.
 * sweeps_done: device int32 or NULL. rows <= 12288 for r <= 32, <= 3072 for r <= 128;
 * r > 128 or more rows return NTF_EUNSUPPORTED. */
ntf_status ntf_hals_update(ntf_handle* h, float* W, const float* P, const float* G,
                           int64_t rows, int32_t r, int32_t max_sweeps, double tol,
                           int32_t* sweeps_done, void* stream);

/* Projected-gradient block solver (Sec. 2.2): `steps` steps of
 * W <- max(0, Y - (Y G - P) / L), L = ||G||_2 (largest eigenvalue of G, by power iteration
 * in float64 from the all-ones vector: G is entrywise nonnegative for nonnegative factors),
 * Y = W (accel = 0) or Nesterov's point W_s + ((t_{s-1} - 1) / t_s)(W_s - W_{s-1}) with
 * t_0 = 1, t_s = (1 + sqrt(1 + 4 t_{s-1}^2)) / 2 (accel = 1). W: rows x r in place (input =
 * starting point); P: rows x r; G: r x r float32, symmetric. L_out: one device double that
 * receives L (workspace of the call). r > 128: NTF_EUNSUPPORTED. */
ntf_status ntf_pgd_update(ntf_handle* h, float* W, const float* P, const float* G,
                          int64_t rows, int32_t r, int32_t steps, int32_t accel,
                          double* L_out, void* stream);

/* ADMM block solver (Sec. 2.1.2: AO-ADMM solves each NNLS block with a few ADMM steps).
 * Scaled ADMM on the splitting W = Z with rho = trace(G) / r, U_0 = 0 and Z_0 = W:
 * W_s = (P + rho (Z_{s-1} - U_{s-1})) (G + rho I)^-1, Z_s = max(0, W_s + U_{s-1}),
 * U_s = U_{s-1} + W_s - Z_s; the block's result is Z_s, with the inner stopping rule of
 * Sec. 4.1 (stop after step s >= 2 when ||Z_s - Z_{s-1}||_F <= tol ||Z_1 - Z_0||_F, or at
 * s = 1 if Z_1 = Z_0, at most max_steps). W: rows x r in place; P: rows x r; G: r x r
 * float32, symmetric positive semidefinite (G = 0 gives W = 0). steps_done: one device
 * int32 (may be NULL). (G + rho I)^-1 is formed in float64 by the library. r > 128 or
 * max_steps > 64: NTF_EUNSUPPORTED. */
ntf_status ntf_admm_update(ntf_handle* h, float* W, const float* P, const float* G,
                           int64_t rows, int32_t r, int32_t max_steps, double tol,
                           int32_t* steps_done, void* stream);

/* APG (Sec. 2.2.1; the Appendix's pseudocode), the comparison method with extrapolation
 * inside each block update: outer iteration k, block i (the other blocks at their latest
 * values): w = min(w_hat_{k-1}, delta_w sqrt(L_{k-2} / L_{k-1})) with
 * w_hat_{k-1} = (t_{k-1} - 1) / t_k, t_0 = 1, t_k = (1 + sqrt(1 + 4 t_{k-1}^2)) / 2 and
 * L = ||G||_2 of the block problem; A-hat = A_{k-1} + w (A_{k-1} - A_{k-2}) (A_{-1} = A_0,
 * not projected); A_k = max(0, A-hat - (A-hat G - P) / L). When F(A_k) > F(A_{k-1}) the
 * iteration is redone from A_{k-1} without extrapolation. A: in: A_0, out: A_iters.
 * objective (host, iters doubles, may be NULL): F(A_k) (with the 1/2 of eq. objFun);
 * restarts (host, iters int32, may be NULL). delta_w in [0, 1) (the paper leaves it open;
 * 0.9999 is the usual choice). Synchronous: the host reads F(A_k) back once per iteration
 * to decide the restart; returns after the last iteration. r <= 128. */
ntf_status ntf_solve_apg(ntf_handle* h, const ntf_tensor* T, int32_t r, float* const* A,
                         int32_t iters, double delta_w, double* objective, int32_t* restarts,
                         void* stream);

/* iBPG (Sec. 2.2.2; the Appendix's pseudocode): outer iteration k, block i: w as for APG,
 * then `inner_steps` updates of the block with two points,
 * Y1 = A_cur + w (A_cur - A_prev) (gradient), Y2 = A_cur + beta w (A_cur - A_prev)
 * (inertia), A_prev <- A_cur, A_cur <- max(0, Y2 - (Y1 G - P) / L); no restart. The inner
 * rule "until some criteria" is read as exactly inner_steps updates. A_{-1} = A_0.
 * A: in: A_0, out: the last A_cur. objective (host, iters doubles, may be NULL): F after each
 * outer iteration. delta_w in [0, 1) (the pseudocode's 0.99), beta >= 0 (its 1.01).
 * Synchronous. r <= 128. */
ntf_status ntf_solve_ibpg(ntf_handle* h, const ntf_tensor* T, int32_t r, float* const* A,
                          int32_t iters, int32_t inner_steps, double delta_w, double beta,
                          double* objective, void* stream);

/* One HER step of Algorithm 2 on caller buffers.
 *  INIT:        state <- {beta0, 1, *fhat, ...}; `fhat` must point to F(A_0).
 *  EXTRAPOLATE: block `block`: eq. extproj_her, A_hat = max(0, A_new + beta (A_new - A)),
 *               with beta = state->beta (= beta_{k-1}); computed in float64, stored float32.
 *  DECIDE:      Algorithm 2 restart test with *fhat = F-hat_k: if F-hat_k > F-hat_{k-1}
 *               restart (beta_bar <- beta, beta <- beta / eta; A[l] <- A_new[l]), else
 *               accept (beta <- min(beta_bar, gamma beta), beta_bar <- min(1, gamma_bar
 *               beta_bar); A[l] <- A_hat[l]) for every block l (eqs. HER_eq:beta_update,
 *               HER_eq:beta_bar_update). Equality accepts.
 * nblocks/rows/A/A_new/A_hat describe all blocks (rows: host array). `block` is used by
 * EXTRAPOLATE only; `params` by INIT and DECIDE; `fhat` (device double) by INIT and DECIDE. */
ntf_status ntf_her_step(ntf_handle* h, ntf_her_op op, ntf_her_state* state,
                        const ntf_her_params* params, int32_t nblocks, const int64_t* rows,
                        int32_t r, float* const* A, float* const* A_new, float* const* A_hat,
                        int32_t block, const double* fhat, void* stream);

/* Restart surrogate (Sec. 3.1.3; Algorithm 2's F-hat) from the last block's quantities:
 * F = 1/2 (||T||^2 - 2 <P, A> + <G, A^T A>), all in float64. normT2: device double.
 * P, A: rows x r float32; G: r x r float64. fhat: device double (overwritten). */
ntf_status ntf_error(ntf_handle* h, const double* normT2, const float* P, const float* A,
                     const double* G, int64_t rows, int32_t r, double* fhat, void* stream);

/* MTTKRP of mode `mode` of a Tucker-format tensor (Appendix A):
 * P = U^(mode) MTTKRP_mode(G; Q^(p)) with Q^(p) = (U^(p))^T A^(p) (r_p x r, float64
 * accumulation over n_p), the core's MTTKRP on the matrix cores and the expansion by
 * U^(mode); T is never formed. A: `order` device pointers, n_p x r (A[mode] ignored);
 * P: n_mode x r float32, overwritten. Tucker ranks r_p <= 4096. */
ntf_status ntf_tucker_mttkrp(ntf_handle* h, const ntf_tucker* X, const float* const* A,
                             int32_t r, int32_t mode, float* P, void* stream);

/* ||T||_F^2 of a Tucker-format tensor in float64, from the core and the bases' Grams:
 * <G x_1 (U^(1)T U^(1)) ... x_N (U^(N)T U^(N)), G> (||G||^2 for orthonormal bases).
 * out: one device double. */
ntf_status ntf_tucker_norm2(ntf_handle* h, const ntf_tucker* X, double* out, void* stream);

/* ntf_solve on a Tucker-format tensor (Appendix A: HER is unchanged, the MTTKRP and ||T||^2
 * come from the format; the objective is eq. objFunTucker). Same arguments and semantics as
 * ntf_solve; A holds n_p x r factors. */
ntf_status ntf_solve_tucker(ntf_handle* h, const ntf_tucker* X, int32_t r, float* const* A,
                            const ntf_her_params* params, int32_t iters, ntf_her_state* state,
                            int32_t resume, const ntf_trace* trace, void* stream);

/* Algorithm 2 (HER) with A-HALS blocks for `iters` outer iterations (Sec. 3.1). The
 * factors A (host array of `order` device pointers) hold A_0 on entry and the final
 * iterates on return. state (device, may be NULL): if `resume` is nonzero it must hold
 * the state a previous ntf_solve left and A its factors; otherwise it is initialized
 * (beta0, beta_bar = 1, F-hat_0 = F(A_0)). On return it holds the final state. trace may
 * be NULL. The outer iteration is captured once into a HIP graph and replayed.
 * The solver runs A-HALS with the stopping rule of `params` and the restart test on
 * F-hat in float64 on the device; the host never synchronizes inside the loop. */
ntf_status ntf_solve(ntf_handle* h, const ntf_tensor* T, int32_t r, float* const* A,
                     const ntf_her_params* params, int32_t iters, ntf_her_state* state,
                     int32_t resume, const ntf_trace* trace, void* stream);

/* Squared-error loss L = ||T - [[A_1..A_N]]||_F^2 (the objective of eq. objFun without
 * its 1/2) by the Gram trick of Sec. 3.1.3, all in float64:
 * L = ||T||^2 - 2 <P, A> + <G, A^T A>, with A the factor of some mode n, P its MTTKRP and
 * G the float64 Hadamard product of the other factors' Grams (ntf_gram with exclude = n).
 * normT2, loss: device doubles (loss overwritten). P, A: rows x r float32. */
ntf_status ntf_cp_loss(ntf_handle* h, const double* normT2, const float* P, const float* A,
                       const double* G, int64_t rows, int32_t r, double* loss, void* stream);

/* Gradient of the loss with respect to factor n (Sec. 2, eq. def:grad):
 * grad = alpha * s * (A G - P), s = *scale (a device double, e.g. the incoming gradient of
 * the loss in reverse-mode differentiation) or 1 when scale is NULL. alpha = 2 gives the
 * gradient of L above, alpha = 1 that of the paper's F. A, P, grad: rows x r float32 (grad
 * overwritten; it may not alias A or P); G: r x r float64 from ntf_gram(exclude = n).
 * Accumulation in float64. */
ntf_status ntf_cp_grad(ntf_handle* h, const float* A, const float* P, const double* G,
                       int64_t rows, int32_t r, const double* scale, float alpha, float* grad,
                       void* stream);

/* One problem of a batch (see ntf_solve_batched). */
typedef struct ntf_problem {
  ntf_tensor T;                /* order 3, NTF_F32, each dim in [1, 256] */
  int32_t r;                   /* rank, 1..32 */
  int32_t reserved;            /* must be 0 */
  float* A[3];                 /* device factors I_n x r, row-major: A_0 in, result out */
  ntf_her_state* state;        /* device; output state, and input state when resuming;
                                  may be NULL when not resuming */
  double* trace_fhat;          /* device [iters]: F-hat_k, or NULL */
  int32_t* trace_restart;      /* device [iters]: 1 if iteration k restarted, or NULL */
  int32_t* trace_sweeps;       /* device [iters * 3]: A-HALS sweeps per block, or NULL */
} ntf_problem;

/* Algorithm 2 (HER with A-HALS blocks, Sec. 3.1) for `nprob` independent 3-way float32
 * problems of any shapes and ranks, `iters` outer iterations each. One outer iteration of
 * every problem is a short sequence of grouped launches (the tensor passes and folds split
 * each problem into many workgroups; each A-HALS block takes one workgroup per problem,
 * larger problems first), captured once into a HIP graph and replayed `iters` times while
 * the problem set and parameters are unchanged. Per problem the results equal those of
 * ntf_solve up to rounding order (same method, parameters and F-hat_0 = F(A_0)); restart
 * decisions may differ where rounding decides them. probs: host array; all pointers
 * inside are device pointers. resume != 0 continues from each problem's state and
 * factors. The host descriptors and work lists are copied from pinned staging: the call
 * waits until the previous call's copy has completed. */
ntf_status ntf_solve_batched(ntf_handle* h, int32_t nprob, const ntf_problem* probs,
                             const ntf_her_params* params, int32_t iters, int32_t resume,
                             void* stream);

/* || T - [[A_1..A_N]] ||_F^2 from the explicit residual, float64 accumulation (the data
 * fitting error of Sec. 4.1, eq. err_true_def, times 2). out: device double. */
ntf_status ntf_residual_norm2(ntf_handle* h, const ntf_tensor* T, const float* const* A,
                              int32_t r, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NTF_H */
