/*
 * ocsc.h -- C ABI of libocsc: online convolutional sparse coding (OCSC) on
 * AMD Instinct MI355X (gfx950).
 *
 * The calls follow the online CSC problem and Algorithm 3 of Wang, Yao, Kwok
 * and Ni, "Scalable Online Convolutional Sparse Coding": per sample, the
 * frequency-domain code update (eq. fcsc_code), the per-frequency history
 * update (eqs. B_update and C_update) and the dictionary update DictOCSC
 * (Algorithm 2, eq. sub_d_sol, Proposition 2).
 *
 * Conventions shared by every call
 *   - Sizes: K filters of filt_h x filt_w taps; samples and codes live on a
 *     pad_h x pad_w grid (P = pad_h * pad_w), both powers of two.  Spectra are
 *     stored as the non-redundant half, Pf = pad_h * (pad_w/2 + 1) complex
 *     values per plane (row-major, column index fastest).
 *   - DFT: unnormalised forward transform, 1/P on the inverse.  Convolution is
 *     circular on the padded grid; a filter occupies the top-left
 *     filt_h x filt_w block of its plane.
 *   - Real type: double for OCSC_FP64 contexts, float for OCSC_FP32 contexts.
 *     Every "real" buffer below is of that type.
 *   - Pointers named *_dev are device pointers (hipMalloc'd memory or a torch
 *     tensor's data_ptr()), 16-byte aligned, on the context's device; the caller owns them and
 *     must keep them alive until the call's work on the context stream has
 *     completed.  The library owns all learner state and workspace.
 *   - Asynchrony: calls enqueue work on the context stream and return without
 *     waiting, except those that return values in host memory
 *     (ocsc_objective, ocsc_objective_terms, ocsc_surrogate, ocsc_diagnostics),
 *     ocsc_sync, and the state getters/setters (which wait for their copy).
 *   - Errors: every call returns an ocsc_status.  Arguments and call order are
 *     validated before any device work, so validation errors never leave the
 *     context half-updated.  No C++ exception crosses the ABI.  The message of
 *     the last failure is available from ocsc_last_error.
 *   - Threads: a context must be used by one host thread at a time; distinct
 *     contexts are independent.
 */
#ifndef OCSC_H_
#define OCSC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ocsc_ctx ocsc_ctx;

typedef enum {
  OCSC_OK = 0,
  OCSC_E_INVALID_ARG = -1, /* a size, pointer or hyper-parameter is out of range */
  OCSC_E_STATE = -2,       /* calls made out of order (see each call) */
  OCSC_E_OOM = -3,         /* device allocation failed */
  OCSC_E_HIP = -4,         /* a HIP runtime call failed; text in ocsc_last_error */
  OCSC_E_NUMERIC = -5,     /* non-finite input or result */
  OCSC_E_UNSUPPORTED = -6  /* valid request the library has no kernel for */
} ocsc_status;

typedef enum {
  OCSC_FP64 = 0, /* all arithmetic in double */
  OCSC_FP32 = 1  /* all arithmetic in float; objective reductions in double */
} ocsc_precision;

typedef struct {
  int32_t struct_size; /* = sizeof(ocsc_opts) */
  int32_t iters_code;  /* code-ADMM iterations per sample (J_z), >= 1; default 10 */
  int32_t iters_dict;  /* DictOCSC iterations per update (J of Algorithm 2), >= 1; default 10 */
  int32_t max_batch;   /* largest B accepted by ocsc_code_update; default 1 */
  int32_t precision;   /* ocsc_precision; default OCSC_FP64 */
  int32_t flags;       /* OCSC_FLAG_* bits; default 0 */
  double rho_dict;     /* dictionary-ADMM penalty rho_d; <= 0 selects rho * P (eq. sub_d_sol) */
  void* stream;        /* hipStream_t to enqueue on; NULL is the default (null) stream */
} ocsc_opts;

/* opts.flags: create a private non-blocking stream and ignore opts.stream. */
#define OCSC_FLAG_OWN_STREAM 1
/* opts.flags: also keep the history H_p = sum_i conj(z_ip) z_ip^T (Proposition 1)
 * and the running sums of ||x_i||^2 and ||U_i||_1, so that ocsc_surrogate can
 * evaluate the online objective.  Costs a second K x K real matrix per
 * frequency and, with a batch of B, B extra rank-one updates per history fold. */
#define OCSC_FLAG_KEEP_HISTORY 2
/* opts.flags: warm-start DictOCSC: each ocsc_dict_update continues from the
 * V and Theta of the previous one instead of V = Theta = 0. */
#define OCSC_FLAG_WARM_START 4
/* opts.flags: precision form of the history (FP32 contexts, K <= 256, cold
 * start).  ocsc_history_accumulate adds the minibatch to H and G with the
 * product conj(Z)^T Z on the BF16 matrix cores (FP32 accumulation, z split
 * into two BF16 parts, the products hi*hi + hi*lo + lo*hi), then recomputes
 * C_p = (H_p + rho_d I)^-1 for every frequency from FP64 Cholesky factors,
 * instead of the Sherman-Morrison recursion (for K > 128: the inverses of
 * two 128-blocks joined by their Schur complement).  Implies
 * OCSC_FLAG_KEEP_HISTORY.  K > 128 is available only in this form: its D-step
 * streams C_p from HBM instead of holding it in LDS.  K > 128 also needs a
 * workspace of up to 2048 x 1.25 MB.  A factorisation whose matrix is not
 * positive definite (a pivot <= 0 or NaN: a non-finite history, or an
 * indefinite H given to ocsc_set_state) leaves NaN in C at that frequency and
 * is reported once, as OCSC_E_NUMERIC, by the next ocsc_sync,
 * ocsc_objective, ocsc_objective_terms, ocsc_surrogate or ocsc_diagnostics. */
#define OCSC_FLAG_CHOLESKY 8
/* opts.flags, with OCSC_FLAG_CHOLESKY only (else OCSC_E_UNSUPPORTED): after
 * every D-step, one step of iterative refinement of d_p = (H_p + rho_d I)^-1 rhs_p
 * (eq. sub_d_sol) against the kept history: r_p = rhs_p - (H_p + rho_d I) d_p
 * formed from the FP32 H_p and d_p with FP64 sums, then d_p += C_p r_p.  It
 * removes the error of the FP32 rounding of C_p (not that of H_p itself), at
 * the cost of two more passes over K x K reals per frequency in each of the
 * iters_dict D-steps. */
#define OCSC_FLAG_REFINE 16

/* Fill *opts with the defaults listed above. */
void ocsc_default_opts(ocsc_opts* opts);

/*
 * Create a learner (Algorithm 3, initialisation): history G = 0 and
 * C_p = I / rho_d at every frequency, t = 0, dictionary spectrum zero until
 * ocsc_set_dictionary.
 *   1 <= K <= 128 in FP32 and 1 <= K <= 92 in FP64 (the D-step holds C_p in
 *   LDS), K <= 256 with OCSC_FLAG_CHOLESKY; 1 <= filt_h <= pad_h;
 *   1 <= filt_w <= pad_w; pad_h, pad_w powers of
 *   two, both in [32, 128] (planes transformed in LDS) or both in {256, 512}
 *   (two-pass transforms; then max_batch * K <= 65535); lambda >= 0 (the l1
 *   weight beta of eq. csc); rho > 0 (the code-ADMM penalty).  opts may be NULL
 *   (defaults).  The device is the current HIP device at the time of the call.
 * Errors: OCSC_E_INVALID_ARG (nothing allocated, *out untouched),
 *   OCSC_E_UNSUPPORTED (size/precision without a kernel), OCSC_E_OOM, OCSC_E_HIP.
 */
int ocsc_init(ocsc_ctx** out, int K, int filt_h, int filt_w, int pad_h, int pad_w,
              double lambda, double rho, const ocsc_opts* opts);

/* Free the context and all library-owned device memory.  NULL is accepted. */
int ocsc_destroy(ocsc_ctx* ctx);

/*
 * Set the dictionary from spatial filters D_dev: real [K][filt_h][filt_w].
 * The spectrum F(zero-pad(D_k)) replaces the current dictionary (Algorithm 3,
 * initialisation with D_0).  History and t are unchanged.
 */
int ocsc_set_dictionary(ocsc_ctx* ctx, const void* D_dev);

/*
 * Export the dictionary: D_dev_out real [K][filt_h][filt_w] receives the crop of
 * the real inverse DFT of the current dictionary spectrum (Algorithm 3, last
 * loop: D(:,k) = H(F^-1 D~(:,k))).
 */
int ocsc_get_dictionary(ocsc_ctx* ctx, void* D_dev_out);

/*
 * Code B samples against the current dictionary (eq. fcsc_code by scaled
 * ADMM, iters_code iterations from U = W = 0 per sample; threshold lambda/rho).
 *   x_dev: real [B][pad_h][pad_w] samples on the padded grid.
 *   codes_dev_out: real [B][K][pad_h][pad_w] receives the sparse codes U, or NULL.
 * The last Z-step spectra and the sample spectra are kept for the next
 * ocsc_history_accumulate; codes of an earlier call that were not yet
 * accumulated are discarded.  1 <= B <= max_batch.
 */
int ocsc_code_update(ocsc_ctx* ctx, const void* x_dev, int B, void* codes_dev_out);

/*
 * Like ocsc_code_update, but the B samples join the samples already pending
 * (coded since the last ocsc_history_accumulate) instead of replacing them,
 * in the next pending slots; the next ocsc_history_accumulate folds them all
 * in slot order.  This lets a request loop code requests as they arrive and
 * fold them once.  OCSC_E_INVALID_ARG if the pending samples would exceed
 * max_batch.
 */
int ocsc_code_append(ocsc_ctx* ctx, const void* x_dev, int B, void* codes_dev_out);

/*
 * Code one batch on each of n contexts -- grids of different sizes -- with
 * all their code-ADMM iterations (eq. fcsc_code) in one persistent,
 * cooperative launch: a fixed grid of resident workgroups takes each phase's
 * work items grouped by grid (FFT size) and meets at a grid-wide barrier
 * between phases (Z-steps; plane steps or inverse column passes; row passes;
 * forward column passes).  The sample spectra are computed first by each
 * context's usual transform.  Each context ends as after
 * ocsc_code_update(ctxs[s], x_devs[s], Bs[s], codes_devs[s]), with the same
 * values bit for bit.
 *   1 <= n <= 8 distinct contexts with the same precision, iters_code and
 *   device, K <= 128 each (OCSC_E_UNSUPPORTED above); 1 <= Bs[s] <= max_batch;
 *   x_devs[s]: real [Bs[s]][pad_h][pad_w] of that context;
 *   codes_devs: NULL, or n entries, each NULL or real [Bs[s]][K][pad_h][pad_w].
 * Enqueued on the first context's stream after the earlier work of every
 * member's stream; later work on every member's stream waits for it.
 * Two-pass grids use the default column and row blocks.
 */
int ocsc_code_update_group(ocsc_ctx* const* ctxs, const void* const* x_devs, const int* Bs,
                           void* const* codes_devs, int n);

/*
 * Fold the spectra kept by the last ocsc_code_update into the history, in
 * sample order (eqs. B_update and C_update, unnormalised):
 *   G_p += conj(z_p) x_p;  C_p <- C_p - (C_p u)(C_p u)^H / (1 + u^H C_p u), u = conj(z_p),
 * so that C_p = (sum_i conj(z_ip) z_ip^T + rho_d I)^-1; t += B.
 * OCSC_E_STATE if there are no pending codes (none coded, or already folded).
 * With OCSC_FLAG_KEEP_HISTORY, H_p += conj(z_p) z_p^T as well.
 * The fold of G and C may be deferred into the first sweep of the next
 * ocsc_dict_update; every observable result is the same up to rounding.
 */
int ocsc_history_accumulate(ocsc_ctx* ctx);

/*
 * DictOCSC (Algorithm 2): iters_dict ADMM iterations from V = 0, Theta = 0
 * (with OCSC_FLAG_WARM_START: from the V and Theta the previous call left) of
 *   d_p = C_p (G_p + rho_d (F(V)_p - Theta_p))            (eq. sub_d_sol, column form)
 *   V_k = alpha_k / max(||alpha_k||, 1), alpha_k = crop(Re F^-1(d_k + Theta_k))  (Prop. 2)
 *   Theta += d - F(V)
 * The last d becomes the dictionary spectrum.  OCSC_E_STATE if t = 0.
 */
int ocsc_dict_update(ocsc_ctx* ctx);

/*
 * DictOCSC for n contexts on different grids that share one dictionary (a
 * generalisation of Algorithm 2; the paper uses one grid).  Each context
 * keeps its own history and runs its own D-step (eq. sub_d_sol); one
 * consensus V-step (Proposition 2 applied to the weighted mean)
 *   V = proj( sum_s P_s alpha_s / sum_s P_s ),  alpha_s = crop(Re F_s^-1(d_s + Theta_s)),
 * gives every context the same V; then Theta_s += d_s - F_s(V).  The weights
 * P_s make the fixed point minimise the sum of all samples' losses.  Each
 * context's last d_s becomes its dictionary spectrum.  Cold start only.
 *   ctxs: n (1..8) distinct contexts with equal K, filter size, precision,
 *   iters_dict and device, each with t >= 1 (else OCSC_E_STATE); a context
 *   created with OCSC_FLAG_WARM_START: OCSC_E_UNSUPPORTED.
 * The work is enqueued on the first context's stream after every member's
 * earlier work; later work on each member's stream waits for it.  Pending
 * codes of the members are discarded; deferred folds are applied.
 */
int ocsc_dict_update_group(ocsc_ctx* const* ctxs, int n);

/*
 * Objective of eq. csc per sample against the current dictionary:
 *   out_host[b] = 1/2 ||x_b - sum_k F^-1(D~_k F(U_bk))||^2 + lambda ||U_b||_1,
 * evaluated through Parseval's theorem with double-precision accumulation.
 *   x_dev: real [B][pad_h][pad_w]; codes_dev: real [B][K][pad_h][pad_w];
 *   out_host: B doubles in host memory.  Waits for completion.
 * May overwrite the library's code workspace, but not the spectra kept for
 * ocsc_history_accumulate.  1 <= B <= max_batch.  OCSC_E_NUMERIC when a value
 * is not finite (the calls that do not wait never inspect values: a
 * non-finite sample propagates through the codes and the history, and this
 * call, ocsc_surrogate and ocsc_diagnostics report it).
 */
int ocsc_objective(ocsc_ctx* ctx, const void* x_dev, const void* codes_dev, int B,
                   double* out_host);

/*
 * The two terms of the objective above, separately: out_host[2b] receives
 * 1/2 ||x_b - sum_k F^-1(D~_k F(U_bk))||^2 and out_host[2b + 1] receives
 * ||U_b||_1 (without lambda).  The first term gives the reconstruction PSNR
 * of the paper's evaluation (section 4): 10 log10(peak^2 P / (2 term)).
 * out_host: 2B doubles in host memory.  Same rules as ocsc_objective.
 */
int ocsc_objective_terms(ocsc_ctx* ctx, const void* x_dev, const void* codes_dev, int B,
                         double* out_host);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * objective of ocsc_objective with every intermediate buffer taken from a
 * static scratch array of the library instead of the context's workspace,
 * and the result left in device memory.  The call allocates nothing (no
 * hipMalloc, hipFree, host copy or synchronisation), so it may be captured
 * in a graph.
 *   out_dev: B doubles in caller-owned device memory, 8-byte aligned;
 *   out_dev[b] = 1/2 ||x_b - sum_k F^-1(D~_k F(U_bk))||^2 + lambda ||U_b||_1,
 *   the same values as ocsc_objective, bit for bit.
 *   x_dev, codes_dev, B: as for ocsc_objective, except that B is bounded by
 *   the scratch instead of max_batch: B (K + 1) spectra of Pf complex values
 *   plus 8 B (ceil(Pf / 256) + 64) bytes of partial sums must fit in
 *   OCSC_NOALLOC_SCRATCH_BYTES (else OCSC_E_INVALID_ARG, nothing enqueued);
 *   at 128 x 128 with K = 100 that is B <= 4 in FP32 and B <= 2 in FP64.
 * Enqueued on the context stream; returns without waiting, so values are not
 * inspected (a non-finite input propagates to out_dev; ocsc_objective
 * reports it).  The context's workspace, state and pending codes are not
 * touched, and no kernel timing is recorded for the call.
 * The scratch is one array per device (32 MiB, held from the first
 * ocsc_init on that device until the process ends), shared by every context
 * on the device; nothing in it needs to start at zero, and each call
 * overwrites what the last one left.  Calls that overlap on one device -- on
 * different streams, or from several host threads -- race on it: order them
 * on one stream or with events.
 */
#define OCSC_NOALLOC_SCRATCH_BYTES (32 * 1024 * 1024)
int ocsc_objective_noalloc(ocsc_ctx* ctx, const void* x_dev, const void* codes_dev, int B,
                           double* out_dev);

/*
 * Online surrogate of Proposition 1 (unnormalised), in double:
 *   F_t(D~) = 1/(2P) sum_p c_p [d_p^H H_p d_p - 2 Re d_p^H G_p]
 *             + 1/2 sum_i ||x_i||^2 + lambda sum_i ||U_i||_1,
 * with d_p = D~[:, p], sums over the t samples folded so far and c_p the
 * Parseval weight of the half spectrum (1 on the columns 0 and pad_w/2, else 2).
 * D~ = F(zero-pad(D_dev)) for spatial filters D_dev real [K][filt_h][filt_w]
 * (device), or the current dictionary spectrum when D_dev is NULL.
 * out_host: one double in host memory.  Waits for completion.
 * OCSC_E_STATE unless the context was created with OCSC_FLAG_KEEP_HISTORY.
 */
int ocsc_surrogate(ocsc_ctx* ctx, const void* D_dev, double* out_host);

/*
 * Diagnostics of the dictionary update, in double; out_host (host memory)
 * receives 2 + 2K values:
 *   [0]            ||F^-1(D~ - F(zero-pad(V)))||_F, the primal residual of the
 *                  last DictOCSC iterate (equals the last change of Theta);
 *   [1]            ||F^-1 D~||_F over the padded grid;
 *   [2 + k]        ||V_k||_2 (each <= 1 by Proposition 2);
 *   [2 + K + k]    ||D_k||_2 of the exported filters (ocsc_get_dictionary).
 * Waits for completion.
 */
int ocsc_diagnostics(ocsc_ctx* ctx, double* out_host);

/* Wait until all work enqueued on the context stream has finished.
 * OCSC_E_NUMERIC if, in the precision form, a Cholesky factorisation met a
 * pivot that was not positive since the last call that waits (see
 * OCSC_FLAG_CHOLESKY). */
int ocsc_sync(ocsc_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Steady-state step as a HIP graph: two bodies of Algorithm 3 (code update,
 * history accumulate, dictionary update) captured once and replayed, which
 * removes the per-launch host cost of the ~40 launches of a step.
 *   x_dev: real [2][B][pad_h][pad_w], read by each launch (the caller refills it);
 *   codes_dev_out: real [2][B][K][pad_h][pad_w] or NULL.
 * Capture needs a context on a non-default stream (OCSC_E_UNSUPPORTED) with
 * no pending codes and no deferred fold (OCSC_E_STATE); capturing does not
 * run the steps.  Each ocsc_graph_launch runs both steps on the context
 * stream (t += 2B) with the same results as the eager calls; it needs the
 * same state (OCSC_E_STATE otherwise).  Eager calls may be interleaved.
 * ------------------------------------------------------------------------- */
typedef struct ocsc_graph ocsc_graph;
int ocsc_graph_create(ocsc_ctx* ctx, const void* x_dev, int B, void* codes_dev_out, ocsc_graph** out);
int ocsc_graph_launch(ocsc_graph* graph);
/* Waits for the context stream, then frees the graph.  NULL is accepted. */
int ocsc_graph_destroy(ocsc_graph* graph);

/* ---------------------------------------------------------------------------
 * Launch shapes of the code update (the per-sample ADMM of eq. fcsc_code:
 * Z-step and plane kernel, 2 launches per code iteration) and their
 * autotuner.  Every valid shape with two_pass 0 or 1 computes the same values
 * bit for bit (the per-element arithmetic and the order of every sum are
 * fixed); only the speed differs, so a tuned context reproduces an untuned
 * one exactly.  The split plane step (two_pass 2) factors the column DFTs
 * differently: its shapes agree bit for bit among themselves, and with the
 * others to rounding.
 *   plane_threads: threads per workgroup of the plane kernel, one plane (or
 *                  one row residue of a plane, two_pass 2) per workgroup:
 *                  256, 512 or 1024, at most pad_h * pad_w / 4.  Grids with
 *                  a side above 128 use fixed two-pass kernels and accept
 *                  only 256 there (two_pass 1).
 *   zstep_freqs:   frequencies per Z-step workgroup, 16, 32 or 64
 *                  (16 * zstep_freqs threads).
 *   zstep_samples: samples per Z-step workgroup, 1, 2 or 4 (the dictionary
 *                  spectrum is read once for them).
 *   col_bytes:     two-pass grids: bytes of each spectrum row that one
 *                  column-pass workgroup transforms (its block of columns):
 *                  128, 256 or 512, with pad_h * col_bytes <= 131072.
 *   row_block:     two-pass grids: rows per row-pass workgroup, 4, 8 or 16.
 *                  (col_bytes and row_block are checked but unused on
 *                  one-pass grids.)
 *   chunk_samples: 0, or 1, 2, 4, 8 or 16: a batch is coded in groups of
 *                  this many samples, each group running all its iterations
 *                  before the next starts (its workspace can then stay in
 *                  the Infinity Cache); 0 runs the whole batch together.
 *   two_pass:      1 on two-pass grids; on 64 x 64 and 128 x 128 grids 0 (the
 *                  one-pass plane kernel) or 1 (the column and row passes,
 *                  more workgroups for small batches; the first selection
 *                  allocates a max_batch x K spectrum buffer, OCSC_E_OOM);
 *                  0 on other grids.  On every grid also 2: each plane
 *                  split by row residue over F workgroups (F = 2 on grids up
 *                  to 128, for batches that leave CUs idle; on 256 and 512
 *                  grids 2 to 16, so that one residue's rows fit in LDS and
 *                  the plane step is one kernel instead of three); the last
 *                  radix-F step of the column DFTs then runs in the Z-step.
 * Defaults: plane_threads 1024 for 128 x 128 grids, else 256; 16; 1; 128; 8; 0;
 * 1 on two-pass grids, else 0.
 * ocsc_autotune times whole code updates for the group size.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t plane_threads;
  int32_t zstep_freqs;
  int32_t zstep_samples;
  int32_t col_bytes;
  int32_t row_block;
  int32_t chunk_samples;
  int32_t two_pass;
} ocsc_tuning;

int ocsc_get_tuning(const ocsc_ctx* ctx, ocsc_tuning* out);
/* OCSC_E_INVALID_ARG for a shape outside the lists above (the context keeps
 * its shape). */
int ocsc_set_tuning(ocsc_ctx* ctx, const ocsc_tuning* tuning);
/* Time every valid shape of both kernels on the context's own code
 * workspace for batches of B samples (1 <= B <= max_batch) and keep the
 * fastest of each.  The workspace contents are overwritten, so the call
 * needs no pending codes (OCSC_E_STATE); a deferred history fold is applied
 * first.  The learner state (dictionary, history, t) is not changed.  Writes
 * the chosen shape to out and the summed time of one Z-step and one plane
 * launch of the whole batch with it to best_ms (both nullable).  Waits for completion; not
 * allowed during stream capture. */
int ocsc_autotune(ocsc_ctx* ctx, int B, ocsc_tuning* out, double* best_ms);

/* Text of the last failure on this context (or of the last failed ocsc_init
 * when ctx is NULL).  Valid until the next call on the same context. */
const char* ocsc_last_error(const ocsc_ctx* ctx);

/* ---------------------------------------------------------------------------
 * State access, for checkpoints and for checking intermediate results.
 * Complex values are interleaved (re, im) pairs of the context's real type.
 * ------------------------------------------------------------------------- */
typedef enum {
  OCSC_STATE_DICT_HAT = 0, /* complex [K][Pf]: dictionary spectrum D~ */
  OCSC_STATE_G = 1,        /* complex [K][Pf]: history b^p (unnormalised sum) */
  OCSC_STATE_CINV = 2,     /* real [Pf][K][K]: C_p = (H_p + rho_d I)^-1 packed as
                              R[i][j] = Re C_ij (j >= i), R[j][i] = Im C_ij (j > i) */
  OCSC_STATE_V = 3,        /* real [K][filt_h][filt_w]: last feasible V of DictOCSC */
  OCSC_STATE_THETA = 4,    /* complex [K][Pf]: last scaled dual Theta of DictOCSC */
  OCSC_STATE_ZHAT = 5,     /* complex [max_batch][K][Pf]: last Z-step spectra (read only) */
  OCSC_STATE_XHAT = 6,     /* complex [max_batch][Pf]: last sample spectra (read only) */
  OCSC_STATE_H = 7,        /* real [Pf][K][K]: history H_p, packed like CINV (needs
                              OCSC_FLAG_KEEP_HISTORY) */
  OCSC_STATE_SUMS = 8,     /* double [2]: sum_i ||x_i||^2 and sum_i ||U_i||_1 (needs
                              OCSC_FLAG_KEEP_HISTORY) */
  OCSC_STATE_RHS = 9       /* complex [K][Pf]: D-step right-hand side G + rho_d (F(V) - Theta)
                              carried between dictionary updates (needs OCSC_FLAG_WARM_START) */
} ocsc_state;

/* Size in bytes of one state item. */
int ocsc_state_bytes(const ocsc_ctx* ctx, int which, int64_t* bytes_out);
/* Copy a state item to dst_dev (device memory of ocsc_state_bytes bytes).
 * Pending history folds are applied first.  Waits for the copy.  Items that
 * need a flag the context lacks: OCSC_E_INVALID_ARG. */
int ocsc_get_state(ocsc_ctx* ctx, int which, void* dst_dev);
/* Overwrite a state item from src_dev.  Every item but ZHAT and XHAT
 * (OCSC_E_INVALID_ARG otherwise).  Pending codes are discarded.  Waits.
 * A checkpoint is DICT_HAT, G, CINV and the count; with OCSC_FLAG_KEEP_HISTORY
 * also H and SUMS; with OCSC_FLAG_WARM_START also V, THETA and RHS. */
int ocsc_set_state(ocsc_ctx* ctx, int which, const void* src_dev);
/* Number of samples folded into the history so far (t of Algorithm 3). */
int ocsc_get_count(const ocsc_ctx* ctx, int64_t* t_out);
/* Overwrite t (used when a checkpoint is restored). */
int ocsc_set_count(ocsc_ctx* ctx, int64_t t);

/* ---------------------------------------------------------------------------
 * Kernel timing.  When enabled, the library brackets each launch with HIP
 * events on the context stream and accumulates per-kernel-class durations.
 * ------------------------------------------------------------------------- */
typedef enum {
  OCSC_KC_FFT = 0,       /* sample / dictionary / objective plane transforms */
  OCSC_KC_ZSTEP = 1,     /* code Z-step, one launch per code iteration */
  OCSC_KC_CODEPLANE = 2, /* fused inverse DFT, soft threshold, dual, forward DFT */
  OCSC_KC_HISTORY = 3,   /* history fold, alone or fused with the first D-step sweep */
  OCSC_KC_DSTEP = 4,     /* D-step sweep over C without a fold */
  OCSC_KC_VSTEP = 5,     /* V-step, Theta update and next D-step right-hand side */
  OCSC_KC_OTHER = 6,
  OCSC_KC_COUNT = 7
} ocsc_kernel_class;

/* Time the kernel classes whose bit (1u << class) is set in class_mask; 0
 * disables timing.  Every call clears the accumulators. */
int ocsc_profile_enable(ocsc_ctx* ctx, unsigned class_mask);
/* Total milliseconds and launch count of one kernel class since enabling.
 * Waits for outstanding timed launches. */
int ocsc_profile_read(ocsc_ctx* ctx, int kernel_class, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* OCSC_H_ */
