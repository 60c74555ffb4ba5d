/*
 * bdu.h -- FP64 bidiagonal updating on one MI355X (gfx950).
 *
 * A handle holds a factorization A = Q Bd P^T in device memory, with Q m x m
 * and P n x n orthogonal (column-major, leading dimension = rows) and Bd
 * upper bidiagonal (diagonal d[0..n-1], superdiagonal e[0..n-2]), the
 * bidiagonal factorization of Brust & Saunders, "Fast and Accurate SVD-Type
 * Updating in Streaming Data", eq. (bidiag).  An update replaces it by a
 * factorization of A + B C^T (eq. main) with the Givens method of Section 3.4
 * (Algorithm 2): project u = Q^T b, v = P^T c (eq. bidiagsubproblem),
 * generate the rotations that fold u v^T into Bd and chase the fill back to
 * bidiagonal form, and accumulate them into Q and P (eq. bidiagplus).  A
 * rank-r update is r rank-1 passes in column order, each projecting its
 * column with the current Q and P (Section 3.2, eq. (rk1)).
 *
 * Everything is FP64.  The numbers produced are exactly those of the
 * schedule and rounding conventions the library documents: projections are
 * sequential fma dot products, rotations are r = sqrt(fma(a,a,b*b)),
 * c and s by IEEE division, applied as fma(c,x,-(s*y)), fma(s,x,c*y).
 *
 * Pointers: any matrix or vector argument may be a host pointer or a device
 * pointer (the library asks the HIP runtime which).  The library never keeps
 * a caller pointer after a call returns.
 *
 * Status codes are negative on failure; nothing throws across this ABI.
 * One handle is not thread-safe; distinct handles may be used from
 * different threads.  A device fault poisons the handle: every later call on
 * it returns BDU_EDEVICE.
 */
#ifndef BDU_H
#define BDU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bdu_ctx *bdu_handle;
typedef struct bdu_batch_ctx *bdu_batch;

enum {
    BDU_OK = 0,
    BDU_EINVAL = -1,     /* bad shape, NULL argument, or m < n */
    BDU_ENOMEM = -2,     /* device allocation failed or over the memory budget */
    BDU_EDEVICE = -3,    /* a HIP call failed; the handle is poisoned */
    BDU_ENONFINITE = -4, /* a NaN or infinite input was rejected (bdu_set_finite_check) */
    BDU_EBUSY = -5,      /* serving queue full */
    BDU_ESPAN = -6,      /* tracking: r = 1 with b or c in the span of the tracked basis */
    BDU_ESCRATCH = -7    /* bdu_update_noalloc: r (m + n) exceeds bdu_noalloc_capacity() */
};

/* Create a handle from A = Q Bd P^T (eq. bidiag).  Requires m >= n >= 2.
 * Q: m*m doubles, P: n*n doubles, column-major; d: n doubles; e: n-1
 * doubles.  The library copies all four into device memory it owns and
 * builds (or reuses) the rotation schedule for the shape (m, n). */
int bdu_create(int64_t m, int64_t n, const double *Q, const double *d,
               const double *e, const double *P, bdu_handle *out);

/* A <- A + B C^T (eq. main), B m x r and C n x r column-major (leading
 * dimensions m and n), r >= 1: r rank-1 passes of Section 3.4 in column order.
 * Work is queued on the handle's stream; host inputs are copied before the
 * call returns, device inputs must stay valid until the stream reaches the
 * update (bdu_sync). */
int bdu_update(bdu_handle h, const double *B, const double *C, int r);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * update as bdu_update, with the same results bit for bit, but B and C are
 * staged in a fixed device array of bdu_noalloc_capacity() doubles
 * (8 MiB) that the library holds on each device until the process ends,
 * instead of the handle's staging buffers, which bdu_update grows with
 * hipMalloc when r exceeds their capacity.  No allocation or free is made.
 * Requires r (m + n) <= bdu_noalloc_capacity(); BDU_ESCRATCH otherwise,
 * with nothing changed.  Every call on one device shares that device's
 * array, which keeps the last call's contents: calls that overlap on one
 * device (different streams, no synchronization between them) race and
 * must be serialized by the caller.  Call with the handle's device
 * current.  Other errors as bdu_update. */
int bdu_update_noalloc(bdu_handle h, const double *B, const double *C, int r);
int64_t bdu_noalloc_capacity(void);

/* Same as bdu_update on each handle in turn (results are bit-identical to
 * that loop), but every stage of every handle is issued as one launch over
 * all handles (one per applier tiling present).  Handles must be distinct
 * (else BDU_EINVAL); shapes may differ.  The work runs on the first handle's
 * stream and the call returns when it is done.  rs[i] >= 1. */
int bdu_update_batched(const bdu_handle *hs, const double *const *Bs,
                       const double *const *Cs, const int *rs, int count);

/* Batches: the batched form of the update for a fixed set of streams
 * updated step after step (the many-stream use of Section 3.4's update).
 * bdu_batch_create takes `count` distinct handles (shapes may differ) and the
 * largest rank a step will carry; the batch keeps the handles, builds the
 * launch lists once and owns a HIP stream.  bdu_batch_update queues one step:
 * handle i takes the rank-rs[i] update B_i C_i^T (0 <= rs[i] <= max_rank;
 * 0 = no update this step; Bs[i], Cs[i] host or device as in bdu_update).
 * Results are bit-identical to bdu_update on each handle.  From the second
 * step on, a step's launches are captured once in a HIP graph and replayed
 * (not while stage timing is on).  The call returns once host inputs are
 * consumed; bdu_batch_sync waits for the batch stream.  The batch stream
 * does not synchronize implicitly with the null stream (so that capturing
 * its graph never conflicts with null-stream work of other threads): each
 * step is ordered after the work queued on the null stream and on every
 * member's stream before the call, by events.  Later calls on a member
 * handle are ordered after the batch's last step.  The handles must
 * outlive the batch, and must not be destroyed or used by another thread
 * while a step is being queued.  bdu_batch_info fills out[5] = {handles,
 * max_rank, launch groups, graph captured (0/1), steps queued}. */
int bdu_batch_create(const bdu_handle *hs, int count, int max_rank, bdu_batch *out);
/* As bdu_batch_create, with flags: BDU_BATCH_EAGER launches every step
 * eagerly (no graph capture) on the first handle's stream instead of a
 * stream of the batch's own; for callers that queue steps from several
 * threads while other threads also use the device. */
#define BDU_BATCH_EAGER 1
int bdu_batch_create_flags(const bdu_handle *hs, int count, int max_rank, int flags, bdu_batch *out);
int bdu_batch_update(bdu_batch b, const double *const *Bs, const double *const *Cs,
                     const int *rs);
int bdu_batch_sync(bdu_batch b);
int bdu_batch_info(bdu_batch b, int64_t *out);
int bdu_batch_destroy(bdu_batch b);

/* One rank-1 pass from already projected vectors u = Q^T b (m doubles) and
 * v = P^T c (n doubles) (eq. bidiagsubproblem, the right-hand side).  Useful
 * when the caller holds the projections, and to test the rotation stages on
 * their own. */
int bdu_update_projected(bdu_handle h, const double *u, const double *v);

/* Projection only: u = Q^T b (m doubles), v = P^T c (n doubles), as the
 * next update would compute them; u and v may be host or device pointers. */
int bdu_project(bdu_handle h, const double *b, const double *c, double *u,
                double *v);

/* Copy the current factorization out (waits for queued work).  Any output
 * pointer may be NULL to skip it. */
int bdu_read(bdu_handle h, double *Q, double *d, double *e, double *P);

/* Rotations of the most recent pass in schedule order: side[k] = 0 for a
 * left rotation on rows/Q columns (i, i+1), 1 for a right rotation on
 * columns/P columns (i, i+1); idx[k] = i (1-based); c[k], s[k] its
 * coefficients.  Returns the count, or a negative status; writes at most cap
 * entries (any output may be NULL). */
int64_t bdu_last_rotations(bdu_handle h, int32_t *side, int64_t *idx,
                           double *c, double *s, int64_t cap);

/* Run the handle's work on this HIP stream (hipStream_t passed as void*;
 * NULL = the null stream). */
int bdu_set_stream(bdu_handle h, void *stream);
int bdu_sync(bdu_handle h);
int bdu_destroy(bdu_handle h);
const char *bdu_strerror(int status);

/* Device bytes a handle of shape (m, n) holds (factors, projections,
 * rotation streams), for admission control. */
int64_t bdu_footprint_bytes(int64_t m, int64_t n);

/* Applier tiling: chains per wavefront k0 in {6, 12, 18}, compute
 * wavefronts per workgroup nw, matrix rows per lane rpl in {1, 2}.
 * nw in {1, 2, 4, 8} with k0 in {6, 12} (except k0 = 6, nw = 8, rpl = 2):
 * every wavefront also loads or stores the matrix columns it needs.
 * "Staged": nw in {3, 7, 15} with k0 = 12 (rpl = 1 only for 15) and
 * nw in {3, 5, 7} with k0 = 18 (rpl = 1); the workgroup adds one memory
 * wavefront that streams columns and rotation coefficients through LDS for
 * the compute wavefronts.
 * Default (12, 7, 1).  Applies to handles created afterwards.  Results do
 * not depend on it. */
int bdu_set_tiling(int k0, int nw, int rpl);
int bdu_get_tiling(int *k0, int *nw, int *rpl);

/* Autotuning of the applier tiling (its panel width 64 * rpl rows and its
 * block depth k0 * nw chains).  bdu_set_tiling(0, 0, 0) selects "auto": a
 * handle created afterwards takes the tiling recorded for its shape (m, n),
 * else the default.  bdu_autotune times every supported tiling on `streams`
 * synthetic streams of shape (m, n) (Q = I, P = I; the applier's work does
 * not depend on the values), one batched rank-1 step after another, records
 * the fastest for (m, n) and returns out[4] = {k0, nw, rpl, microseconds per
 * step}.  It allocates and frees about `streams` times bdu_footprint_bytes;
 * tilings that do not fit are skipped (BDU_ENOMEM if none fits).
 * bdu_tune_save / bdu_tune_load write / read the recorded table as text
 * lines "m n k0 nw rpl us"; load returns the number of entries read.
 * bdu_handle_tiling reports the tiling a handle was created with. */
int bdu_autotune(int64_t m, int64_t n, int streams, int64_t *out);

/* Where the rotation generator keeps the working band (offsets -2..3) and
 * u, v, about 64 bytes per row: allow = 1 (default) in LDS when they fit
 * (n up to 2449 for square shapes), else in device memory; allow = 0 always in device
 * memory.  Applies to handles created afterwards; results do not depend on
 * it. */
int bdu_set_generation_in_lds(int allow);

/* Split passes: with on >= 1, a handle with n >= 32 whose schedule ends phase 1
 * (Section 3.4: the upper-left chase, with the fold of the remaining rank-1
 * term) at a tick where no rotation chain is in flight generates each pass
 * in parts and applies the phase-1 rotations to Q and P on a stream of its
 * own while the phase-2 rotations are generated; the handle's stream waits
 * for both.  With on = 2 (default) a single handle instead generates the
 * whole pass in segments (bdu_plan_segments), each applied while the next is
 * generated (the generator keeps the carried pairs of chains in flight
 * across a segment end); on = 1 splits only after phase 1.  A batch does the
 * same on a second stream of the batch, for each group of handles (one
 * applier tiling), running as many segments as the group's largest plan
 * has (a handle with fewer has nothing to do in the extra ones).  Same rotations in the same order, so results do not
 * depend on it.  Applies to handles and batches created afterwards. */
int bdu_set_split_pass(int on);

/* Input check: with on = 1, bdu_create, bdu_update, bdu_update_projected,
 * bdu_update_batched and bdu_batch_update scan their inputs (after copying
 * them to the device) and return BDU_ENONFINITE, changing no handle, if any
 * value is NaN or infinite.  Costs one extra pass over the inputs and a
 * stream synchronization per call; off (0) by default. */
int bdu_set_finite_check(int on);
int bdu_tune_save(const char *path);
int bdu_tune_load(const char *path);
int bdu_handle_tiling(bdu_handle h, int *k0, int *nw, int *rpl);

/* Serving (the served form of the update): resident streams admitted
 * against a device-memory budget, bounded per-stream request queues, and
 * continuous batching at the granularity of rank-1 passes (a rank-r request
 * is r passes, Section 3.2, eq. (rk1)).  Streams are grouped in size
 * classes by n; each class has its own worker thread and HIP stream, so the
 * classes' rounds run concurrently and small streams do not wait for the
 * rounds of large ones.  Each round a class's worker takes the next pass of
 * the oldest pending request of up to max_batch of its streams (oldest
 * first) and runs them as one batched rank-1 step, so every stream's passes
 * are applied in submission order and each result is bit-identical to the
 * stream's own sequence of bdu_update calls.  A round lasts one pass, so
 * short requests are not held back by long ones.  A class keeps one batch
 * over all its streams (rank 0 for those without work in a round, launched
 * eagerly), rebuilt only when a stream of the class opens or closes: rounds
 * allocate no device memory.
 *
 * bdu_server_create: budget_bytes of device memory for resident streams
 *   (each costs bdu_footprint_bytes(m, n)), queue_cap requests per stream,
 *   size classes n <= 1024, <= 2048, <= 4096 and larger.
 * bdu_server_create_classes: the same with the classes' ascending upper
 *   bounds of n given (nbounds of them, 0..15, each >= 2; one more class
 *   takes every larger n).
 * bdu_server_class_of: the class (0-based) a stream of n columns joins.
 * bdu_server_open: admit a stream (arguments as bdu_create); BDU_ENOMEM when
 *   the budget would be exceeded (counted, the server is unchanged).
 * bdu_server_submit: queue A_s <- A_s + B C^T (B m x r, C n x r, host or
 *   device; copied before returning).  BDU_EBUSY when the stream's queue
 *   holds queue_cap requests (counted, nothing queued).  ticket may be NULL
 *   (nobody waits; the request is released when done); otherwise the ticket
 *   must be waited for once, which releases it.
 * bdu_server_wait: block until the request is done; its latency (submit to
 *   completion) in ms.  bdu_server_poll: 1 done, 0 pending.
 * bdu_server_drain: wait until no request is queued or running.
 * bdu_server_pause: 1 stops the workers from starting rounds, 0 resumes.
 * bdu_server_read / bdu_server_close: wait until the stream has no queued or
 *   running request, then read (as bdu_read) / destroy it and return its
 *   budget (requests submitted to a stream while it closes fail with
 *   BDU_EINVAL).  Both fail (BDU_EINVAL) on a paused server with queued
 *   requests.
 * bdu_server_stats: counts[9] = {completed, rejected busy, rejected for
 *   memory, rounds, passes run in rounds, open streams, budget bytes in
 *   use, requests pending, failed}; latency[4] = {p50, p99, mean, max} in ms
 *   over completed requests.  bdu_server_reset_stats zeroes the counters
 *   and the latency record (streams and queues stay).
 * bdu_server_destroy: runs what is queued (unless paused), stops the
 *   workers and destroys every stream; no call on the server may be in
 *   progress. */
typedef struct bdu_server_ctx *bdu_server;
int bdu_server_create(int64_t budget_bytes, int queue_cap, int max_batch, bdu_server *out);
int bdu_server_create_classes(int64_t budget_bytes, int queue_cap, int max_batch, const int64_t *bounds,
                              int nbounds, bdu_server *out);
int bdu_server_class_of(bdu_server s, int64_t n);
int bdu_server_open(bdu_server s, int64_t m, int64_t n, const double *Q, const double *d,
                    const double *e, const double *P, int *stream_id);
int bdu_server_submit(bdu_server s, int stream_id, const double *B, const double *C, int r,
                      int64_t *ticket);
int bdu_server_wait(bdu_server s, int64_t ticket, double *latency_ms);
int bdu_server_poll(bdu_server s, int64_t ticket);
int bdu_server_drain(bdu_server s);
int bdu_server_pause(bdu_server s, int paused);
int bdu_server_read(bdu_server s, int stream_id, double *Q, double *d, double *e, double *P);
int bdu_server_close(bdu_server s, int stream_id);
int bdu_server_stats(bdu_server s, int64_t *counts, double *latency);
int bdu_server_reset_stats(bdu_server s);
int bdu_server_destroy(bdu_server s);

/* Stage timing.  bdu_timing_enable(1) clears the log and brackets every
 * later kernel launch with HIP events on the stream the kernel runs on;
 * bdu_timing_enable(0) stops it.  bdu_timing_read waits for the logged events
 * and returns, per stage (0 projection, 1 spike, 2 generation, 3 application),
 * the summed milliseconds ms[4] and the number of launches launches[4]. */
int bdu_timing_enable(int on);
int bdu_timing_read(double *ms, int64_t *launches);

/* The device rotation generator of eq. (giv1) on count pairs (a[i], b[i]):
 * mode 1 annihilates a, mode 2 annihilates b; outputs c, s and the
 * survivor r.  Host or device pointers.  For checking the device arithmetic
 * (IEEE sqrt and division) against a reference. */
int bdu_givens_device(const double *a, const double *b, int mode, double *c,
                      double *s, double *r, int64_t count);

/* ---- orthogonality monitor and correction ----------------------------- */

/* Over a long stream of updates the accumulated rotations leave Q and P
 * orthogonal only up to rounding; the paper reorthogonalizes its factors a
 * few times without saying how.  Drift of a factor X: ||X^T X - I||_F,
 * computed on the FP64 matrix cores (the sums' order is not fixed: results
 * agree with a plain fp64 product to within the rounding of a length-m dot
 * product).  eq / ep (either may be NULL) receive the drift of Q and P.
 * Synchronizes the handle's stream.  BDU_ENOMEM if the scratch (about
 * 8 max(m,n)^2 + 8 ld m bytes, allocated on first use and kept) does not
 * fit. */
int bdu_orth_error(bdu_handle h, double *eq, double *ep);

/* Measure the drift as above and, for each factor whose drift exceeds tol
 * (every factor if tol <= 0), take one Newton-Schulz step
 * X <- X - X (X^T X - I) / 2 towards its orthogonal polar factor (the
 * nearest orthogonal matrix): from drift e it leaves a drift of order e^2,
 * and the represented matrix Q Bd P^T moves by O(e) ||A||.  eq / ep receive
 * the drift measured before the step. */
int bdu_reorthogonalize(bdu_handle h, double tol, double *eq, double *ep);

/* ---- truncated bidiagonal approximation (Section 1.3) ----------------- */

/* The best rank-r truncated bidiagonal approximation of the handle's
 * A = Q Bd P^T (eqs. (trBD), (errtrBD)): keep the r columns i of Bd (0-based)
 * with the largest t_i = d_i^2 + e_{i-1}^2 (e_{-1} = 0; each product and
 * the sum rounded on their own; ties keep the lower index), in order of
 * decreasing t.  idx (r, int64) receives those columns, err2 the exact
 * squared Frobenius error (the dropped t_i summed in increasing i from 0),
 * Qr (m x r) the columns d_i q_i + e_{i-1} q_{i-1} and Pr (n x r) the columns
 * p_i, so that A_r = Qr Pr^T.  Any output may be NULL; host or device
 * pointers.  1 <= r <= n.  Synchronizes the handle's stream. */
int bdu_truncated_bd(bdu_handle h, int64_t r, int64_t *idx, double *err2, double *Qr, double *Pr);

/* ---- Householder bidiagonal update (Section 3.3) ---------------------- */

/* The paper's second update method, BHU (Algorithm 1 on the compact
 * representation of Theorem 1, with eqs. (house), (TR), (QP)): replaces the
 * handle's A = Q Bd P^T by Q+ Bd+ P+^T = A + b c^T, where Bd+ is the
 * Householder bidiagonalization of Bd + (Q^T b)(P^T c)^T computed without
 * forming that matrix, Q+ = Q Q_k and P+ = P P_k.  b: m doubles, c: n
 * doubles, host or device.  Reflectors H = I - 2 y y^T with unit y and
 * leading value -sign(x_1) ||x|| (sign(0) = +1); the identity where the
 * entries to annihilate are already zero; left reflectors on columns 1..n-1
 * (m = n) or 1..n (m > n), right ones on rows 1..n-2 (so the first column of
 * P is kept).  Not bit-identical to a CPU run: products are summed in a
 * different order, and agreement is within a tolerance.  Device scratch of
 * (3 ldq + 3 ldp) n + 10 ldq + 2 ldp + 64 doubles (ldq, ldp = m, n rounded
 * up to 128) is allocated on the first call and kept by the handle
 * (BDU_ENOMEM if it does not fit).  Errors: BDU_EINVAL (null argument),
 * BDU_ENONFINITE (with the input check on), BDU_EDEVICE.  Stream-ordered on
 * the handle's stream. */
int bdu_update_householder(bdu_handle h, const double *b, const double *c);

/* ---- subspace tracking (Section 4, eqs. (lrup)-(bdlrup)) ------------ */

/* A thin rank-r factorization A = U B V^T (U m x r and V n x r with
 * orthonormal columns, B upper bidiagonal r x r) tracked under rank-1
 * updates A + b c^T, kept at rank r. */
typedef struct bdu_track_ctx *bdu_track;

/* U (m x r), V (n x r): column-major, leading dimension m (n); d r entries,
 * e r-1 (may be NULL when r = 1).  Host or device pointers; the library
 * keeps device copies.  Requires 1 <= r <= m, r <= n.
 * BDU_EINVAL for bad sizes or NULL inputs, BDU_ENOMEM, BDU_EDEVICE;
 * BDU_ENONFINITE with the input check on. */
int bdu_track_create(int64_t m, int64_t n, int64_t r, const double *U, const double *d,
                     const double *e, const double *V, bdu_track *out);

/* One tracking update with b (m) and c (n), host or device.
 * Complements (eq. (defup)): b_hat = U^T b, b_perp = b - U b_hat; row sums
 *   run in chunks of 256 rows (a sequential fma from 0 inside a chunk, rows
 *   ascending, the chunk partials added in ascending order from 0) and
 *   (U b_hat)_i = sum_j U(i,j) b_hat_j as fma, j ascending.  With s0 = b^T b
 *   and s1 = b_perp^T b_perp: if 2 s1 < s0 a second pass projects b_perp
 *   again (b_hat += U^T b_perp, b_perp -= U (U^T b_perp), s2 its squared
 *   norm).  delta = sqrt(s1) after one pass, sqrt(s2) after two if
 *   2 s2 >= s1, else 0: b lies in span(U) to working precision (the "twice
 *   is enough" test of Kahan and Parlett).  delta is also 0 when its square
 *   would be at most tau^2 s0, tau = m 2^-53 (the worst-case rounding error
 *   of the projection sums).  The same for c, V (tau = n 2^-53) and gamma.
 * A side with a positive norm is augmented by its unit complement (eq.
 *   (qrlr)); the middle matrix (eq. (equivlrup)) is
 *     both sides:  [B 0; 0 0] + [b_hat; delta][c_hat; gamma]^T, (r+1)^2;
 *     left only:   [B; 0] + [b_hat; delta] c_hat^T, (r+1) x r;
 *     right only:  [B 0] + b_hat [c_hat; gamma]^T, run as its transpose with
 *                  rows and columns reversed (upper bidiagonal plus rank 1,
 *                  (r+1) x r);
 *     neither:     B + b_hat c_hat^T, r x r;
 *   one BGU pass (bdu_update_projected) from identity factors gives
 *   Q2 Bbar P2^T.
 * Both sides augmented: the row and column k of Bbar with the smallest
 *   column norm are removed (d_k^2 + e_{k-1}^2 as fma(d_k, d_k, e_{k-1}
 *   e_{k-1}); ties: the highest k; the superdiagonal entry joining k-1 and
 *   k+1 becomes 0).  Otherwise the result is exactly rank r and nothing is
 *   removed (the paper's unaugmented case after eq. (bdlrup)).
 * U <- [U, b_perp/delta] Q2(:, kept), V <- [V, c_perp/gamma] P2(:, kept),
 *   each entry a sequential fma over U's (V's) columns in order, the
 *   appended column last and absent on an unaugmented side (eq. (bdlrup));
 *   in the reversed case U <- U J P2 J and V <- [V, c_perp/gamma] diag(J, 1)
 *   Q2(:, 1:r) J, J the reversal of r entries, and d, e are reversed back.
 * BDU_ESPAN, changing nothing, when r = 1 and a side is not augmented (a
 * 2 x 1 or 1 x 1 middle matrix has no BGU pass).  Inputs are consumed
 * before returning; the work is queued on the tracker's stream. */
int bdu_track_update(bdu_track t, const double *b, const double *c);

/* Wait for the tracker's queued work. */
int bdu_track_sync(bdu_track t);

/* Copy the tracked factors out (any pointer may be NULL; host or device). */
int bdu_track_read(bdu_track t, double *U, double *d, double *e, double *V);

/* delta, gamma and the removed index (0-based, of the r+1 columns; -1 when
 * a side was not augmented) of the last successful update; BDU_EINVAL
 * before the first one. */
int bdu_track_last(bdu_track t, double *delta, double *gamma, int64_t *dropped);

/* The last successful update's projections b_hat, c_hat (r each) and unit
 * complements b_perp/delta (m) and c_perp/gamma (n; unspecified on a side
 * that was not augmented).  Any pointer may be NULL; host or device.
 * BDU_EINVAL before the first update.  Lets a caller check the update
 * from its inputs (the rest of the update depends only on these, delta
 * and gamma). */
int bdu_track_last_projection(bdu_track t, double *bh, double *ch, double *qb, double *qc);

/* Orthogonality of the tracked factors (Section 4.2: the products of the
 * thin factors with the middle factors lose orthogonality slowly, and the
 * paper checks for that periodically and reorthogonalizes a few times).
 * eu / ev (either may be NULL) receive ||U^T U - I||_F and ||V^T V - I||_F,
 * computed on the FP64 matrix cores as bdu_orth_error does for Q and P.
 * Synchronizes the tracker's stream.  Scratch of about
 * 16 max(m, n) r + 8 r^2 bytes is allocated on first use and kept. */
int bdu_track_orth_error(bdu_track t, double *eu, double *ev);

/* Measure as above and, on each side whose drift exceeds tol (every side
 * if tol <= 0), take one Newton-Schulz step X <- X - X (X^T X - I) / 2
 * (the step of bdu_reorthogonalize).  eu / ev receive the drift measured
 * before the step. */
int bdu_track_reorthogonalize(bdu_track t, double tol, double *eu, double *ev);

/* The periodic check: after every period-th successful bdu_track_update
 * (counted from this call), bdu_track_reorthogonalize(t, tol, ...) runs on
 * the tracker's stream and the update then synchronizes.  period = 0 turns
 * the check off (the default).  BDU_EINVAL for period < 0 or a NaN tol. */
int bdu_track_set_drift_check(bdu_track t, int64_t period, double tol);

/* Checks run so far, sides corrected so far, and the drift of U and V
 * measured by the last check (before its correction).  Any pointer may be
 * NULL. */
int bdu_track_drift_stats(bdu_track t, int64_t *checks, int64_t *corrections, double *eu, double *ev);

int bdu_track_destroy(bdu_track t);

/* ---- schedule inspection (host only, no device needed) ---------------- */

/* Statistics of the rotation schedule for (m, n) under the current tiling:
 * out[0] left rotations, out[1] right rotations, out[2] spike rotations,
 * out[3] generation chains, out[4] generation ticks, out[5] left stream
 * slots, out[6] right stream slots, out[7] generation threads, out[8] the
 * tick where a split pass ends its first part (0: passes do not split).
 * out holds 9 values. */
int bdu_plan_stats(int64_t m, int64_t n, int64_t *out);

/* The schedule in order as the device decodes it: side, first index (1-based),
 * phase (0 spike, 1, 2) and the generation tick of each rotation (spike
 * rotations get tick -1).  The fold step appears once, in its place, with
 * side 2, index N-1 and phase 3.  Writes at most cap entries and returns the
 * total count. */
int64_t bdu_plan_rotations(int64_t m, int64_t n, int32_t *side, int64_t *idx,
                           int32_t *phase, int64_t *tick, int64_t cap);

/* Segments of a single-handle pass: returns their number (0: none, at most
 * 8); segment k generates the ticks below tcut[k] not generated before, and
 * then its application runs over the applier blocks below bcut[k] not
 * applied before (phase-1 blocks first, then phase-2 blocks; the first
 * segment also applies the spike).  block (optional, at most cap entries)
 * receives the applier block of each rotation in the order of
 * bdu_plan_rotations (numbered the same way, on either side; -1 for spike
 * rotations and the fold). */
int bdu_plan_segments(int64_t m, int64_t n, int32_t *tcut, int32_t *bcut, int32_t *block, int64_t cap);

/* The applier blocks of one side (0: Q, the left rotations; 1: P) for (m, n)
 * under the current tiling, phase-1 blocks first: six values per block in
 * out (at most cap blocks): base, lmax (-1: empty), nfront, phase, start
 * and off as the kernels read them (the block's local column lam is matrix
 * column base - 1 - lam in phase 1 and base - 1 + lam in phase 2; start is
 * the staged applier's first chunk of k0 + 3 fronts of the block, off its
 * first slot in the side's rotation stream).  Returns the number of blocks,
 * or BDU_EINVAL. */
int bdu_plan_blocks(int64_t m, int64_t n, int side, int64_t *out, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
