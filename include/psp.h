/*
 * psp.h - C ABI of libpsp, an MI355X (gfx950) solver for the free-space
 * Poisson problem  -Lap u = rho  on R^3 with u -> 0 at infinity, by the
 * near-field-free super-potential Gaussian-sum FFT method of Exl & Schaffer
 * (Section 1, eq. problem1 and conv; Section 2).
 *
 * What a solve computes (Algorithm 2, eq. convtheorem):
 *   rho, sampled on an n^3 grid of spacing h, is zero-padded to (2n)^3; a
 *   forward 3D DFT is taken; each mode k is multiplied by
 *       m_k = -(2 pi / L)^2 |k|^2 Vhat_k / (2n)^3,      L = 2 n h,
 *   where Vhat_k is the Fourier integral of the Gaussian-sum approximation
 *   of the biharmonic kernel |y|/(8 pi) over the box [-L/2, L/2]^3
 *   (eq. gs_x, Gten0, Gten_sep); an inverse DFT (no scaling) follows and
 *   the first n points of every axis are returned as u.
 *   On a rectangular box or grid (psp_plan_create_box, psp_plan_create_grid)
 *   axis p has its own n_p, h_p and L_p = 2 n_p h_p: |k|^2 / L^2 becomes
 *   sum_p k_p^2 / L_p^2, (2n)^3 becomes 8 n_1 n_2 n_3, and the kernel is
 *   truncated to the box of sides L_p.
 *   The operator is translation invariant, so no grid origin is needed.
 *
 * Conventions shared by every entry point:
 *   - Arrays rho and u are C-ordered n*n*n (n1*n2*n3 for a plan from
 *     psp_plan_create_grid), element [i1][i2][i3] at (i1*n2 + i2)*n3 + i3,
 *     i3 contiguous, in the plan's dtype (double for
 *     PSP_F64, float for PSP_F32), in device memory of the current HIP
 *     device, at least 16-byte aligned.  The caller owns them.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Solves are asynchronous on that stream; a kernel-side failure is
 *     reported by a later call or by stream synchronisation.
 *   - No exception crosses the ABI.  Every call returns a psp_status;
 *     psp_last_error() gives a thread-local detail string for the last
 *     non-OK status returned on this thread.
 *   - The library owns plans, workspaces, cached kernel spectra and servers.
 */
#ifndef PSP_H
#define PSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psp_plan psp_plan;       /* opaque, library owned */
typedef struct psp_server psp_server;   /* opaque, library owned */

/* Precision tier.  PSP_F32 keeps the kernel spectrum and the Gaussian-sum
 * data in FP64 and runs the FFT passes and the multiply in FP32: twiddles
 * and multiplier entries are the FP64 values rounded once to FP32. */
#ifdef __cplusplus
/* int-sized in C++ too, so that any value a C caller passes is a value of
 * the type (the library rejects the unknown ones) */
#define PSP_ENUM_INT : int
#else
#define PSP_ENUM_INT
#endif
typedef enum PSP_ENUM_INT { PSP_F64 = 0, PSP_F32 = 1 } psp_dtype;

typedef enum PSP_ENUM_INT {
    PSP_OK = 0,
    PSP_EINVAL = -1,        /* bad argument (h <= 0, R < 1, NULL pointer ...) */
    PSP_ENOMEM = -2,        /* device or host allocation failed, or over budget */
    PSP_EUNSUPPORTED = -3,  /* n odd, out of [4, 384] or 2n not 2^a 3^b,
                               or an entry point a grid plan cannot use */
    PSP_ESTATE = -4,        /* call order (solve before precompute ...) */
    PSP_EHIP = -5,          /* a HIP runtime call failed */
    PSP_EBUSY = -6,         /* server queue full; request already on the device */
    PSP_ECANCELED = -7      /* request withdrawn by psp_serve_cancel */
} psp_status;

/* ---- plans (Algorithm 1) -------------------------------------------------
 * psp_plan_create: validates (n, h, R, dtype) and computes the R Gaussian-sum
 * weights and exponents on the host (Section 2, eq. sin_1_x: sinc quadrature
 * of 1/(8 pi r) on (eps, delta] with eps = 1e-4 * n h and
 * delta = sqrt(3) * n h).  Host work only; no device memory is touched.
 * n: points per axis, even, 4 <= n <= 384, with 2n = 2^a 3^b (Algorithm 1
 * takes any grid size; the FFT passes are built for every such length:
 * n = 4, 6, 8, 12, 16, 18, 24, 32, 36, 48, 54, 64, 72, 96, 108, 128, 144,
 * 162, 192, 216, 256, 288, 324, 384); h > 0 finite; 1 <= R <= 2048.
 * Other n: PSP_EUNSUPPORTED.
 * *out receives the plan (NULL on failure). */
psp_status psp_plan_create(int n, double h, int R, psp_dtype dtype, psp_plan **out);

/* As psp_plan_create with an explicit cutoff 0 < eps < delta (finite). */
psp_status psp_plan_create_ex(int n, double h, int R, psp_dtype dtype,
                              double eps, double delta, psp_plan **out);

/* A rectangular box (Section 3, Tables 4, 6, 8): n points per axis with
 * spacing h[p] along axis p (h: 3 host doubles, axis 1 = the slowest index
 * i1 of rho[i1][i2][i3]).  The padded box has sides L_p = 2 n h_p, the
 * kernel is truncated to it, the 1D integrals of eq. Gten_sep are taken per
 * axis and the spectral Laplacian is -(2 pi)^2 sum_p k_p^2 / L_p^2.
 * eps <= 0 and delta <= 0 select the defaults eps = 1e-4 max_p(L_p/2) and
 * delta = |(L_1, L_2, L_3)|/2; otherwise 0 < eps < delta (finite).  The
 * solve itself is the same as for a cubic box; everything else follows
 * psp_plan_create (same errors, plus PSP_EINVAL for h == NULL). */
psp_status psp_plan_create_box(int n, const double *h, int R, psp_dtype dtype,
                               double eps, double delta, psp_plan **out);

/* The general grid (Algorithm 1 takes a point count and a spacing per
 * axis): n[p] points and spacing h[p] along axis p (n, h: 3 host values;
 * each n[p] as for psp_plan_create).  rho and u are n[0] x n[1] x n[2],
 * C-order.  Defaults as for psp_plan_create_box, with L_p = 2 n_p h_p.
 * With unequal counts every pass runs at its own axis's padded length and
 * takes the tuned shape of a cube of that size.  Such plans solve through
 * psp_solve, psp_graph_capture and, beside cubic plans, psp_solve_batched
 * and psp_graph_capture_batched (each grid with its own launch sequence);
 * psp_solve_padded_debug, psp_autotune, psp_plan_set_shape,
 * psp_profile_enable and k3 chunks / i1 groups return PSP_EUNSUPPORTED for
 * them.  Equal counts give the psp_plan_create_box
 * plan. */
psp_status psp_plan_create_grid(const int *n, const double *h, int R, psp_dtype dtype,
                                double eps, double delta, psp_plan **out);

/* Algorithm 1 steps 2-3 on the current device, on `stream`: the 2 R (n+1) 1D
 * integrals of eq. Gten_sep (FP64 with double-double node phases: closed
 * forms for narrow Gaussians, 15-point Gauss-Kronrod on equal panels
 * otherwise), the kernel-spectrum multiplier octant (n+1)^3 by an FP64 MFMA
 * contraction, FFT twiddle tables.  Idempotent.  Multiplier octants are shared between plans with the
 * same (n, h, R, eps, delta) on the same device.  Synchronises `stream`. */
psp_status psp_kernel_precompute(psp_plan *p, void *stream);

/* Algorithm 2: u = crop(IFFT(m * FFT(pad(rho)))).  rho and u must not alias.
 * Uses a library-owned workspace bound to (plan, stream), allocated on the
 * first call with that stream.  Returns PSP_ESTATE before precompute. */
psp_status psp_solve(const psp_plan *p, const void *rho_dev, void *u_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of psp_solve, with the same kernels and bitwise the same result, whose two
 * intermediates live in a fixed array of 128 MiB (134217728 bytes) that the
 * library holds on every GPU it runs on until the process ends, instead of
 * a workspace allocation.  Allocates nothing (no hipMalloc, hipFree or
 * allocating library call); the caller passes rho and u as for psp_solve.
 * PSP_ENOMEM if the plan's intermediates do not fit the array (for a cube:
 * n <= 128 in FP64, n <= 162 in FP32; see psp_plan_workspace_bytes),
 * PSP_ESTATE before precompute, PSP_EINVAL for NULL or aliased pointers or
 * another current device.  Every call on one GPU uses that GPU's array:
 * calls whose solves overlap on the device (other streams, other threads)
 * race and give undefined results; calls on one stream are ordered and
 * safe.  Nothing in the array needs to start at zero. */
psp_status psp_solve_noalloc(const psp_plan *p, const void *rho_dev, void *u_dev, void *stream);

/* `count` (<= 65535) independent solves: one launch per pass for each
 * distinct n in the batch (the pass kernels read each solve's pointers from
 * a device job table).  plans may differ in n (and h, R) but must share one
 * dtype and device and all be precomputed; rho_dev[i] and u_dev[i] follow
 * plans[i].  Grid plans with unequal counts per axis run after the cubic
 * ones, each with its own per-axis launch sequence.  Results are bitwise
 * equal to psp_solve of the same plan and rho.  Workspaces (one per cubic
 * solve of the batch, one per distinct grid) are library-owned, bound to the
 * stream and reused by later batches on it. */
psp_status psp_solve_batched(int count, const psp_plan *const *plans,
                             const void *const *rho_dev, void *const *u_dev,
                             void *stream);

/* How batches (psp_solve_batched, psp_graph_capture_batched and the serving
 * loop) launch their passes, process-wide, for batches started afterwards:
 * 0 (default): one launch per pass per distinct (n, shape);
 * 1: persistent kernels, one launch per pass for all solves with 2n <= 256
 *    (workgroups of 384 threads take work items from an atomic counter in
 *    the batch's device table until none is left) and no radix-16 plan,
 *    grouped launches for the rest;
 * 2: as 1 with one workgroup per work item instead of persistent ones.
 * Results are bitwise the same in every mode.  PSP_EINVAL for another value. */
psp_status psp_set_batch_mode(int mode);

/* Test hook: the uncropped (2n)^3 result of Algorithm 2 (real part), C-order
 * with side 2n, dtype of the plan.  PSP_EUNSUPPORTED for grids with unequal
 * counts and for plans whose workspace psp_plan_set_tuning shrank. */
psp_status psp_solve_padded_debug(const psp_plan *p, const void *rho_dev, void *upad_dev,
                                  void *stream);

/* Debugging of out-of-bounds writes: with enable != 0, every workspace
 * allocated afterwards (plans, batches, graphs, the serving loop) places its
 * two intermediates 64 KB into their allocations, between 64 KB bands filled
 * with the byte 0xA5.  psp_plan_check_guards synchronises the device and sets
 * *intact = 1 if every band of the plan's workspaces still holds the pattern
 * (0 otherwise; workspaces allocated without guards are skipped). */
psp_status psp_debug_guards(int enable);
psp_status psp_plan_check_guards(psp_plan *p, int *intact);

/* Test hook: copies the R weights w_s and exponents a_s (host arrays). */
psp_status psp_plan_get_gs(const psp_plan *p, double *omega, double *alpha);

/* Test hook: computes the 1D tables J0[s][k], J2[s][k], s < R, k <= n, on
 * the current device (the plan's device once precomputed) exactly as the
 * precompute does and copies them to host memory (row-major R x (n+1)
 * each; axis 1's tables for a rectangular box).  Needs a GPU; synchronises
 * the device's null stream. */
psp_status psp_plan_get_tables(psp_plan *p, double *J0, double *J2);

/* Test hook: copies the device multiplier octant m[a][b][c] (a <= n1,
 * b <= n2, c <= n3; row-major (n1+1)(n2+1)(n3+1) doubles, (n+1)^3 for a
 * cube) to host memory.  Needs precompute; syncs. */
psp_status psp_plan_get_multiplier(psp_plan *p, double *m_host);

/* Tuning of single solves (batched solves and graphs use the defaults).
 * k3_tiles > 0: the forward i2, fused i1 and inverse i2 passes run over the
 *   half-spectrum axis k3 in chunks of k3_tiles tiles (8 bins per tile in
 *   FP64, 16 in FP32), with a chunk-sized padded intermediate.
 * i1_group > 0 (with one chunk): the forward i3 -> i2 and inverse i2 -> i3
 *   passes run over groups of i1_group slabs, with a group-sized i3
 *   intermediate that can stay in the last-level cache between the two.
 * 0, 0 (the default) is one chunk and no grouping.  Frees the plan's
 * workspaces; call it while no solve of this plan is in flight. */
psp_status psp_plan_set_tuning(psp_plan *p, int k3_tiles, int i1_group);

/* Launch shape of the five passes H1..H5 (index 0..4), the autotuner's search
 * space, as two int[5] arrays:
 *   plan[i]: radix plan of pass i: 0 the default factorisation of 2n, 1 an
 *            alternative for 2n in {128, 256, 384, 512, 768}, 2 a radix-16
 *            factorisation for 2n in {128, 192, 256, 384, 512} or a radix-12
 *            one for 768 (other lengths have only 0);
 *   tile[i]: passes 0 and 4 (transforms along i3): workgroup size, 0: 256
 *            threads, 1: 128, 2: 512, 3: 64, 4..7: 0..3 with nontemporal
 *            stores of the pass's output; passes 1..3 (along i2, i1, i2): 0: one
 *            128-byte row of k3 columns per workgroup (8 FP64 or 16 FP32
 *            columns), 1: half of one, 2: one row with the exchanges between
 *            FFT stages through half-size LDS buffers by position half,
 *            3: one row with half the threads per column (two butterflies
 *            per thread and stage), 4: 2 and 3 together, 5: one row with the
 *            exchanges through half-size LDS buffers by column half, 6: 5 and
 *            3 together; 7..13: 0..6 with nontemporal accesses (pass 1
 *            its stores of the intermediate, pass 2 its stores, pass 3 its
 *            loads of the intermediate and its stores); pass 2 also
 *            14..20: 0..6 with nontemporal loads and stores.
 * A tile choice changes only which workgroup transforms which column, how
 * values move between stages and the accesses' cache policy: the results
 * are bitwise the same.  A radix plan changes the rounding, not the
 * accuracy class.  Batched solves and graphs group their members by (n,
 * shape).  Set: PSP_EINVAL for a value out of range; call it while no solve
 * of this plan is in flight.  Get: copies the plan's current shape. */
psp_status psp_plan_set_shape(psp_plan *p, const int *plan, const int *tile);
psp_status psp_plan_get_shape(const psp_plan *p, int *plan, int *tile);

/* The process-wide tuning table: the shape that plans of (n, dtype) created
 * afterwards start with (and the serving loop's plans use).  Unset entries
 * give the default shape (all zeros).  psp_tuning_get reports it. */
psp_status psp_tuning_set(int n, psp_dtype dtype, const int *plan, const int *tile);
psp_status psp_tuning_get(int n, psp_dtype dtype, int *plan, int *tile);

/* Autotuner: times every (radix plan, tile) candidate of every pass on this
 * plan's own workspace on `stream` (two inputs, a hashed pseudo-random density
 * and a smooth compactly supported bump; `reps` timed solves per candidate
 * round and input after one warm-up, median over the repetitions on both,
 * HIP events around each launch), picks per pass the fastest candidate (the
 * default unless another is at least 1% faster), then for each pass in turn
 * times its four fastest candidates and the other cache policies of its pick
 * as whole solves inside that pick (the sum of the two inputs' medians over
 * `reps` solves each; a cache policy can slow its own pass and speed up the
 * next) and keeps one that is more than 0.2% faster, sets the result as the
 * plan's shape and enters it in the tuning table.  Outputs (host arrays, each may be
 * NULL): best_plan[5], best_tile[5], best_ms[5] the chosen candidate and
 * that pass's time in ms; cand_ms[5 * 63]: the time of candidate
 * (plan, tile) of pass i at cand_ms[i * 63 + plan * 21 + tile], -1 where the
 * candidate does not exist.  Allocates three n^3
 * buffers for the duration; synchronises `stream`.  PSP_ESTATE before
 * precompute or while profiling; PSP_EINVAL for reps outside [1, 1000]. */
psp_status psp_autotune(psp_plan *p, int reps, void *stream, int *best_plan, int *best_tile,
                        float *best_ms, float *cand_ms);

/* Bytes of device workspace one solve of this plan needs (per stream). */
psp_status psp_plan_workspace_bytes(const psp_plan *p, size_t *bytes);

/* Bytes of the plan's device multiplier octant. */
psp_status psp_plan_spectrum_bytes(const psp_plan *p, size_t *bytes);

/* Per-pass device timing.  psp_profile_enable makes the next `max_solves`
 * psp_solve calls of this plan record 6 HIP events on their own stream:
 * before each of the 5 passes (forward i3, forward i2, fused i1 with the
 * multiply, inverse i2, inverse i3) and after the last.  psp_profile_read
 * waits for them and returns the number of recorded solves and the average
 * milliseconds of each pass (pass_ms[0..4]) and of the whole solve
 * (pass_ms[5]); it then clears the recording.  pass_ms has 6 entries. */
psp_status psp_profile_enable(psp_plan *p, int max_solves);
psp_status psp_profile_read(psp_plan *p, int *count, double *pass_ms);

/* Measured ceilings of the current device, for rooflines: the rate of a
 * streaming copy from buf_a to buf_b (bytes each, device memory owned by
 * the caller, >= 1 MiB, a multiple of 16; counts bytes read plus written)
 * in GB/s, and the FP64 matrix-core rate of back-to-back independent
 * 16x16x4 FP64 MFMA instructions in TFLOP/s; best of 5 timed runs each on
 * `stream`.  Allocates nothing; synchronises `stream`; overwrites buf_b. */
psp_status psp_device_peaks(void *buf_a, void *buf_b, size_t bytes, void *stream,
                            double *copy_gbps, double *fp64_mfma_tflops);

void psp_plan_destroy(psp_plan *p);

/* ---- captured solves (hipGraph) -------------------------------------------
 * psp_graph_capture records one solve of (plan, rho_dev, u_dev) as a HIP graph
 * with its own workspace; psp_graph_launch replays it on `stream` (one host
 * call for all passes).  psp_graph_capture_batched does the same for a
 * batch (as psp_solve_batched; the graph owns the workspaces and the device
 * job table).  Replays of one graph must not overlap each other; the graph
 * keeps pointers to rho/u and to the plans' spectra, which must outlive it.
 * Capture synchronises `stream`. */
typedef struct psp_graph psp_graph;
psp_status psp_graph_capture(const psp_plan *p, const void *rho_dev, void *u_dev, void *stream, psp_graph **out);
psp_status psp_graph_capture_batched(int count, const psp_plan *const *plans, const void *const *rho_dev,
                                     void *const *u_dev, void *stream, psp_graph **out);
psp_status psp_graph_launch(psp_graph *g, void *stream);
void psp_graph_destroy(psp_graph *g);

/* ---- serving --------------------------------------------------------------
 * A continuous-batching request loop.  Requests are admitted while their
 * device footprint (workspace plus, on a spectrum-cache miss, the multiplier
 * octant) fits `hbm_budget_bytes` and fewer than `max_slots` are in flight;
 * admitted requests are grouped per tier and size class (n <= 128 or larger)
 * into batched launches on the least busy stream of a small pool, so new
 * arrivals overlap work already on the device.  Spectra
 * are cached per (n, h, R) on the device in LRU order inside the budget.
 * rho_dev/u_dev stay caller-owned and must live until the request is done;
 * rho must be fully written (its producing work complete) when submitted,
 * since the loop reads it on its own streams.  The server uses five streams
 * (two per size class and one for spectrum precomputes); small requests are
 * kept from waiting in order behind large ones only while those streams have
 * hardware queues of their own, so run the process with GPU_MAX_HW_QUEUES
 * of at least 8 (HIP's default of 4 makes streams share queues). */
psp_status psp_serve_create(size_t hbm_budget_bytes, int max_slots, psp_server **out);

/* Non-blocking enqueue; *ticket identifies the request.  PSP_EBUSY if the
 * queue holds 65536 requests; PSP_ENOMEM if one request alone exceeds the
 * budget; validation errors as psp_plan_create. */
psp_status psp_serve_submit(psp_server *sv, int n, double h, int R, psp_dtype tier,
                            const void *rho_dev, void *u_dev, uint64_t *ticket);

/* Withdraw a request that is still queued: it completes at once with result
 * PSP_ECANCELED and u is not written.  PSP_EBUSY if it has already been
 * admitted to the device (it then completes normally), PSP_EINVAL for an
 * unknown or finished ticket. */
psp_status psp_serve_cancel(psp_server *sv, uint64_t ticket);

/* Non-blocking status: *done = 1 once u is complete on the device; then
 * *result is the request's status and *latency_ms its submit-to-completion
 * time.  The server keeps the outcome of the most recent 2^20 completed
 * requests; an older or unknown ticket gives PSP_EINVAL.  Any output pointer
 * may be NULL. */
psp_status psp_serve_poll(psp_server *sv, uint64_t ticket, int *done, psp_status *result,
                          double *latency_ms);

/* Blocks until every submitted request is complete. */
psp_status psp_serve_drain(psp_server *sv);

/* Device bytes the server holds now and the most it has held. */
psp_status psp_serve_stats(psp_server *sv, size_t *bytes_in_use, size_t *bytes_peak,
                           uint64_t *completed, uint64_t *cache_hits, uint64_t *cache_misses);

/* Drains, then frees everything the server owns. */
void psp_serve_destroy(psp_server *sv);

/* ---- errors ---------------------------------------------------------------*/
const char *psp_strerror(psp_status e);
const char *psp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PSP_H */
