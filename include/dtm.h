/*
 * dtm.h -- dead-time Markov stationary PDFs for asynchronous single-photon
 * LiDAR on AMD Instinct MI355X (gfx950).
 *
 * The library implements the accelerated Markov pipeline of Zhang,
 * Weerasooriya, Chennuri and Chan, "Real-Time Markov Modeling for
 * Single-Photon LiDAR: 1000x Acceleration and Convergence Analysis"
 * (arXiv 2509.20500):
 *
 *   bin tables    lambda_j = lambda(s_j) and cumulative flux F_j = F(s_j)
 *                 (Eq. arrival_flux; F is defined in Theorem 1),
 *   base matrix   P~_base = rownorm((1 lambda^T) (.) exp(-Lambda L - D))
 *                 (Section 3.4),
 *   dead time     P~ = J_l P~_base, rows rolled by l = ceil(x_d / Delta)
 *                 (Theorem 2, Section 3.4),
 *   stationary    pi P~ = pi, the leading left eigenvector (Section 2.3),
 *                 here by power iteration.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Units: time in ns; signal and background flux in expected photons per
 *   laser period (S = alpha*calE, B = t_r*lambda_b of Section 2.1).
 * - Bins are 0-based with centres s_j = (j + 1/2) Delta, Delta = t_r / n_b.
 * - Matrices are dense, row-major, rows = current state, columns = next
 *   state; element (i, j) lives at P[i*ld + j], ld >= n (in elements).
 * - Row i of the dead-time matrix is row (i + l) mod n of the base matrix:
 *   the reactivation bin of state s_i is l bins later (Theorem 2).
 * - Lambda (the wrap term of Theorem 1) is the one-period integral F(t_r).
 *   It equals S + B when the pulse lies inside [0, t_r).
 * - "_dev" pointers are device memory, "_host" pointers host memory; the
 *   caller owns every buffer.  No entry point allocates device memory.
 * - Every function enqueues its work on `stream` (a hipStream_t; NULL is the
 *   null stream) and returns without waiting, unless its comment says it
 *   synchronises.
 * - Argument, aliasing and size errors are detected on the host before any
 *   launch and nothing is written.  A failed launch returns DTM_EHIP.
 *   Non-convergence of one pixel is a soft, per-pixel status.
 * - Thread safety: calls on different streams may run concurrently; a plan
 *   must not be used by two threads at once.
 */
#ifndef DTM_H
#define DTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define DTM_OK        0
#define DTM_EINVAL   (-1)  /* invalid argument (scene, size, pointer, option) */
#define DTM_ENOTCONV (-2)  /* power iteration stopped at max_iter (soft)      */
#define DTM_EHIP     (-3)  /* a HIP runtime call or kernel launch failed      */
#define DTM_EALIAS   (-4)  /* input and output buffers overlap                */
#define DTM_ENOSPACE (-5)  /* workspace too small                             */
#define DTM_ENOTSUP  (-6)  /* valid request the library does not support      */

typedef void* dtm_stream_t; /* a hipStream_t */

typedef enum dtm_dtype { DTM_F64 = 0, DTM_F32 = 1 } dtm_dtype;

/* One pixel: the problem statement theta = (t_r, t_d, sigma_t, tau, S, B, n_b)
 * of Section 2.2 with the flux model of Eq. (arrival_flux):
 *   lambda(t) = S * N(t - tau; 0, sigma^2) + B / t_r,  t in [0, t_r)
 * (the Gaussian is cut to the period, so tau may lie anywhere).
 * Valid: t_r > 0, t_d >= 0 (the chain depends on t_d mod t_r only; the Monte
 * Carlo simulator uses t_d itself), sigma > 0, S >= 0, B >= 0, S + B > 0,
 * 2 <= n_b <= DTM_MAX_BINS, reserved == 0, every field finite; otherwise
 * DTM_EINVAL.  Also DTM_EINVAL: a scene whose flux underflows at every bin,
 * which leaves every row of the matrix zero (the chain is undefined).  The
 * test: the largest g_j = lambda_j exp(-F_j) over the first bin and the three
 * bins around tau (where g peaks), evaluated on the host in float64 under the
 * plan's flux sampling, must reach the smallest normal number of the
 * computing dtype (1.2e-38 float32, 2.2e-308 float64; dtm_validate_scene
 * checks float64).  With B = 0 and lambda sampled at the centres this
 * rejects scenes with no centre within about 13 sigma (float32) or
 * 37 sigma (float64) of tau, the exact distance depending on S / sigma; the
 * bin-averaged variants keep the pulse's mass and accept them. */
typedef struct dtm_scene {
  double period_ns;       /* t_r */
  double dead_time_ns;    /* t_d */
  double pulse_center_ns; /* tau */
  double pulse_sigma_ns;  /* sigma_t */
  double signal_flux;     /* S */
  double background_flux; /* B */
  int32_t n_bins;         /* n_b */
  int32_t reserved;       /* must be 0 */
} dtm_scene;

#define DTM_MAX_BINS 65536

/* Stop rules of the power iteration (Section 4: the convergence rate is set
 * by |lambda_2|, which the bound rule estimates from successive changes). */
#define DTM_STOP_CHANGE 0 /* stop when ||x_{t+1} - x_t||_1 < tol_l1              */
#define DTM_STOP_BOUND  1 /* with c_t the L1 change and rho the contraction
                             estimated from successive changes: once the next
                             change is predicted to meet c rho/(1-rho) <=
                             safety * tol_l1, the next sweep is a float64
                             check; stop when its residual r = ||x P~ - x||_1
                             meets r rho/(1-rho) <= safety * tol_l1 (the check
                             sweep's output is returned)                        */

/* Option flags */
#define DTM_FLAG_NO_FINAL_CHECK 0x1 /* skip the float64 residual sweep            */
#define DTM_FLAG_NO_DENSE       0x2 /* plan without the dense matrix pool: only the
                                       factored solver and the spectral analysis */
/* dtm_solve_batched without a warm start: begin the power iteration from
 * x0_j = lambda(s_j) / sum_k lambda(s_k), the stationary vector of the
 * chain without dead time (Section 2.2: registrations are then the arrivals),
 * instead of the uniform vector (uniform when that flux underflows at every
 * centre, which the bin-averaged variants allow).  Same stop rule and
 * float64 check; the single-pixel and factored solvers start from uniform
 * regardless. */
#define DTM_FLAG_START_FLUX    0x40

/* Discretisation variants (default: the paper's model, Section 3.4 with
 * Theorem 2's shift and lambda sampled at the bin centres).  With
 * q = x_d / Delta (x_d = t_d mod t_r, bins (j Delta, (j+1) Delta]):
 *   SHIFT_NEAREST  the exact "shift then quantize" bin that Theorem 2
 *                  approximates: row i is base row i + ceil(q - 1/2)
 *                  (q - 1/2 within a relative 1e-9 of an integer is taken
 *                  as that integer; a centre on an edge is in the lower bin);
 *   SHIFT_INTERP   reactivation between two centres: q = m + f, row i is
 *                  (1 - f) base row i + m plus f base row i + m + 1
 *                  (factored solver and spectral analysis only: a plan with
 *                  a dense pool returns DTM_ENOTSUP);
 *   LAMBDA_BIN_MEAN  lambda_j = (F(e_{j+1}) - F(e_j)) / Delta, the flux
 *                  averaged over the bin, in place of lambda(s_j);
 *   BIN_INTEGRAL   lambda_j e^{-F(s_j)} replaced by its bin average
 *                  (e^{-F(e_j)} - e^{-F(e_{j+1})}) / Delta: the exact
 *                  first-arrival mass of the bin.
 * SHIFT_NEAREST and SHIFT_INTERP exclude each other, as do LAMBDA_BIN_MEAN
 * and BIN_INTEGRAL (else DTM_EINVAL). */
#define DTM_FLAG_SHIFT_NEAREST   0x4
#define DTM_FLAG_SHIFT_INTERP    0x8
#define DTM_FLAG_LAMBDA_BIN_MEAN 0x10
#define DTM_FLAG_BIN_INTEGRAL    0x20

typedef struct dtm_solve_opts {
  double tol_l1;       /* target L1 distance (rule 1) or change threshold (rule 0) */
  double safety;       /* rule 1: fraction of tol_l1 the bound must reach (0,1]   */
  int32_t max_iter;    /* sweeps, >= 1                                             */
  int32_t check_every; /* single-pixel path: host polls after this many sweeps, then
                          after the sweeps the stop rule predicts are left (at
                          least 1, at most 4 check_every)                          */
  int32_t stop_rule;   /* DTM_STOP_CHANGE or DTM_STOP_BOUND                        */
  int32_t flags;       /* DTM_FLAG_*                                               */
} dtm_solve_opts;

/* Per-pixel solver report.  status is DTM_OK or DTM_ENOTCONV (or DTM_EINVAL
 * for an invalid warm start that was replaced; see flags). */
#define DTM_INFO_WARM_REJECTED 0x1 /* x0 was not a positive finite vector: uniform used */
#define DTM_INFO_RESTARTED     0x2 /* warm start did not converge: re-ran from uniform   */
#define DTM_INFO_CHECKED       0x4 /* residual_l1 comes from a float64 check sweep       */
#define DTM_INFO_STALLED       0x8 /* changes stopped shrinking at the precision floor   */
#define DTM_INFO_REFINED      0x10 /* float32 could not certify: re-solved in float64    */
#define DTM_INFO_CONTINUED    0x20 /* still running after the tile's dense_sweeps:
                                      finished in float64 on the factored product
                                      of the same matrix                           */
typedef struct dtm_solve_info {
  int32_t iterations;  /* sweeps performed (each reads the matrix once)         */
  int32_t status;
  int32_t flags;       /* DTM_INFO_*                                            */
  int32_t dense_sweeps; /* sweeps that read the pixel's stored matrix: iterations,
                           less the float64 sweeps of a DTM_INFO_CONTINUED or
                           DTM_INFO_REFINED pixel (which regenerate the matrix
                           from its tables); 0 from the factored solver        */
  double change_l1;    /* ||x_T - x_{T-1}||_1 of the last iterate             */
  double residual_l1;  /* ||x P~ - x||_1 of the input of the last sweep        */
  double rho_hat;      /* estimate of |lambda_2| from successive changes       */
} dtm_solve_info;

const char* dtm_status_string(int status);
int dtm_version(void); /* major*10000 + minor*100 + patch */

/* Host only, pure.  Returns DTM_OK or DTM_EINVAL for an invalid scene. */
int dtm_validate_scene(const dtm_scene* s);

/* Host only, pure: the dead-time shift of Theorem 2,
 *   l = ceil(x_d / Delta) mod n_b,  x_d = t_d mod t_r,
 * evaluated as q = x_d * n_b / t_r, with q snapped to the nearest integer when
 * it is one to 1e-9 relative (a dead time of whole bins is not rounded up). */
int dtm_shift_bins(const dtm_scene* s, int32_t* l_out);

/* Host only, pure: the shift a plan uses under the discretisation flags
 * (see DTM_FLAG_SHIFT_NEAREST / DTM_FLAG_SHIFT_INTERP): with q = x_d n_b / t_r
 * and the same 1e-9 integer snapping, NEAREST gives l = ceil(q - 1/2),
 * INTERP gives q = l + frac with 0 <= frac < 1, neither gives Theorem 2's l
 * and frac = 0; l is taken mod n_b.  Other flag bits are ignored; both
 * SHIFT flags together, an invalid scene or a null output return
 * DTM_EINVAL. */
int dtm_model_shift(const dtm_scene* s, int32_t flags, int32_t* l_out, double* frac_out);

/* ---- single pixel ------------------------------------------------------- */

/* Device workspace every single-pixel call below needs, in bytes, for a
 * matrix of n bins.  Holds the bin tables and the solver's partial sums. */
size_t dtm_workspace_bytes(int32_t n, dtm_dtype dt);

/* Bin tables (Eq. arrival_flux, Theorem 1): writes lambda_dev[j] = lambda(s_j)
 * in dt (n elements) and F_dev[j] = F(s_j) in float64 (n + 1 elements; the
 * last one is Lambda = F(t_r)).  F comes from normal tail probabilities
 * (erfc) at the bin edges and centres: a float64 exclusive prefix scan of
 * per-chunk flux integrals, then per-bin integrals and the half-bin integral
 * up to the centre.  Either output may be NULL. */
int dtm_bin_tables(const dtm_scene* s, dtm_dtype dt, void* lambda_dev, double* F_dev,
                   void* workspace_dev, size_t workspace_bytes, dtm_stream_t stream);

/* Base matrix (Section 3.4): P_base_dev[k*ld + j] =
 *   lambda_j exp(-Lambda [k > j] - F_j + F_k) / R_k,
 * R_k the row sum, for every row at once from one prefix and one suffix
 * float64 scan of g_j = lambda_j e^{-F_j} (the factor e^{F_k} cancels).
 * n x n. */
int dtm_build_base(const dtm_scene* s, dtm_dtype dt, void* P_base_dev, int64_t ld,
                   void* workspace_dev, size_t workspace_bytes, dtm_stream_t stream);

/* Dead time as a row permutation (Theorem 2): P_dev[i, :] =
 * P_base_dev[(i + l) mod n, :].  Out of place; overlapping buffers give
 * DTM_EALIAS.  Both matrices use the same ld. */
int dtm_apply_deadtime_shift(const dtm_scene* s, dtm_dtype dt, const void* P_base_dev,
                             void* P_dev, int64_t ld, dtm_stream_t stream);

/* Base matrix and shift fused: writes P~ = J_l P~_base directly (row i is
 * built from reactivation bin (i + l) mod n); no extra traffic. */
int dtm_build_transition(const dtm_scene* s, dtm_dtype dt, void* P_dev, int64_t ld,
                         void* workspace_dev, size_t workspace_bytes, dtm_stream_t stream);

/* Stationary vector of a row-stochastic n x n matrix P_dev (any such matrix,
 * e.g. from dtm_build_transition) by power iteration x <- x P / sum(x P)
 * from x0_dev (n elements of dt; NULL = uniform 1/n).  Writes pi_dev (n
 * elements of dt, sums to 1) and *info_host.  The accumulation of x P is
 * compensated in float32.  Synchronises `stream` before returning; returns
 * DTM_OK even when info_host->status is DTM_ENOTCONV.  opt NULL = defaults
 * (tol 1e-6, safety 0.25, max_iter 1000, check_every 4, DTM_STOP_BOUND). */
int dtm_stationary_pdf(const void* P_dev, int32_t n, int64_t ld, dtm_dtype dt,
                       const dtm_solve_opts* opt, const void* x0_dev, void* pi_dev,
                       void* workspace_dev, size_t workspace_bytes,
                       dtm_solve_info* info_host, dtm_stream_t stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): dtm_stationary_pdf with the solver's
 * workspace taken from a static device array of the library instead of a
 * caller's buffer.  Same arguments, results and synchronisation as
 * dtm_stationary_pdf without workspace_dev / workspace_bytes.  Allocates
 * nothing: no hipMalloc, hipFree or allocating library call.  The array holds
 * DTM_NOALLOC_SCRATCH_BYTES bytes per GPU (held from the first call on that
 * GPU until the process ends), enough for n <= DTM_NOALLOC_MAX_BINS in either
 * dtype; a larger n returns DTM_ENOSPACE before any launch.  Every call on
 * one GPU shares that GPU's array and the solver initialises what it reads
 * on every call; calls that overlap on one GPU (two streams or two threads)
 * race on the array and must be serialised by the caller.  The device is the
 * current one (hipSetDevice); `stream` must belong to it. */
#define DTM_NOALLOC_MAX_BINS 8192
#define DTM_NOALLOC_SCRATCH_BYTES 8912896 /* 8.5 MiB */
int dtm_stationary_pdf_noalloc(const void* P_dev, int32_t n, int64_t ld, dtm_dtype dt,
                               const dtm_solve_opts* opt, const void* x0_dev, void* pi_dev,
                               dtm_solve_info* info_host, dtm_stream_t stream);

/* ---- batched: many pixels with uneven n_b and dead time ------------------ */

/* Launch shape of the batched kernels.  Zero fields take the built-in or
 * autotuned defaults. */
typedef struct dtm_tile_config {
  int32_t fused_threads;   /* threads per workgroup of the one-block solver: 256 or 512
                              (0 = 512 if a one-block pixel has more than 1024 bins,
                              else 256)                                                 */
  int32_t fused_unroll;    /* rows in flight per thread in a one-block sweep: 2, 4 or 8
                              (the banded sweep keeps 16 column vectors in flight)     */
  int32_t fused_max_bins;  /* pixels with n_b above this take the banded path (>= 2)    */
  int32_t band_rows;       /* rows per workgroup in the banded sweep, multiple of 16,
                              at most 8192 (0 = 1024)                                  */
  int32_t dense_sweeps;    /* sweeps of a pixel's dense matrix (<= max_iter; 0 =
                              min(max_iter, 32)); a pixel still running after them
                              continues from its iterate in float64 with the factored
                              product of the same matrix (see
                              dtm_solve_factored_batched) up to max_iter sweeps in all
                              (DTM_INFO_CONTINUED).  The banded path launches this many
                              sweeps whatever the pixels need                          */
  int32_t band_cpt;        /* column vectors per thread in the banded sweep: 1, 2 or 4
                              (0 = 1); a workgroup covers 256 x band_cpt x (4 float /
                              2 double) columns of its rows                            */
  int32_t independent_paths; /* plans with both kinds of pixels: 0 = every matrix is
                              written before any is swept (the two paths wait for each
                              other's builds), 1 = each path sweeps as soon as its own
                              matrices are written                                     */
  int32_t fused_blocks;    /* one-block sweeps: 0 = one workgroup per pixel; k > 0 = k
                              persistent workgroups, each taking the next pixel in
                              launch order from a counter (so the banded launches of
                              a mixed plan keep the CUs the k workgroups leave)         */
  int32_t band_min_items;  /* banded path: once the pixels still running after a sweep
                              have fewer than this many work items (row band x column
                              block) in all, the remaining banded sweeps do nothing
                              and those pixels continue in float64 as after
                              dense_sweeps (DTM_INFO_CONTINUED): a sweep of so few
                              items cannot keep HBM busy.  0 = never (>= 0)            */
} dtm_tile_config;

typedef struct dtm_plan dtm_plan; /* opaque host object */

/* Validates every scene (DTM_EINVAL names nothing: use dtm_validate_scene to
 * find the pixel), fixes offsets, pixel order and launch shapes.  Copies the
 * scenes; scenes_host may be freed afterwards.  opt NULL = defaults; tiles
 * NULL = defaults.  n_pixels >= 1: an empty batch (or scenes_host NULL) is
 * DTM_EINVAL.  On every error *plan_out is set to NULL. */
int dtm_plan_create(const dtm_scene* scenes_host, int32_t n_pixels, dtm_dtype dt,
                    const dtm_solve_opts* opt, const dtm_tile_config* tiles,
                    dtm_plan** plan_out);
void dtm_plan_destroy(dtm_plan* plan);

/* Device workspace the plan needs (per-pixel metadata, bin tables, the dense
 * matrices of every pixel, iterates and partial sums), in bytes. */
size_t dtm_plan_workspace_bytes(const dtm_plan* plan);
/* Sum over pixels of n_b (length of the packed pi) and of n_b^2 (packed
 * matrices). */
int64_t dtm_plan_pi_elems(const dtm_plan* plan);
int64_t dtm_plan_matrix_elems(const dtm_plan* plan);
/* pi_offsets[p] = sum_{q<p} n_b(q) (n_pixels + 1 entries) and
 * mat_offsets[p] = sum_{q<p} n_b(q)^2; either may be NULL. */
int dtm_plan_offsets(const dtm_plan* plan, int64_t* pi_offsets_host, int64_t* mat_offsets_host);
/* The launch shape the plan uses (after defaults and autotuning). */
int dtm_plan_tiles(const dtm_plan* plan, dtm_tile_config* tiles_out);

/* Binds the plan to a workspace and uploads its metadata there.
 * Synchronises `stream`.  Must precede the calls below; re-binding moves it. */
int dtm_plan_bind(dtm_plan* plan, void* workspace_dev, size_t workspace_bytes,
                  dtm_stream_t stream);

/* Solves every pixel: bin tables, transition matrix (shift fused), power
 * iteration with the plan's stop rule, float64 residual check.  Pixels up to
 * fused_max_bins take one workgroup each in two launches: every matrix is
 * written (with the first sweep taken on the way), then the remaining sweeps
 * read them; larger pixels take the banded launches.  A pixel still running
 * after dense_sweeps sweeps, or a banded pixel still running once the banded
 * pixels hold fewer than band_min_items work items, goes on in float64 on
 * the factored product of the same matrix (DTM_INFO_CONTINUED; the report's
 * dense_sweeps counts the sweeps before).  Writes pi
 * packed by pi_offsets (dtype of the plan) and one dtm_solve_info per pixel
 * to infos_dev (device memory, plan order = input order).  x0_packed_dev
 * (packed like pi, dtype of the plan) seeds the iteration; NULL = uniform.
 * A warm start that is not positive and finite is replaced by uniform; one
 * that does not converge within max_iter is re-run from uniform.  Launches
 * only: no host synchronisation, no allocation, no memset, so the call can
 * be captured in a hipGraph and replayed. */
int dtm_solve_batched(const dtm_plan* plan, const void* x0_packed_dev, void* pi_packed_dev,
                      dtm_solve_info* infos_dev, dtm_stream_t stream);

/* Factored solver: power iteration on the same matrix without forming it.
 * With g_j = lambda_j exp(-F_j), c = exp(-Lambda), S_k the row normaliser of
 * the base matrix and u_k = x_{(k - l) mod n} / S_k, the left product of the
 * dead-time matrix of Section 3.4 is
 *   (x P~)_j = g_j (c U_{n-1} + (1 - c) U_j),   U_j = sum_{k <= j} u_k,
 * one float64 block scan per sweep (O(n) instead of O(n^2)).  Same stop
 * rule as dtm_solve_batched, every sweep in float64 (eps 1.1e-16), so tol can
 * go down to ~1e-12.  Uses only the plan's tables and a float64 scratch
 * region of its workspace; works with DTM_FLAG_NO_DENSE plans.  With
 * DTM_FLAG_SHIFT_INTERP (q = l + f), u_k = ((1 - f) x_{k-l} + f x_{k-l-1}) / S_k.
 * Launch only. */
int dtm_solve_factored_batched(const dtm_plan* plan, const void* x0_packed_dev, void* pi_packed_dev,
                               dtm_solve_info* infos_dev, dtm_stream_t stream);

/* Spectral convergence analysis (Section 4): for every pixel, the second
 * eigenvalue lambda_2 of P~ (magnitude and phase; the spectral gap is
 * 1 - |lambda_2|) and, when mixing_eps > 0, the empirical mixing steps
 *   min n : max_s (1/2) || e_s P~^n - pi ||_1 <= mixing_eps   (n <= max_steps <= 2^30,
 * else -1).  lambda_2 comes from orthogonal iteration with Rayleigh-Ritz on
 * the deflated operator x -> x P~ - (x 1) pi: a subspace of six vectors
 * (n - 1 when n <= 6) is mapped by the operator and re-orthonormalised each
 * step, and the eigenvalues of its 6 x 6 Rayleigh quotient (Ritz values)
 * approach the six eigenvalues of largest modulus after the Perron value;
 * lambda_2 is the largest, which converges at the rate |lambda_8 / lambda_2|
 * per step, so a third eigenvalue close to lambda_2 in modulus does not
 * slow or spoil it.  The Rayleigh quotient is formed every eighth step until
 * two of them give Ritz values within 1e-9 of each other, then every step;
 * the search stops when lambda_2 has moved by at most 1e-13 (1 + |lambda_2|)
 * and |lambda_3| by at most 1e-11 (1 + |lambda_2|) in two successive steps; max_steps also caps
 * the steps of this search (DTM_SPECTRAL_UNSETTLED when reached).  Uses the
 * factored operator (O(n) per step per vector).  The mixing search runs on
 * the plan's second stream beside the lambda_2 search, both after pi, and is
 * joined back into `stream` before the call returns.  It advances
 * every start state: for plans whose pixels have at most 1024 bins on chip
 * (the call then only launches); above that in the scratch (2 n^2 float64
 * per pixel), and the call then copies the per-pixel scratch offsets from
 * the host and synchronises `stream` before returning.  scratch_bytes below
 * dtm_spectral_scratch_bytes gives DTM_ENOSPACE; max_steps outside
 * [1, 2^30] or an unbound plan DTM_EINVAL. */
#define DTM_SPECTRAL_UNSETTLED 0x1 /* lambda_2 had not settled after max_steps steps  */
#define DTM_SPECTRAL_TIED      0x2 /* another eigenvalue, not lambda_2's conjugate,
                                      has lambda_2's modulus to 1e-9 (relative): the
                                      modulus stands, the phase is one of several   */
typedef struct dtm_spectral_info {
  double lambda2_re, lambda2_im;  /* lambda_2 (one of a conjugate pair: im >= 0)    */
  double lambda2_abs, lambda2_arg;/* |lambda_2| and its phase in [0, pi]             */
  double lambda3_abs;             /* largest modulus among the other Ritz values
                                     (lambda_2's conjugate left out): |lambda_3|    */
  double ritz_change;             /* change of lambda_2 (or of |lambda_3|, the larger)
                                     between the last two Rayleigh-Ritz steps        */
  int32_t iterations;             /* subspace steps                                  */
  int32_t mixing_steps;           /* -1: not reached / not requested                 */
  int32_t flags;                  /* DTM_SPECTRAL_*                                  */
  int32_t reserved;
} dtm_spectral_info;
size_t dtm_spectral_scratch_bytes(const dtm_plan* plan, int32_t with_mixing);
int dtm_spectral_batched(const dtm_plan* plan, double mixing_eps, int32_t max_steps,
                         dtm_spectral_info* out_dev, void* scratch_dev, size_t scratch_bytes,
                         dtm_stream_t stream);

/* Monte Carlo simulation of the detector the chain models (Section 2.1), for
 * checking the model against physics (Section 3.5 does the same): for every
 * pixel, runs_per_pixel independent runs of `cycles` laser periods with
 * Poisson arrivals of rate lambda(t), a non-paralyzable dead time and
 * free-running rearm; registrations in periods >= burn_cycles are counted in
 * n_b bins of X = T mod t_r (bin ceil(X / Delta) - 1).
 *
 * Random numbers: Philox4x32-10 with key = seed and counter = (draw block,
 * period, run, pixel index); the sampling steps (block 0: Poisson counts by
 * inversion of one uniform each; then a block per four pulse photons, two
 * Box-Muller pairs, and a block per four background photons; time-ordered
 * visit with the rearm time carried from period to period) are fixed, so
 * another implementation of the same steps reproduces the counts exactly.
 *
 * A run may be cut into segments of consecutive periods that are simulated
 * side by side from the armed state and then repaired where a segment's true
 * start differed (the repair walks each such segment from its true start
 * until the two trajectories meet); the counts are those of one sequential
 * walk of the run whatever the segmentation.
 *
 * hist_packed_dev: uint32 counts packed like pi (runs summed), overwritten.
 * overflow_dev: one uint32 per pixel (input order), zeroed by the caller; set
 * when the 64 periods a wave draws at once held more photons than its pool
 * (their mean plus ten standard deviations; the excess is dropped).
 * lanes_per_run: 0 = automatic, else a power of two <= 64 (lanes that share
 * one segment; the counts do not depend on it).
 * segments_per_run: 0 = automatic (about 2^18 segments in all, none shorter
 * than 256 periods), else 1 .. cycles (1 = no cut; the counts do not depend
 * on it).
 * scratch_dev / scratch_bytes: segment states, at least
 * dtm_mc_scratch_bytes(plan, runs_per_pixel, cycles, segments_per_run) bytes,
 * 256-byte aligned (may be NULL when that is 0; DTM_ENOSPACE when short).
 * Requires S + B <= 24, n_b <= 16384, 1 <= runs_per_pixel <= 65535,
 * 0 <= burn_cycles < cycles < 2^32 and runs_per_pixel * (cycles -
 * burn_cycles) < 2^26 (so no bin can pass 2^32), at most 2^27 segments in
 * all and at most 65535 launch blocks per pixel; else DTM_EINVAL or
 * DTM_ENOTSUP and nothing is launched.  The plan must be bound; launch only
 * (four kernels on `stream`; the scratch must stay untouched until they
 * finish). */
size_t dtm_mc_scratch_bytes(const dtm_plan* plan, int32_t runs_per_pixel, int64_t cycles,
                            int32_t segments_per_run);
int dtm_mc_histograms(const dtm_plan* plan, int32_t runs_per_pixel, int64_t cycles,
                      int64_t burn_cycles, uint64_t seed, int32_t lanes_per_run,
                      int32_t segments_per_run, uint32_t* hist_packed_dev, uint32_t* overflow_dev,
                      void* scratch_dev, size_t scratch_bytes, dtm_stream_t stream);

/* HIP graph of one dtm_solve_batched call: every launch of the solve is
 * captured once and replayed by dtm_graph_launch, which saves the per-launch
 * host cost of the banded path's sweep loop.  The plan, its workspace and the
 * three buffers must stay valid while the graph exists; the replay reads and
 * writes exactly what the captured call does.  Synchronises `stream`. */
typedef struct dtm_graph dtm_graph; /* opaque host object */
int dtm_graph_create(const dtm_plan* plan, const void* x0_packed_dev, void* pi_packed_dev,
                     dtm_solve_info* infos_dev, dtm_stream_t stream, dtm_graph** graph_out);
int dtm_graph_launch(dtm_graph* graph, dtm_stream_t stream);
void dtm_graph_destroy(dtm_graph* graph);

/* Batched a2 / a3 / fused a2+a3, writing every pixel's n_b x n_b matrix
 * packed by mat_offsets (ld = n_b).  Launch only. */
int dtm_build_base_batched(const dtm_plan* plan, void* P_packed_dev, dtm_stream_t stream);
int dtm_apply_deadtime_shift_batched(const dtm_plan* plan, const void* P_base_packed_dev,
                                     void* P_packed_dev, dtm_stream_t stream);
int dtm_build_transition_batched(const dtm_plan* plan, void* P_packed_dev,
                                 dtm_stream_t stream);

/* ---- learned warm start ------------------------------------------------------
 * A small network predicts pi from the scene parameters to seed the power
 * iteration (dtm_solve_batched's x0; the solver's float64 residual decides,
 * uniform is the fallback):
 *   features phi (5, see dtm_mlp_features) -> Linear(5, 256) -> GELU
 *   -> Linear(256, 256) -> GELU -> Linear(256, 1024) -> (rotate by the
 *   pulse bin) -> (+ prior logits) -> softmax,
 * the optional prior being the log of the flux start (dtm_mlp_flux_prior).
 * With a pulse bin k per row (dtm_mlp_features' shift output), the
 * network's output m is the logit of bin (m + k) mod 1024: it works in a
 * frame centred on the laser pulse.  The model is periodic in the arrival
 * time, so moving the pulse by whole bins rotates pi (up to the Gaussian's
 * tail beyond the period's ends); in that frame pi depends on the scene
 * only through S, B, sigma, t_d and the pulse's offset within its bin.
 * GELU is the erf form.  GEMMs use bfloat16 operands with float32
 * accumulation on the matrix cores; everything else is float32.  All state
 * lives in a caller-owned workspace described by dtm_mlp_layout: float32
 * master parameters (W1 is stored as 16 x 256 with input rows 5..15 zero),
 * their bfloat16 copies, gradients, Adam moments, the activations of one
 * batch of up to max_batch rows and the weight gradients' split partial
 * products.  Weights are row-major (in x out). */
#define DTM_MLP_IN 5
#define DTM_MLP_IN_PAD 16
#define DTM_MLP_HIDDEN 256
#define DTM_MLP_OUT 1024
#define DTM_MLP_MAX_BATCH 65536

typedef struct dtm_mlp_layout {
  size_t params, params_bf16, grads, adam_m, adam_v, act, partial, total; /* byte offsets, total size */
  int64_t off_w1, off_b1, off_w2, off_b2, off_w3, off_b3;         /* element offsets of each tensor
                                                                     in params / grads / moments */
  int64_t n_params;
  int32_t max_batch;
  int32_t reserved;
} dtm_mlp_layout;

int dtm_mlp_workspace_layout(int32_t max_batch, dtm_mlp_layout* layout_out);
/* Features of n device scenes into feat_dev (n x 5 float32):
 * 2 u, sigma [ns], 2 (ln S - ln 0.05)/ln 100 - 1,
 * 2 (ln B - ln 0.01)/ln 100 - 1, (t_d mod t_r)/t_r,
 * where the pulse bin is k = floor(tau / (t_r / 1024)) and
 * u = tau / (t_r / 1024) - k - 1/2 in [-1/2, 1/2) is the pulse's offset from
 * that bin's centre (both in float64).  shift_dev (n int32, may be NULL)
 * receives k. */
int dtm_mlp_features(const dtm_scene* scenes_dev, int32_t n, float* feat_dev, int32_t* shift_dev,
                     dtm_stream_t stream);
/* Refresh the bfloat16 copies after writing the float32 parameters. */
int dtm_mlp_sync_bf16(void* workspace_dev, int32_t max_batch, dtm_stream_t stream);
/* Prior logits for the network's output (n x 1024 float32):
 * log(lambda_j / sum_k lambda_k) at the 1024 bin centres (j + 1/2) t_r / 1024
 * of each device scene, lambda of Eq. (arrival_flux): the logarithm of the
 * solver's flux start (DTM_FLAG_START_FLUX).  With it the network learns a
 * correction to that start rather than the whole PDF. */
int dtm_mlp_flux_prior(const dtm_scene* scenes_dev, int32_t n, float* prior_dev, dtm_stream_t stream);
/* probs_dev (batch x 1024 float32) = softmax(rotate(network(feat_dev), k)
 * + prior_dev): probs_dev[i][j] uses the network's output (j - k_i) mod 1024
 * with k_i = shift_dev[i] (taken mod 1024).  prior_dev (batch x 1024 float32)
 * and shift_dev (batch int32) may each be NULL (no prior; k = 0). */
int dtm_mlp_forward(void* workspace_dev, int32_t max_batch, const float* feat_dev, const float* prior_dev,
                    const int32_t* shift_dev, int32_t batch, float* probs_dev, dtm_stream_t stream);
/* Forward (with the same optional prior and shift), cross-entropy
 * -sum_j target_j log q_j per row (loss_dev, batch floats, may be NULL), and
 * the gradients of the mean loss into the workspace's grads.  rows_dev
 * (batch int32, may be NULL) makes batch row i the row rows_dev[i] of
 * feat_dev, prior_dev, shift_dev and target_dev (a shuffled mini-batch read
 * in place; the caller guarantees the indices are rows of those arrays);
 * NULL takes rows 0 .. batch-1.  The weight gradients split the batch over
 * blocks when their outputs have few tiles; the partial products are added
 * in a fixed order, so results are reproducible. */
int dtm_mlp_backward(void* workspace_dev, int32_t max_batch, const float* feat_dev, const float* prior_dev,
                     const int32_t* shift_dev, const float* target_dev, const int32_t* rows_dev, int32_t batch,
                     float* loss_dev, dtm_stream_t stream);
/* One Adam step (bias-corrected, step >= 1) on every parameter. */
int dtm_mlp_adam(void* workspace_dev, int32_t max_batch, float lr, float beta1, float beta2,
                 float eps, int32_t step, dtm_stream_t stream);
/* The network's GEMM: C (M x N float32, ldc) = op(A) op(B), A and B bfloat16
 * row-major, op = transpose when trans_* != 0 (v_mfma_f32_16x16x32_bf16,
 * float32 accumulation). */
int dtm_mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const void* A_dev, int32_t lda,
                      int32_t trans_a, const void* B_dev, int32_t ldb, int32_t trans_b,
                      float* C_dev, int32_t ldc, dtm_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DTM_H */
