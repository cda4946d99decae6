/*
 * mwf.h -- messenger-field Wiener filtering of HEALPix maps on AMD MI355X (gfx950).
 *
 * Method: Elsner & Wandelt, "Fast Wiener filtering of CMB maps", Sect. 2.
 * Data d = s + n (Eq. 1); the Wiener filter solves (S^-1 + N^-1) s = N^-1 d (Eq. 2).
 * With a messenger field t of covariance T = tau * 1, tau = min(diag N), and
 * Nbar = N - T, each sweep solves
 *     Eq. (3)  (Nbar^-1 + (lambda T)^-1) t = Nbar^-1 d + (lambda T)^-1 s   in pixel space,
 *     Eq. (4)  (S^-1 + (lambda T)^-1) s = (lambda T)^-1 t                  in harmonic space,
 * with a spherical-harmonic transform pair in between; lambda is lowered to 1
 * (Sect. 3), where the pair reduces to Eq. (2).
 *
 * Conventions used by every call below:
 *   - Maps: HEALPix RING order, npix = 12 nside^2 values per map, maps of a
 *     batch stored back to back (stride npix).
 *   - alm: complex, interleaved (re, im), packed m-major: entry (l, m), 0 <= m <= l <= lmax,
 *     sits at index m (2 lmax + 1 - m) / 2 + l; N_lm = (lmax+1)(lmax+2)/2 entries
 *     per map, maps back to back (stride 2 N_lm reals). Y_lm carries the
 *     Condon-Shortley phase. Only m >= 0 is stored (real fields).
 *   - The forward transform is the pixel-area-weighted adjoint of the synthesis:
 *     a_lm = Omega sum_p conj(Y_lm(p)) f_p, Omega = 4 pi / npix.
 *   - Pixel noise: N is diagonal with inverse variance ninv[p] >= 0; ninv = 0
 *     (or mask[p] = 0) marks an unobserved pixel. tau = 1 / max_p ninv[p].
 *   - Harmonic filter of Eq. (4): s_lm = C_l / (C_l + lambda tau Omega) a_lm
 *     (0 where C_l = 0); pixel step of Eq. (3): t = s + w (d - s) with
 *     w_p = lambda tau ninv_p / (1 + (lambda - 1) tau ninv_p).
 *   - Element type: double for WF_F64; float for WF_F32, WF_BF16X3 and WF_BF16X6.
 *     WF_F32 runs the Legendre contraction on fp32 matrix cores; the bf16 modes
 *     split both operands into bf16 pieces on bf16 matrix cores with fp32
 *     accumulation: three pieces and six products (WF_BF16X6, fp32-level: within
 *     1e-5 of FP64 after a full solve) or two pieces and three products
 *     (WF_BF16X3, ~5e-6 per transform but 2-4e-5 after an 80-sweep solve: it does
 *     not meet the 1e-5 bar of the other reduced-precision modes).
 *     The Legendre recurrence and the ring FFTs are fp64 on every path.
 *   - Device pointers are HIP device memory owned by the caller; host pointers
 *     are ordinary host memory, copied before the call returns.
 *   - Calls that take a hip_stream (a hipStream_t, NULL = default stream) only
 *     enqueue work and return; kernel faults surface at wf_sync().
 *   - A plan is not thread-safe: drive each plan from one host thread.
 *   - Every int-returning call returns WF_OK (0) or a negative WF_E* code;
 *     wf_last_error() then holds a message (per host thread).
 */
#ifndef MWF_H
#define MWF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  WF_OK = 0,
  WF_EINVAL = -1,       /* invalid argument (message in wf_last_error)          */
  WF_ENOMEM = -2,       /* device or host allocation failed / over budget        */
  WF_EDEVICE = -3,      /* HIP runtime error                                      */
  WF_EUNSUPPORTED = -4, /* valid request the library does not handle              */
  WF_EBUSY = -5,        /* no free slot (serving)                                 */
  WF_ENOTREADY = -6     /* result not finished yet (serving)                      */
};

enum { WF_F64 = 0, WF_F32 = 1, WF_BF16X3 = 2, WF_BF16X6 = 3 };

/* Plan flags. WF_FLAG_TIMING: record HIP events around every kernel launch of a
 * solve on the caller's stream and report the summed durations in wf_stats; the
 * events are created without the system-scope fence (they only time), and the solve
 * then synchronises the stream before returning.
 * WF_FLAG_CHI2: every solve also records, for each map and each sweep k, the chi^2
 * of the iterate after that sweep (Sect. 3's convergence monitor, at lambda = 1):
 *   chi2_k = sum_lm w_m |s_lm|^2 / C_l + sum_p N^-1_p (d_p - s_p)^2,
 * w_m = 1 for m = 0 and 2 for m > 0, modes with C_l = 0 left out, s_p the synthesis
 * of s_lm; read with wf_chi2 (wf_stats.chi2_last holds map 0's last value, at the
 * cost of a synchronisation). The terms are accumulated by FP64 atomics, so their
 * last bits depend on the order of the additions. Plan solves only (not groups or
 * serving). */
enum { WF_FLAG_TIMING = 1, WF_FLAG_CHI2 = 2 };

typedef struct wf_plan_s* wf_plan_t;
typedef struct wf_group_s* wf_group_t;

typedef struct {
  int32_t dtype;      /* WF_F64 (default), WF_F32, WF_BF16X3 or WF_BF16X6              */
  int32_t max_batch;  /* largest nmaps accepted by the batched calls (>= 1; 0 -> 1)    */
  int32_t flags;      /* 0 or WF_FLAG_TIMING                                           */
  const char* tune_cache; /* NULL, or a text file of launch shapes found by wf_autotune:
                           read at plan time, appended to by wf_autotune            */
} wf_plan_opts;

typedef struct {
  int32_t sweeps_done;   /* sweeps run by the last solve                                */
  int32_t timed;         /* 1 when the kernel times below were measured (WF_FLAG_TIMING) */
  double ms_ring;        /* summed duration of the ring-FFT / pixel-update launches      */
  double ms_analysis;    /* summed duration of the Legendre analysis launches           */
  double ms_synthesis;   /* summed duration of the filter + Legendre synthesis launches */
  int32_t n_ring, n_analysis, n_synthesis;   /* number of launches of each kind        */
  int32_t pad_;
  double chi2_last;      /* WF_FLAG_CHI2: chi^2 of map 0 after the last sweep, else 0     */
} wf_stats;

/*
 * wf_plan -- build the geometry, coefficient tables and device work buffers for
 * one (nside, lmax, C_l, N^-1, mask) problem (Sect. 2: T = min(diag N) fixes tau).
 *   out      receives the plan handle (set to NULL on failure)
 *   nside    HEALPix resolution, a power of two in [1, 1024] (a ring pair's transform
 *            runs in one workgroup's LDS: at 1024 the longest polar rings take a
 *            Bluestein transform of 8192 points, 136 KiB in FP64 with its padding, of
 *            the 160 KiB a CU has; at 2048 it would not fit)
 *   lmax     band limit, 0 <= lmax <= 4 nside - 1 (and <= 2048)
 *   cl       host, lmax+1 doubles, finite and >= 0 (signal power C_l; 0 filters the mode out)
 *   ninv     host, npix doubles, finite and >= 0 (inverse noise variance per pixel)
 *   mask     host, npix bytes, 1 = observed, 0 = unobserved (forces ninv = 0); NULL = all observed
 *   opts     NULL for defaults
 *   hip_stream stream used for the table uploads (the call synchronises it)
 * Errors: WF_EINVAL (bad nside/lmax, non-finite or negative input, no observed
 * pixel), WF_EUNSUPPORTED (dtype not built), WF_ENOMEM, WF_EDEVICE.
 * The plan owns copies of everything; the caller keeps its arrays.
 */
int wf_plan(wf_plan_t* out, int32_t nside, int32_t lmax, const double* cl,
            const double* ninv, const uint8_t* mask, const wf_plan_opts* opts,
            void* hip_stream);

/*
 * wf_solve -- run the messenger iteration (Sect. 2) from s = t = 0, one sweep
 * per entry of the lambda schedule (Sect. 3: lambda is lowered to 1).
 *   d        device, npix elements of the plan dtype: the data map
 *   s_wf     device, npix elements: receives the final signal map
 *   s_alm    device, 2 N_lm elements, or NULL: receives the final filtered alm
 *   lambda   host, nsweeps doubles, finite and > 0
 *   nsweeps  >= 1
 *   stats    NULL or receives counters
 * Errors: WF_EINVAL (NULL pointers, bad schedule), WF_EDEVICE.
 */
int wf_solve(wf_plan_t plan, const void* d, void* s_wf, void* s_alm,
             const double* lambda, int32_t nsweeps, void* hip_stream,
             wf_stats* stats);

/*
 * wf_chi2 -- the chi^2 history of the last solve on this plan, if it recorded one (a
 * plan created with WF_FLAG_CHI2, or wf_solve_adaptive):
 *   nmaps, nsweeps  those of that solve (checked)
 *   out             host, nmaps * nsweeps doubles: out[map * nsweeps + k] = chi2_k
 * Waits for the solve. Errors: WF_EINVAL (no such solve, other sizes), WF_EDEVICE.
 */
int wf_chi2(wf_plan_t plan, int32_t nmaps, int32_t nsweeps, double* out);

/*
 * wf_solve_batch -- wf_solve for nmaps independent data maps that share the
 * plan's C_l, N^-1 and mask (d, s_wf: nmaps * npix; s_alm: nmaps * 2 N_lm).
 * 1 <= nmaps <= max_batch.
 */
int wf_solve_batch(wf_plan_t plan, int32_t nmaps, const void* d, void* s_wf,
                   void* s_alm, const double* lambda, int32_t nsweeps,
                   void* hip_stream, wf_stats* stats);

/*
 * wf_solve_banded -- wf_solve of one map with a band limit per sweep (Sect. 3: the
 * transforms of a sweep need only reach l_max^SHT while lambda smooths the small
 * scales away). Sweep k runs the transforms and the filter for l, m <= lmax_sht[k]:
 * s_lm of that sweep is zero above it, and the pixel map it synthesises has no
 * such modes.
 *   lmax_sht  host, nsweeps entries, non-decreasing, each in [0, lmax]
 *   other arguments as for wf_solve; s_alm (full lmax layout) is zero above the
 *   last sweep's band limit.
 * The sweeps below lmax run on plans of the same problem at those band limits,
 * made on first use and kept with this plan (their tables and work buffers count
 * against device memory). WF_FLAG_CHI2 and WF_FLAG_TIMING work as for wf_solve.
 * Errors: WF_EINVAL (bad schedule or band limits, NULL d or s_wf), WF_ENOMEM,
 * WF_EDEVICE.
 */
int wf_solve_banded(wf_plan_t plan, const void* d, void* s_wf, void* s_alm,
                    const double* lambda, const int32_t* lmax_sht, int32_t nsweeps,
                    void* hip_stream, wf_stats* stats);

/*
 * Adaptive cooling (Sect. 3). Level j works at l_j = l_iter0 * 2^j with
 *   lambda_j = C_{l_j} / (tau Omega)      (the lambda at which f_{l_j} = 1/2)
 *   band limit L_j = min(lmax, l_j + l_pad)   (lmax when full_band = 1)
 * until lambda_j <= 1 (or l_j > lmax): that level is the last, lambda = 1, L = lmax.
 * The monitor is the chi^2 of the iterate at lambda = 1 (see WF_FLAG_CHI2), with
 * sigma = sqrt(2 n_obs), n_obs the observed pixels. The chi^2 of iterate k is known
 * once the ring pass of sweep k + 1 has synthesised its map; the decision it allows
 * applies from sweep k + 2 on (the ring work of sweep k + 1 is already running).
 * With iterates k - 1 and k both of the current level and D = chi2_{k-1} - chi2_k:
 *   last level:   D < stop_tol * sigma stops; the result is iterate k + 1;
 *   other levels: |D| < plateau_tol * sigma moves to the next level.
 * A level other than the last also ends once max_level_sweeps sweeps have been
 * started at it (0: no limit). The solve ends after max_sweeps sweeps in any case.
 */
typedef struct {
  int32_t l_iter0;          /* first l_iter, >= 1 (the paper starts at 20)             */
  int32_t l_pad;            /* band-limit margin above l_iter, >= 0 (the paper: ~100)   */
  int32_t full_band;        /* 1: every sweep at lmax (cooling without truncation)     */
  int32_t max_level_sweeps; /* >= 0                                                     */
  double plateau_tol;       /* >= 0, in units of sigma                                  */
  double stop_tol;          /* >= 0, in units of sigma (the paper: 1e-4)                */
} wf_adaptive_opts;

/* wf_adaptive_defaults -- l_iter0 20, l_pad 100, full_band 0, max_level_sweeps 50,
 * plateau_tol 1, stop_tol 1e-4. Host-only. */
void wf_adaptive_defaults(wf_adaptive_opts* opts);

/*
 * wf_adaptive_levels -- the level table above, host-only:
 *   lmax, cl    band limit and C_l (host, lmax + 1 entries); tau, omega as in the plan
 *   max_levels  capacity of lambda_out and lmax_out
 *   nlevels     receives the number of levels (the last has lambda 1 and band lmax)
 * Errors: WF_EINVAL (bad options, tau or omega not > 0, more than max_levels levels).
 */
int wf_adaptive_levels(int32_t lmax, const double* cl, double tau, double omega,
                       const wf_adaptive_opts* opts, int32_t max_levels,
                       double* lambda_out, int32_t* lmax_out, int32_t* nlevels);

/*
 * wf_solve_adaptive -- the messenger iteration of one map from s = t = 0 under the
 * adaptive schedule above, with the band limit of each level (wf_solve_banded).
 * Waits for its own work: the host reads the chi^2 of every iterate (a 4 KB copy
 * on the plan's second stream while the sweep's Legendre work runs).
 *   d, s_wf, s_alm  as for wf_solve (s_alm may be NULL)
 *   opts            NULL for wf_adaptive_defaults
 *   max_sweeps      >= 1
 *   lambda_out, lmax_out, chi2_out  host, max_sweeps entries each: lambda and band
 *                   limit of every sweep run, and the chi^2 of its iterate
 *   nsweeps_out     receives the number of sweeps run
 *   converged       NULL, or receives 1 if the stop rule ended the solve, else 0
 * The plan's chi^2 history (wf_chi2 with nmaps 1, nsweeps = *nsweeps_out) is set too.
 * Errors: WF_EINVAL, WF_ENOMEM, WF_EDEVICE.
 */
int wf_solve_adaptive(wf_plan_t plan, const void* d, void* s_wf, void* s_alm,
                      const wf_adaptive_opts* opts, int32_t max_sweeps,
                      double* lambda_out, int32_t* lmax_out, double* chi2_out,
                      int32_t* nsweeps_out, int32_t* converged, void* hip_stream,
                      wf_stats* stats);

/*
 * wf_constrained_batch -- constrained realisations (Sect. 3: the Wiener-filter map plus
 * a fluctuation map has the fiducial power spectrum). For each map i, with a signal
 * draw s_rand from S and a noise draw n_rand from N built from the caller's unit
 * normal draws,
 *   s_rand   = sum_lm sqrt(C_l) xi_lm Y_lm         (xi_l0 real: its imaginary part is ignored)
 *   n_rand_p = eta_p / sqrt(ninv_p)                (0 where unobserved)
 *   s_CR     = s_rand + WF(d - s_rand - n_rand)
 * where WF is the messenger solve of wf_solve_batch with the same lambda schedule.
 *   d      device, nmaps * npix (plan dtype): the data maps
 *   xi     device, nmaps * 2 N_lm (plan dtype): packed alm of unit draws,
 *          E|xi_lm|^2 = 1 (real N(0,1) at m = 0, (g1 + i g2)/sqrt 2 above)
 *   eta    device, nmaps * npix (plan dtype): N(0,1) per pixel
 *   s_cr   device, nmaps * npix: receives s_CR
 *   s_alm  device, nmaps * 2 N_lm, or NULL: receives the alm of s_CR
 * The plan keeps three work buffers for this call (two maps and one alm set per
 * map of max_batch), made on first use. Errors: as wf_solve_batch, and WF_EINVAL for
 * NULL xi or eta.
 */
int wf_constrained_batch(wf_plan_t plan, int32_t nmaps, const void* d, const void* xi,
                         const void* eta, void* s_cr, void* s_alm, const double* lambda,
                         int32_t nsweeps, void* hip_stream, wf_stats* stats);

/*
 * wf_solve_batch_static -- wf_solve_batch with every work buffer (ring coefficients,
 * Legendre partial sums, filtered coefficients) in one static workspace per device
 * instead of the plan's own buffers. For callers that cannot allocate (code under
 * HIP stream capture, tight serving loops, harnesses that forbid allocation): the
 * call allocates no device memory and creates no stream or event. The plan (made
 * beforehand) is only read; its device must be current.
 *   arguments as for wf_solve_batch. The result equals wf_solve_batch's on the same
 *   plan (same kernels; the ring launches run one after another on hip_stream).
 *   The workspace holds 128 MiB per device, taken when the library's device code is
 *   loaded on that device and held until the process ends: enough for one FP64 map
 *   at nside 512 / lmax 1024 (105 MiB) or one FP32 map there (69 MiB).
 *   Every call on a device shares the workspace and leaves its contents behind
 *   (the call clears what must start at zero): calls that overlap on one device,
 *   on any streams, race and give wrong results. No chi^2 history or kernel
 *   timings are recorded (WF_FLAG_CHI2 / WF_FLAG_TIMING are ignored;
 *   wf_chi2 afterwards reports no history).
 * Errors: as wf_solve_batch; WF_EINVAL when the solve needs more workspace than
 * 128 MiB (the message gives the need) or the plan's device is not current.
 */
int wf_solve_batch_static(wf_plan_t plan, int32_t nmaps, const void* d, void* s_wf,
                          void* s_alm, const double* lambda, int32_t nsweeps,
                          void* hip_stream, wf_stats* stats);

/*
 * sht_map2alm -- forward transform of nmaps maps: a_lm = Omega sum_p conj(Y_lm(p)) f_p
 * (the basis change of Sect. 2 from pixels to harmonics).
 *   map  device, nmaps * npix elements; alm device, nmaps * 2 N_lm elements.
 */
int sht_map2alm(wf_plan_t plan, int32_t nmaps, const void* map, void* alm,
                void* hip_stream);

/*
 * sht_alm2map -- synthesis f_p = sum_lm a_lm Y_lm(p) of nmaps real fields
 * (the basis change back to pixels). a_l0 must be real; its imaginary part is ignored.
 */
int sht_alm2map(wf_plan_t plan, int32_t nmaps, const void* alm, void* map,
                void* hip_stream);

/*
 * wf_footprint -- device bytes a plan of this shape with max_batch = nmaps would
 * hold (tables + work buffers), for admission control. Host-only.
 */
int wf_footprint(int32_t nside, int32_t lmax, int32_t dtype, int32_t nmaps,
                 size_t* bytes);

/*
 * wf_plan_info -- shape of a plan (any pointer may be NULL):
 *   npix, nalm   pixels and packed alm per map
 *   tau          min(diag N) = 1 / max ninv
 *   units_all    (l, m, ring pair) triples of one Legendre transform of one map,
 *                2 nside N_lm
 *   units_active the triples actually visited after dropping ring pairs whose
 *                lambda_lm stays below 2^-448 for every l <= lmax
 */
int wf_plan_info(wf_plan_t plan, int64_t* npix, int64_t* nalm, double* tau,
                 int64_t* units_all, int64_t* units_active);

/*
 * wf_pixel_angles -- colatitude theta and longitude phi of every pixel centre of
 * HEALPix RING order at this nside (host arrays of npix doubles).
 */
int wf_pixel_angles(int32_t nside, double* theta, double* phi);

/*
 * wf_autotune -- time every launch shape of the matrix-core Legendre kernels
 * (analysis: 1, 2, 4 or, for WF_F32, 8 column tiles per workgroup -- from 4 tiles on,
 * the Legendre values of a 256-pair block are generated once for 64 or 128 columns;
 * synthesis: 1, 2 or 4 column tiles
 * per wave, or 8 for WF_F32, or the wide kernel: 256 ring pairs and 64 columns per
 * workgroup of 32 x 32 tiles) on this plan at nmaps maps, keep the fastest in the plan,
 * record it in the process-wide cache (and in opts.tune_cache if given: lines
 * "key ana_ct syn_nct wide") so that later plans of the same shape start with it.
 * Task groups and serving lanes use the per-wave synthesis shape. Overwrites the
 * plan's work buffers (run it before a solve, not between the calls of one). Waits
 * for its own launches.
 *   ana_ct, syn_nct  NULL, or receive the chosen shape (syn_nct 64 for the wide
 *                    kernel; 0 for WF_F64 plans, which have a single shape)
 * Errors: WF_EINVAL (nmaps outside [1, max_batch]), WF_EDEVICE.
 */
int wf_autotune(wf_plan_t plan, int32_t nmaps, void* hip_stream, int32_t* ana_ct,
                int32_t* syn_nct);

/*
 * Task groups: several plans (different nside / lmax / C_l / N^-1, one shared
 * matrix-core dtype) stepped together, one kernel launch per phase for all of
 * them, so that a batch of uneven map sizes (the independent maps of Sect. 3's
 * timing runs at several resolutions) fills the GPU as one launch would.
 *
 * wf_group_create -- group nplans existing plans; plan i runs nmaps[i] maps
 *   (1 <= nmaps[i] <= its max_batch). The group borrows the plans: they must
 *   outlive it and must not run other calls while a group solve is in flight.
 *   Errors: WF_EINVAL (NULL plan, mixed dtypes, bad nmaps), WF_EUNSUPPORTED
 *   (WF_F64 plans: run those with wf_solve_batch).
 */
int wf_group_create(wf_group_t* out, int32_t nplans, const wf_plan_t* plans,
                    const int32_t* nmaps);

/*
 * wf_group_solve -- wf_solve_batch for every plan of the group with one shared
 * lambda schedule. d[i], s_wf[i] (and s_alm[i] unless s_alm is NULL) are device
 * buffers laid out as for plan i's wf_solve_batch. Results equal those of the
 * separate wf_solve_batch calls up to the floating-point summation order fixed by
 * the group's launch shape. The call synchronises the stream once before it
 * uploads the group's task table.
 * Errors: WF_EINVAL (NULL buffers, bad schedule), WF_ENOMEM, WF_EDEVICE.
 */
int wf_group_solve(wf_group_t group, const void* const* d, void* const* s_wf,
                   void* const* s_alm, const double* lambda, int32_t nsweeps,
                   void* hip_stream, wf_stats* stats);

/*
 * wf_group_autotune -- time two-sweep group solves over every launch shape (6
 * combinations, 8 for WF_F32) and keep the fastest for this group. Overwrites s_wf.
 */
int wf_group_autotune(wf_group_t group, const void* const* d, void* const* s_wf,
                      void* hip_stream, int32_t* ana_ct, int32_t* syn_nct);

/* wf_group_destroy -- free a group (not its plans); waits for the device. */
void wf_group_destroy(wf_group_t group);

/*
 * Serving. A server owns a non-blocking HIP stream on the device current at
 * creation, two host threads and device memory up to an HBM budget. Requests
 * (independent messenger solves, each with its own nside, lmax, C_l, N^-1, mask,
 * data and lambda schedule) are admitted in arrival order as request slots and
 * memory free up; requests of the same (nside, lmax, dtype) share a lane, a plan
 * whose maps are the lane's slots, and every step advances every admitted request
 * by one sweep with one kernel launch per phase for all lanes. A request therefore
 * joins the running batch at the next step and its result is the one a plan of
 * the same dtype computes for it alone (same kernels, column-independent sums).
 */
typedef struct wf_server_s* wf_server_t;

typedef struct {
  int64_t submitted, completed;   /* requests accepted by submit / finished               */
  int64_t steps;                  /* batched steps launched                               */
  int64_t map_sweeps;             /* sweeps of finished requests                          */
  int64_t peak_slots;             /* most requests admitted at once                       */
  int64_t lanes_created, lanes_evicted;
  int64_t bytes_in_use;           /* budget charged now (lanes + shape tables)            */
  int64_t peak_bytes;
  int64_t slots_in_use, pending, lanes;
} wf_server_stats;

/*
 * wf_server_create -- start a server.
 *   hbm_budget_bytes  device bytes its lanes and tables may hold (>= 16 MiB); a lane
 *                     of (nside, lmax, dtype) with c slots needs about
 *                     wf_footprint(nside, lmax, dtype, c) plus 12 nside^2 * 8 c bytes
 *   max_slots         requests admitted at once, over all lanes (>= 1); a lane holds
 *                     at most min(max_slots, 16) slots, fewer if that exceeds half
 *                     the budget
 * Errors: WF_EINVAL, WF_ENOMEM, WF_EDEVICE.
 */
int wf_server_create(wf_server_t* out, size_t hbm_budget_bytes, int32_t max_slots);

/*
 * wf_server_submit -- queue one solve; copies every input and returns at once.
 *   cl (lmax+1), ninv, mask (npix, or NULL), d (npix): host doubles / bytes, as for
 *   wf_plan and wf_solve; lambda: host, nsweeps entries (Sect. 3's cooling)
 *   dtype     WF_F32, WF_BF16X6 or WF_BF16X3 (matrix-core Legendre contraction)
 *   ticket    receives the request's id for wf_server_poll
 * Errors: WF_EINVAL (as wf_plan / wf_solve), WF_EUNSUPPORTED (WF_F64),
 * WF_ENOMEM (a one-slot lane of this shape alone exceeds the budget), or the
 * status of a server stopped by a device error.
 */
int wf_server_submit(wf_server_t server, int32_t nside, int32_t lmax, const double* cl,
                     const double* ninv, const uint8_t* mask, const double* d,
                     const double* lambda, int32_t nsweeps, int32_t dtype, uint64_t* ticket);

/*
 * wf_server_poll -- WF_ENOTREADY while the request runs. When it has finished:
 * WF_OK, s_wf_host (npix doubles, or NULL) receives the signal map, latency_s
 * (or NULL) the seconds from submit to the result in host memory, and the ticket
 * is released. A request that failed returns its error once. Unknown or already
 * collected tickets: WF_EINVAL. Thread-safe.
 */
int wf_server_poll(wf_server_t server, uint64_t ticket, double* s_wf_host, double* latency_s);

/* wf_server_query -- counters; returns the error status of a stopped server, else WF_OK. */
int wf_server_query(wf_server_t server, wf_server_stats* out);

/*
 * wf_server_destroy -- stop both threads, drop queued requests, wait for the
 * device and free everything (NULL is accepted).
 */
void wf_server_destroy(wf_server_t server);

/*
 * Polarisation (Sect. 3: temperature and polarisation maps filtered together, with
 * separate temperature and polarisation masks). Each map is three fields T, Q, U;
 * each alm set three fields T, E, B. Per pixel the noise is a 3x3 covariance N_p, per
 * mode the signal covariance the 3x3 C_l of the TT, EE, BB and TE spectra (TB = EB = 0).
 *   - Spin-weighted harmonics sY_lm (Goldberg et al. 1967), Q +/- iU = sum_lm
 *     a_{+/-2,lm} (+/-2)Y_lm with a_{+/-2} = -(a_E +/- i a_B); the forward transform is the
 *     pixel-area-weighted adjoint, a_{+/-2,lm} = Omega sum_p (Q +/- iU)_p conj((+/-2)Y_lm(p)).
 *     E and B have no modes below l = 2 (those entries are 0 on output, ignored on input).
 *   - tau = 1 / max over pixels of the largest eigenvalue of N^-1_p (the largest T = tau 1
 *     with N - T positive semi-definite); Eq. (3) per pixel: t = s + W (d - s),
 *     W = lambda tau N^-1 (1 + (lambda - 1) tau N^-1)^-1; Eq. (4) per mode:
 *     s_lm = C_l (C_l + lambda tau Omega 1)^-1 a_lm.
 *   - Layouts: maps [map][field][npix] (T, Q, U; RING order), alm [map][field][N_lm]
 *     (T, E, B; packed as above), doubles (WF_F64 only); nside <= 512.
 */
typedef struct wf_pol_plan_s* wf_pol_plan_t;

/*
 * wf_pol_plan -- tables and work buffers of one polarised problem.
 *   nside    power of two in [1, 512]; lmax in [0, 4 nside - 1]
 *   cl       host, 4 (lmax+1) doubles: TT, EE, BB, TE spectra, one after another; every
 *            block [[TT, TE], [TE, EE]] positive semi-definite, BB >= 0, and EE = BB =
 *            TE = 0 at l < 2
 *   ninv     host, 6 npix doubles: the TT, QQ, UU, TQ, TU, QU entries of N^-1_p, one
 *            array of npix after another; every N^-1_p positive semi-definite
 *   mask     host, npix bytes: bit 0 set where T is observed, bit 1 where Q and U are
 *            (an unobserved field has its rows and columns of N^-1 set to 0); NULL =
 *            all observed
 *   opts     NULL, or dtype WF_F64, max_batch, flags 0 or WF_FLAG_TIMING
 * Errors: WF_EINVAL (shape, non-finite or indefinite input, no observed pixel),
 * WF_EUNSUPPORTED (another dtype), WF_ENOMEM, WF_EDEVICE. The plan copies its inputs.
 */
int wf_pol_plan(wf_pol_plan_t* out, int32_t nside, int32_t lmax, const double* cl,
                const double* ninv, const uint8_t* mask, const wf_plan_opts* opts,
                void* hip_stream);

/*
 * wf_pol_solve_batch -- the messenger iteration of nmaps polarised maps sharing the
 * plan's spectra, noise and masks, from s = t = 0, one sweep per lambda.
 *   d, s_wf  device, nmaps * 3 * npix doubles; s_alm device, nmaps * 3 * 2 N_lm doubles
 *            or NULL; lambda host, nsweeps entries, finite and > 0
 * WF_FLAG_TIMING fills stats->ms_ring (ring phase), ms_analysis (spin-0 T and spin-2
 * E/B analysis) and ms_synthesis (filter and both syntheses), and waits.
 * Errors: WF_EINVAL (NULL buffers, bad schedule, nmaps outside [1, max_batch]), WF_EDEVICE.
 */
int wf_pol_solve_batch(wf_pol_plan_t plan, int32_t nmaps, const void* d, void* s_wf,
                       void* s_alm, const double* lambda, int32_t nsweeps,
                       void* hip_stream, wf_stats* stats);

/* sht_pol_map2alm -- [T, Q, U] maps -> [T, E, B] alm of nmaps maps (device buffers as above). */
int sht_pol_map2alm(wf_pol_plan_t plan, int32_t nmaps, const void* map, void* alm,
                    void* hip_stream);

/* sht_pol_alm2map -- [T, E, B] alm -> [T, Q, U] maps (imaginary parts at m = 0 ignored). */
int sht_pol_alm2map(wf_pol_plan_t plan, int32_t nmaps, const void* alm, void* map,
                    void* hip_stream);

/* wf_pol_plan_info -- npix, N_lm, tau and the active (l, m, ring pair) triples of one
 * transform of one field (any pointer may be NULL). */
int wf_pol_plan_info(wf_pol_plan_t plan, int64_t* npix, int64_t* nalm, double* tau,
                     int64_t* units_active);

/* wf_pol_sync -- wait for the plan's stream work; reports asynchronous device errors. */
int wf_pol_sync(wf_pol_plan_t plan);

/* wf_pol_destroy -- free a polarised plan (NULL is accepted). */
void wf_pol_destroy(wf_pol_plan_t plan);

/* wf_sync -- wait for the plan's stream work; reports asynchronous device errors. */
int wf_sync(wf_plan_t plan);

/* wf_destroy -- free a plan and its device memory (NULL is accepted). */
void wf_destroy(wf_plan_t plan);

/* wf_strerror -- static text for a status code. */
const char* wf_strerror(int status);

/* wf_last_error -- detail of the last failure on this host thread ("" if none). */
const char* wf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MWF_H */
