/*
 * gtod.h -- C-ABI of the MI355X (gfx950) time-ordered-data simulator.
 *
 * The library simulates what a ground-based submillimetre IFU with kinetic
 * inductance detectors records (arXiv 2604.23305, section 2): for every
 * time sample t, spatial pixel p and frequency bin nu it samples the
 * moving PWV screen at the pixel's pointing, interpolates the zenith
 * transmission table and applies the airmass, propagates source plus sky
 * through the radiative-transfer cascade, contracts over frequency with the
 * channel responses to get the power per channel, and adds photon (white)
 * noise and 1/f (pink) noise.  Output: P_tot[p][k][t] in watts.
 *
 * Conventions for every call
 *   - Every call returns a gtod_status: 0 on success, a negative code on
 *     failure.  gtod_last_error() gives a message for the last failure on
 *     a context.
 *   - Angles are radians, frequencies Hz, temperatures K, PWV mm, spectral
 *     powers W/Hz, powers W.
 *   - "host" pointers are read during the call only; the caller keeps
 *     ownership and may free them on return.  "device" pointers are
 *     caller-owned device memory on the context's GPU that must stay valid
 *     until the stream passed to gtod_simulate_tod has passed the call.
 *   - A context is used by one host thread at a time.
 *   - Descriptors are validated before anything is enqueued: a failed call
 *     leaves no partial work behind.
 */
#ifndef GTOD_H
#define GTOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gtod_status;
#define GTOD_OK 0
#define GTOD_EINVAL (-1)        /* bad argument, shape or descriptor      */
#define GTOD_ENOMEM (-2)        /* device allocation failed               */
#define GTOD_EBUDGET (-3)       /* would exceed the context's HBM budget  */
#define GTOD_ENOTFOUND (-4)     /* unknown screen / spectral id           */
#define GTOD_ERANGE (-5)        /* pointing leaves the screen or the PWV
                                   leaves the table (STRICT_RANGE only)   */
#define GTOD_EDEVICE (-6)       /* HIP runtime error                      */
#define GTOD_EUNSUPPORTED (-7)  /* device is not gfx950                   */
#define GTOD_EIO (-8)           /* output file could not be written        */

typedef struct gtod_ctx gtod_ctx;

/* contraction precision */
#define GTOD_PREC_FP32 0        /* FP32 MFMA, FP32 accumulation          */
#define GTOD_PREC_SPLIT_BF16 1  /* hi+lo BF16 MFMA, FP32 accumulation    */

/* init flags */
#define GTOD_INIT_STRICT_RANGE 1u

/*
 * gtod_sim_init -- create a context on one GPU.
 *
 * The fixed telescope and detector parameters of section 2.3 live here:
 * taper, Ruze surface and polarisation efficiencies act on the source at
 * stage 0 (section 2.5); the superconducting gap Delta and pair-breaking
 * efficiency eta_pb enter the photon-noise NEP (section 2.6) and the
 * low-frequency cutoff h nu < 2 Delta; T_CMB is the blackbody behind the
 * source; f_sample converts NEP to the white-noise sigma.
 *
 * hbm_budget_bytes caps everything the context allocates (resident
 * screens, spectral tables and per-stream workspaces); 0 means 90% of the
 * free device memory.  workspace_bytes sizes each stream's scratch
 * (frequency panel and 1/f FFT scratch); 0 picks 1 GiB.
 *
 * Errors: EINVAL (NULL pointers, non-positive f_sample), EUNSUPPORTED
 * (not gfx950), EDEVICE, ENOMEM/EBUDGET (workspace).  *out is NULL on
 * failure.  Free the context with gtod_free(ctx, GTOD_OBJ_CTX, 0).
 */
typedef struct gtod_init_desc {
  int32_t device;
  int32_t precision;          /* default for jobs that pass -1            */
  uint32_t flags;             /* GTOD_INIT_*                              */
  int32_t reserved0;
  uint64_t hbm_budget_bytes;
  uint64_t workspace_bytes;
  double f_sample_hz;
  double eta_taper;           /* eta_t                                    */
  double rho_surf_m;          /* rms surface roughness for Ruze           */
  double eta_pol;             /* 0.5 for a single-polarisation detector  */
  double delta_J;             /* superconducting gap energy, J            */
  double eta_pb;              /* pair-breaking efficiency                 */
  double t_cmb_K;
} gtod_init_desc;

gtod_status gtod_sim_init(const gtod_init_desc* desc, gtod_ctx** out);

/*
 * gtod_load_screen -- make a PWV screen resident (section 2.2 and Eq.
 * xy_atm).  pwv_mm is [ny][nx] FP64, x contiguous; x is the wind axis.
 * Grid index of a screen position: gx = x/dx_m + ix0, gy = y/dy_m + iy0.
 * The screen moves with wind_mps along +x; h_column_m is the height of
 * the water-vapour column.  Bilinear sampling; positions outside the grid
 * take the edge value and are counted (gtod_get_counters), or fail the
 * simulate call with ERANGE when the context is STRICT_RANGE and the scan
 * is analytic.
 *
 * mem_kind 0: pwv_mm is host memory; 1: device memory.  The data are
 * deep-copied into library-owned memory charged to the budget; the call
 * is synchronous.  nx, ny >= 2.
 * Errors: EINVAL, EBUDGET, ENOMEM, EDEVICE.
 */
typedef struct gtod_screen_desc {
  const double* pwv_mm;
  int64_t nx, ny;
  double dx_m, dy_m, ix0, iy0;
  double h_column_m;
  double wind_mps;
  int32_t mem_kind;
  int32_t reserved0;
} gtod_screen_desc;

gtod_status gtod_load_screen(gtod_ctx* ctx, const gtod_screen_desc* desc,
                             int32_t* id);

/* optics stage kinds (stages after the atmosphere, section 2.5) */
#define GTOD_STAGE_REFLECT 0      /* eta(nu), couples to P_JN(t_K)        */
#define GTOD_STAGE_ATM_COUPLED 1  /* eta(nu), couples to the sky:
                                     (1-eta_atm) P_JN(T_atm)
                                     + eta_atm P_JN(T_CMB)               */
#define GTOD_STAGE_OHMIC 2        /* eta = 1 - eps_ref sqrt(nu/nu_ref)    */
#define GTOD_STAGE_REFRACTIVE 3   /* surface (t_refl_K), absorption
                                     exp(-2 pi d n tan(delta)/lambda)
                                     (t_K), surface; AR coating keeps only
                                     the absorbing pass                   */
typedef struct gtod_stage {
  int32_t kind;
  int32_t ar_coated;
  const double* eta;          /* host [F] or NULL to use eta_const        */
  double eta_const;
  double t_K;
  double t_refl_K;
  double eps_ref, nu_ref_hz;
  double d_m, n_index, tan_delta;
} gtod_stage;

/* channel-response modes (section 2.3) */
#define GTOD_FILT_LORENTZ 0     /* eta_peak / (1 + 4R^2 (nu/f - 1)^2)      */
#define GTOD_FILT_FILTERBANK 1  /* numerator eta_peak minus the responses
                                   of all upstream channels (strictly
                                   higher f; equal f: lower index first)  */
#define GTOD_FILT_MATRIX 2      /* user curves eta_filt[F][K]             */

/*
 * gtod_load_filters -- make the whole frequency-dimensional instrument
 * resident and precompute its tables on the device (FP64).
 *
 * nu_hz[F], w_hz[F]: bin centres and quadrature weights of the integrals
 *   over nu (P_KID and NEP^2 are sums of w_j * integrand_j).
 * eta_z[n_pwv][F]: zenith transmission at PWV pwv0_mm + i*dpwv_mm; it is
 *   interpolated linearly in optical depth -ln(eta_z) between rows, and
 *   PWV outside the axis is clamped to it.  t_atm_K: physical temperature
 *   of the atmosphere (stage 0).
 * stages[n_stage]: the optics stages after the atmosphere, in order.
 * Filters: K channels; f_hz, R, eta_peak [K] for LORENTZ / FILTERBANK, or
 *   eta_filt[F][K] (row-major, channel fastest) for MATRIX.  Rows with
 *   h nu < 2 Delta are zeroed (the KID gap cutoff).
 * ref_pwv_mm, ref_el_rad: operating point of the reference spectrum; the
 *   contraction is evaluated as (reference) + (deviation from it), which
 *   is exact algebra and keeps FP32 accumulation error proportional to the
 *   deviation.  The reference NEP^2 also sets the 1/f amplitude
 *   (gtod_job.pink_knee_hz).
 * All pointers are host memory.  Synchronous.
 * Errors: EINVAL (F < 1, K < 1, n_pwv < 2, bad mode/kind, non-positive
 * weights or dpwv, a padded response plane of 4 GiB or more -- F and K
 * rounded up to multiples of 32, times 4 bytes -- or F rounded up to a
 * multiple of 32 above 4194303), EBUDGET, ENOMEM, EDEVICE.
 */
typedef struct gtod_spectral_desc {
  int32_t F;
  int32_t K;
  const double* nu_hz;
  const double* w_hz;
  int32_t n_pwv;
  int32_t filter_mode;
  double pwv0_mm, dpwv_mm;
  const double* eta_z;
  double t_atm_K;
  int32_t n_stage;
  int32_t reserved0;
  const gtod_stage* stages;
  const double* f_hz;
  const double* R;
  const double* eta_peak;
  const double* eta_filt;
  double ref_pwv_mm;
  double ref_el_rad;
} gtod_spectral_desc;

gtod_status gtod_load_filters(gtod_ctx* ctx, const gtod_spectral_desc* desc,
                              int32_t* id);

/* job kinds */
#define GTOD_JOB_SIGNAL 0   /* power, photon noise: rows [t_begin,t_end)  */
#define GTOD_JOB_PINK 1     /* 1/f noise: all t_total samples             */
/* scan kinds (section 2.4) */
#define GTOD_SCAN_STARE 0   /* (phi, theta) = (0, 0)                      */
#define GTOD_SCAN_DAISY 1   /* Eq. daisy: params {r_petal, omega, Omega}  */
#define GTOD_SCAN_TRAJ 2    /* user pattern: device double traj[t_total][2]
                               holding (phi, theta) per sample            */
/* job flags */
#define GTOD_JOB_PHOTON_NOISE 1u  /* add sigma*z (SIGNAL)                 */
#define GTOD_JOB_ACCUMULATE 2u    /* add into tod instead of overwriting  */
#define GTOD_JOB_KELVIN 4u        /* tod in K on the skydip scale (SIGNAL:
                                     (P - a_k) / b_k plus noise / b_k;
                                     PINK: noise / b_k); needs gtod_skydip */

/*
 * One unit of work for gtod_simulate_tod.
 *
 * Pixels: n_pix spaxels with pointing offsets dphi_rad/dtheta_rad (host
 *   [n_pix]).  Pixel p of the job keys the noise counters as pixel
 *   pix0 + p, so that a job covering spaxels [pix0, pix0 + n_pix) of a
 *   larger array draws the same noise as one job over the whole array.
 * Scan: (phi(t), theta(t)) around the scan offset (phi0, theta0), t =
 *   n / f_sample for absolute sample n.  Screen coordinates use
 *   phi(t)+dphi, theta(t)+dtheta (Eq. xy_atm); the airmass and the source
 *   use the full pointing phi(t)+phi0+dphi, theta(t)+theta0+dtheta.
 * Source: pre-convolved P_nu,src cube (device float [n_el][n_az][cube_ld],
 *   cube_ld >= F spectral stride), node (i_az, i_el) at (az0 + i_az*daz,
 *   el0 + i_el*del); bilinear inside the closed grid, zero outside; NULL
 *   for no source.
 * Samples: SIGNAL computes rows t in [t_begin, t_end) of a t_total-long
 *   observation; PINK computes all t_total samples of every (p, k) series.
 * Noise: seed keys Philox4x32-10 with key (seed mod 2^32, seed >> 32);
 *   white noise of sample (t, k, p) uses counter (t, k, p, 0), bin j of
 *   the 1/f spectrum of series (p, k) uses counter (j, k, p, 1).
 *   PINK: one-sided PSD A_k f^-alpha_k in W^2/Hz (section 2.6), with
 *   pink_alpha host [K]; the levels are pink_A host [K] (A_k >= 0, finite)
 *   when it is non-NULL, else A_k = NEP^2_ref,k * pink_knee_hz^alpha_k (the
 *   1/f PSD meets the white photon-noise PSD of the reference spectrum at
 *   the knee).  t_total <= 2^25 for PINK jobs.
 * Outputs (device, caller-owned; layout [n_pix][K][out_ld], time fastest,
 *   holding samples [out_t0, out_t0 + out_ld); out_ld = 0 means out_t0 = 0
 *   and out_ld = t_total):
 *   tod (required): power (+ noise) in W, or brightness temperature in K
 *   with GTOD_JOB_KELVIN.  p_kid, sigma (optional, SIGNAL): noise-free
 *   power and photon-noise sigma, always in W.  pwv (optional, SIGNAL):
 *   [n_pix][out_ld] zenith PWV sampled at each row.
 *   SIGNAL needs out_t0 <= t_begin and t_end <= out_t0 + out_ld; PINK
 *   needs out_t0 = 0 and out_ld >= t_total.
 */
typedef struct gtod_job {
  int32_t kind;
  int32_t screen_id;
  int32_t spec_id;
  int32_t n_pix;
  const double* dphi_rad;
  const double* dtheta_rad;
  int32_t scan_kind;
  int32_t precision;          /* GTOD_PREC_* or -1 for the ctx default    */
  double phi0_rad, theta0_rad;
  double scan_params[8];
  const double* traj;
  const float* cube;
  int32_t n_az, n_el;
  int64_t cube_ld;
  double az0_rad, daz_rad, el0_rad, del_rad;
  int64_t t_begin, t_end, t_total;
  uint64_t seed;
  uint32_t flags;
  int32_t pix0;               /* noise-key index of pixel 0 (default 0)   */
  const double* pink_alpha;
  double pink_knee_hz;        /* used when pink_A is NULL                 */
  const double* pink_A;       /* host [K] 1/f levels (W^2/Hz) or NULL     */
  int64_t out_t0, out_ld;
  float* tod;
  float* p_kid;
  float* sigma;
  float* pwv;
} gtod_job;

/*
 * gtod_simulate_tod -- enqueue n_jobs jobs on hip_stream (a hipStream_t;
 * NULL for the legacy default stream) and return without waiting.
 * All jobs are validated first; on any error nothing is enqueued.  Host
 * arrays named by the jobs are consumed before return.  The jobs of a call
 * run one after another, in array order.  Each stream gets its own
 * workspace on first use, kept until the context is freed; calls on one
 * stream run in order.
 * Errors: EINVAL, ENOTFOUND, ERANGE (STRICT_RANGE), EBUDGET (first use of
 * a stream), EDEVICE (outputs are undefined afterwards).
 */
gtod_status gtod_simulate_tod(gtod_ctx* ctx, const gtod_job* jobs,
                              int32_t n_jobs, void* hip_stream);

/*
 * gtod_simulate_tod_noalloc -- gtod_simulate_tod for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  It allocates nothing (no
 * hipMalloc, hipFree, hipHostMalloc or allocating library routine); the
 * caller still passes inputs and outputs, as for gtod_simulate_tod.
 *
 * Jobs, validation, ordering and results are those of gtod_simulate_tod:
 * the outputs are bit-identical, since no result depends on how rows or
 * series are chunked.  The device scratch (panel, row order, 1/f transform
 * scratch and the staged job parameters) is a static array of
 * GTOD_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs
 * on, from its first use there until the process ends, outside every
 * context's HBM budget.  The pinned host staging and its events are made
 * by gtod_sim_init.
 *
 * Sharing: every call on one GPU -- from any context, stream or host
 * thread -- uses that GPU's one array, and it keeps the last call's
 * contents.  Calls on one stream run in order; calls that overlap on one
 * GPU (other streams, other host threads) race and their outputs are
 * undefined.
 *
 * Limits: a SIGNAL job needs at least 128 rows of 4 F_pad + 56 bytes
 * (F_pad = F rounded up to 32), and a PINK job of t_total samples needs
 * 4 N bytes per series plus 64 KiB (N = the power of two >= t_total);
 * both must fit in GTOD_NOALLOC_SCRATCH_BYTES - 8 MiB.  Larger jobs are
 * rejected with EINVAL before anything is enqueued.
 * Errors: those of gtod_simulate_tod, except EBUDGET.
 */
#define GTOD_NOALLOC_SCRATCH_BYTES (256ull << 20)
gtod_status gtod_simulate_tod_noalloc(gtod_ctx* ctx, const gtod_job* jobs,
                                      int32_t n_jobs, void* hip_stream);

/*
 * gtod_skydip -- brightness-temperature scale of a spectral setup by a
 * simulated skydip (section 2.7): the sky brightness is varied through the
 * zenith PWV while the detected power is recorded, and a linear map between
 * power and line-of-sight brightness temperature is fitted per channel.
 *
 * Sweep: n zenith PWV values evenly spaced over [pwv_lo_mm, pwv_hi_mm]
 *   (both ends included) at elevation el_rad (airmass 1/sin el), no
 *   source, no noise; PWV outside the table axis is clamped to it (ERANGE
 *   instead under GTOD_INIT_STRICT_RANGE).
 * Row i, channel k (all FP64):
 *   p_kid[i][k] = sum_j w_j eta_jk P_j,   P = cascade output (Eq. radtrans)
 *   t_b[i][k]   = T_atm sum_j w_j eta_jk (1 - eta_atm,j) / sum_j w_j eta_jk
 * Fit: least-squares line p_kid = a_k + b_k t_b over the n rows.  A channel
 *   with no response, or whose t_b does not vary, gets a_k = b_k = NaN.
 * The scale is kept with the spectral setup (replacing an earlier one) and
 *   used by jobs with GTOD_JOB_KELVIN.
 * Outputs (host, caller-owned, each may be NULL): a_out, b_out [K] in W and
 *   W/K; p_kid_out, t_b_out [n][K] in W and K.
 * Synchronous: waits for all work on the device first, allocates
 *   2 n F + 2 n K doubles of temporaries for the call.  A call that runs
 *   while another host thread enqueues KELVIN jobs of the same setup races.
 * Errors: ENOTFOUND, EINVAL (el_rad outside (0, pi), pwv_lo_mm >= pwv_hi_mm,
 *   n outside [2, GTOD_SKYDIP_MAX_N]), ERANGE, EBUDGET, ENOMEM, EDEVICE.
 */
#define GTOD_SKYDIP_MAX_N 16384
gtod_status gtod_skydip(gtod_ctx* ctx, int32_t spec_id, double el_rad,
                        double pwv_lo_mm, double pwv_hi_mm, int32_t n,
                        double* a_out, double* b_out, double* p_kid_out,
                        double* t_b_out);

/*
 * gtod_reduce -- common-mode atmosphere subtraction and inverse-variance
 * gridding of a brightness-temperature TOD (section 4.3, Eqs. common_mode
 * and Sj), enqueued on hip_stream.
 *
 * Input: tod [n_pix][K][ld] in K (a GTOD_JOB_KELVIN output of the same
 *   spectral setup and scan) holding samples [t0, t0 + T) of the
 *   observation.  The scan (scan_kind, scan_params, theta0_rad, traj with
 *   t_total rows) and the spaxel offsets (host [n_pix]) are those of the
 *   simulation.
 * Atmosphere: the mean zenith PWV is the mean of pwv (device [n_pix]
 *   [pwv_ld], its first pwv_len columns: the SIGNAL job's PWV output), or
 *   pwv_mean_mm when pwv is NULL.  Channel k's zenith transmission is the
 *   response-weighted mean of the table's transmission at that PWV, and
 *   spaxel i sees eta_i = eta_z,k ^ (1 / sin(theta(t) + theta0 + dtheta_i)).
 * Common mode: S_j = 1 for the spaxels with sqrt(dphi^2 + dtheta^2) >
 *   r_out_rad (at least one is required), and
 *     T*_i = T_b,i / eta_i - (1 - eta_i) / (eta_i N_out)
 *            sum_j S_j T_b,j / (1 - eta_j).
 *   t_star (device [n_pix][K][ld], optional) receives T* in K.
 * Maps (optional; map and weight both NULL or both set, device
 *   [K][map_n][map_n], FP64): sample t of spaxel i falls in the nearest
 *   node of the map_n x map_n grid spanning +-map_half_rad around the
 *   pointing centre, at (phi(t) + dphi_i, theta(t) + dtheta_i); samples
 *   more than half a node spacing outside the grid are dropped.  Per
 *   spaxel, channel and cell the samples' mean and unbiased variance s^2
 *   (m >= 2 samples, s^2 > 0) give weight m / s^2; map = sum w mean /
 *   sum w over the spaxels, weight = sum w (NaN and 0 for no contribution).
 *   Cell sums use LDS atomics, so maps can differ between runs in the last
 *   bits.
 * Uses the stream's workspace (channels are processed in groups that fit).
 * Errors: EINVAL (shapes, no output requested, map_n outside
 *   [2, GTOD_MAP_MAX_N], no off-source spaxel, workspace too small for one
 *   channel), ENOTFOUND, EBUDGET, EDEVICE.
 */
#define GTOD_MAP_MAX_N 48
typedef struct gtod_reduce_desc {
  int32_t spec_id;
  int32_t n_pix;
  const double* dphi_rad;      /* host [n_pix] */
  const double* dtheta_rad;    /* host [n_pix] */
  int32_t scan_kind;
  int32_t map_n;
  double theta0_rad;
  double scan_params[8];
  const double* traj;          /* device [t_total][2] for GTOD_SCAN_TRAJ */
  int64_t t_total;
  int64_t t0, T, ld;
  const float* tod;            /* device [n_pix][K][ld], K */
  const float* pwv;            /* device [n_pix][pwv_ld] or NULL */
  int64_t pwv_ld, pwv_len;
  double pwv_mean_mm;
  double r_out_rad;
  double map_half_rad;
  float* t_star;               /* device [n_pix][K][ld] or NULL */
  double* map;                 /* device [K][map_n][map_n] or NULL */
  double* weight;              /* device [K][map_n][map_n] or NULL */
} gtod_reduce_desc;
gtod_status gtod_reduce(gtod_ctx* ctx, const gtod_reduce_desc* desc,
                        void* hip_stream);

/*
 * gtod_simulate_to_disk -- out-of-core run: simulate a whole observation
 * in pixel groups and stream each group's TOD device -> pinned host ->
 * disk, for outputs larger than the HBM one wants to give them (the
 * paper's RAM manager, section 1, and its output files, section 2.7).
 *
 * signal: a SIGNAL job over the whole observation (t_begin = 0, t_end =
 *   t_total; its output pointers and pix0 are ignored).  pink: NULL, or a
 *   PINK job of the same spec_id, n_pix, t_total and seed.  KELVIN and
 *   PHOTON_NOISE flags apply as in gtod_simulate_tod.
 * Groups: pixels [g G, g G + G) with G = pix_per_group, or as many as
 *   device_bytes allows for two slabs (n_pix_group x K x t_total floats,
 *   plus n_pix_group x t_total for the PWV); each group runs as one
 *   gtod_simulate_tod call with pix0 = g G, so the file holds exactly what
 *   one in-memory run over all pixels would give.  While group g + 1 is
 *   computed, group g is copied to host through host_bytes of pinned
 *   staging (two halves) and written by a writer thread.
 * Files in dir (created or overwritten, NumPy .npy format version 1.0):
 *   tod.npy  float32 [n_pix][K][t_total] (W, or K with GTOD_JOB_KELVIN)
 *   pwv.npy  float32 [n_pix][t_total] zenith PWV (GTOD_SINK_PWV)
 *   time.npy float64 [t_total] seconds from the start (n / f_sample)
 * Synchronous: returns when every file is complete.  stats (host [4], may
 *   be NULL): wall seconds, bytes written, groups, pixels per group.
 * Errors: EINVAL (jobs, a group of one pixel does not fit device_bytes,
 *   host_bytes < 2 MiB), EBUDGET, ENOMEM, EIO (files), EDEVICE, and the
 *   errors of gtod_simulate_tod.
 */
#define GTOD_SINK_PWV 1u
typedef struct gtod_sink_desc {
  const char* dir;
  uint64_t device_bytes;
  uint64_t host_bytes;
  uint32_t flags;
  int32_t pix_per_group;      /* 0: as many as device_bytes allows        */
} gtod_sink_desc;
gtod_status gtod_simulate_to_disk(gtod_ctx* ctx, const gtod_job* signal,
                                  const gtod_job* pink,
                                  const gtod_sink_desc* sink, double* stats);

/* ---- input preparation (section 2.2) ---------------------------------
 * Aperture illumination (Eq. aper_dist, circularly symmetric Gaussian
 * with edge taper t_edge_db, negative, at the rim): A(r) = 10^(t_edge_db
 * (r / r_tel_m)^2 / 20) for r < r_tel_m, else 0.
 */

/*
 * gtod_far_field -- peak-normalised far-field power pattern F = |FT{A}|^2
 * (section 2.2), evaluated exactly for the circularly symmetric aperture as
 * the square of its Hankel transform, H(rho) = int_0^R A(r) J0(2 pi rho r
 * / lambda) r dr, over F frequencies nu_hz (host [F]) on the grid rho =
 * sqrt((a da_rad)^2 + (b db_rad)^2), a < n_a, b < n_b.
 * Output: out (device [F][n_b][n_a], FP32).  Enqueued on hip_stream.
 * Errors: EINVAL (sizes, spacings, r_tel_m <= 0, a grid too oscillatory
 *   for the quadrature: 2 pi rho_max r_tel / lambda_min > 6000).
 */
gtod_status gtod_far_field(gtod_ctx* ctx, const double* nu_hz, int32_t F,
                           int32_t n_a, int32_t n_b, double da_rad,
                           double db_rad, double r_tel_m, double t_edge_db,
                           float* out, void* hip_stream);

/*
 * gtod_convolve_source -- spectral source power from specific intensity
 * (Eq. convolve_src): on the source grid az_i = az0 + i daz, el_j = el0 +
 * j del (i < n_az, j < n_el),
 *   P(i, j, f) = A_p daz del sum_{i', j'} I(i', j', f) cos(el_j')
 *                F_f(sqrt(((i - i') daz)^2 + ((j - j') del)^2)),
 * A_p = pi r_tel_m^2, F_f the far field above at nu_hz[f].
 * in: device [n_el][n_az][ld_in] float (W m^-2 Hz^-1 sr^-1); out: device
 *   [n_el][n_az][ld_out] float (W/Hz), the cube layout gtod_job takes;
 *   in and out must not overlap.  n_az n_el <= 20000.
 * Uses the stream's workspace for far-field tables (frequencies in
 *   batches that fit).  Errors: EINVAL, EDEVICE.
 */
gtod_status gtod_convolve_source(gtod_ctx* ctx, const float* in,
                                 int32_t n_az, int32_t n_el, int64_t ld_in,
                                 const double* nu_hz, int32_t F,
                                 double daz_rad, double el0_rad,
                                 double del_rad, double r_tel_m,
                                 double t_edge_db, float* out,
                                 int64_t ld_out, void* hip_stream);

/*
 * gtod_convolve_screen -- line-of-sight PWV screen by the aperture
 * footprint (section 2.2): each cell becomes the A-weighted mean of the
 * cells whose centres lie within r_tel_m (weights A(r) normalised to 1;
 * half widths floor(r_tel_m / dx_m) <= 32 and floor(r_tel_m / dy_m) <= 32
 * cells), indices clamped at the screen edges.  in, out: device [ny][nx]
 * double, not overlapping.  Enqueued on hip_stream.  Errors: EINVAL,
 * EDEVICE.
 */
gtod_status gtod_convolve_screen(gtod_ctx* ctx, const double* in, int64_t nx,
                                 int64_t ny, double dx_m, double dy_m,
                                 double r_tel_m, double t_edge_db,
                                 double* out, void* hip_stream);

/* object kinds for gtod_free */
#define GTOD_OBJ_SCREEN 0
#define GTOD_OBJ_SPEC 1
#define GTOD_OBJ_CTX 2
/*
 * gtod_free -- release a resident screen or spectral setup (after the
 * device has finished all work queued so far), or the whole context
 * (id ignored).  Returns the memory to the budget.
 * Errors: ENOTFOUND for an unknown id, EINVAL for a bad kind.
 */
gtod_status gtod_free(gtod_ctx* ctx, int32_t kind, int32_t id);

/*
 * gtod_release_stream -- free the workspace a stream acquired on its first
 * gtod_simulate_tod call (panel, 1/f scratch, staging), after waiting for
 * the work already enqueued on it; its bytes return to the budget.  A
 * later call on the stream allocates a new workspace.  For callers that
 * retire streams, so that a long-running process does not keep one
 * workspace per stream it ever used.
 * Errors: ENOTFOUND (the stream has no workspace), EDEVICE.
 */
gtod_status gtod_release_stream(gtod_ctx* ctx, void* hip_stream);

/* ---- utilities (not part of the simulation path) ---------------------- */

/* Message for the last failed call on ctx (NULL ctx: last init failure). */
const char* gtod_last_error(const gtod_ctx* ctx);

/* Bytes currently charged to the budget, and the budget itself. */
gtod_status gtod_memory(const gtod_ctx* ctx, uint64_t* used, uint64_t* budget);

/* Range events since init.  Per row (pixel, sample): out[0] screen
 * positions clamped to the edge, out[1] PWV values clamped to the table
 * axis, out[2] elevations theta(t) + theta0 + dtheta outside (0, pi),
 * where the airmass 1/sin(el) of Eq. airmass is undefined (only a
 * GTOD_SCAN_TRAJ trajectory can reach one; analytic scans are rejected
 * before launch, and the outputs of such rows are undefined).  Per (row,
 * frequency bin): out[3] spectra that deviate from the setup's reference
 * spectrum (ref_pwv_mm, ref_el_rad) by more than 1/8 of their power,
 * |P - P_ref| > P / 8.  While out[3] stays 0 both contraction precisions
 * keep P_KID within 1e-6 of exact arithmetic (the split path represents
 * the deviations with 16 bits); beyond, the error grows with |dP| / P and
 * a reference closer to the observing conditions restores it.
 * Synchronises the device. */
gtod_status gtod_get_counters(gtod_ctx* ctx, uint64_t out[4]);

/* Reference NEP^2 per channel (W^2/Hz) of a spectral setup: the photon-
 * noise level of the reference spectrum.  out: host [K]. */
gtod_status gtod_spec_nep2_ref(gtod_ctx* ctx, int32_t spec_id, double* out);

/* Raw Philox4x32-10 words for n counters (device uint32 ctr[n][4] in,
 * device uint32 out[n][4]) under key (seed mod 2^32, seed >> 32), on the
 * given stream: the same generator the noise kernels use. */
gtod_status gtod_philox(gtod_ctx* ctx, const uint32_t* ctr, uint32_t* out,
                        int64_t n, uint64_t seed, void* hip_stream);

/* Per-kernel timing.  While enabled, every kernel launch is bracketed by
 * HIP events recorded on its launch stream.  gtod_profile_enable(ctx, 1)
 * clears the totals and starts; 0 stops.  gtod_profile_read synchronises
 * the device and writes, for each kernel id k < n_kernels,
 * out[3k] = total milliseconds, out[3k+1] = launches, out[3k+2] =
 * algorithmic work: for the panel, bytes (20F + 32 per row: four source
 * spectra, the deviation row, four screen values); for the contractions,
 * FLOP (6 K F per row: three products); for the 1/f passes, complex
 * points; for the common-mode and gridding kernels of gtod_reduce, bytes
 * (4 per TOD sample read, 4 per T* sample written, 8 per channel and sample
 * of the common-mode term, 16 per spaxel, channel and cell of statistics);
 * for the far-field table, quadrature terms (one J0 each); for the source
 * and screen convolutions, FLOP (2 per tap and output). */
#define GTOD_KERNEL_PANEL 0
#define GTOD_KERNEL_GEMM_F32 1
#define GTOD_KERNEL_GEMM_BF16 2
#define GTOD_KERNEL_PINK1 3
#define GTOD_KERNEL_PINK2 4
#define GTOD_KERNEL_COMMON 5
#define GTOD_KERNEL_GRID 6
#define GTOD_KERNEL_BEAM 7
#define GTOD_KERNEL_SRC_CONV 8
#define GTOD_KERNEL_SCREEN_CONV 9
#define GTOD_N_KERNELS 10
gtod_status gtod_profile_enable(gtod_ctx* ctx, int32_t enable);
gtod_status gtod_profile_read(gtod_ctx* ctx, double* out, int32_t n_kernels);

/* sizeof of the descriptor structs, for binding checks (no device use):
 * out[0..5] = init, screen, stage, spectral, job, reduce. */
void gtod_abi_sizes(int64_t out[6]);

#ifdef __cplusplus
}
#endif
#endif /* GTOD_H */
