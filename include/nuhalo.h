/*
 * nuhalo.h -- C ABI of libnuhalo.so: relic overdensity profiles n(r)/nbar
 * around a spherically symmetric, time-evolving NFW halo by backward N-1-body
 * integration and a Liouville momentum-space quadrature, on one MI355X (gfx950).
 *
 * Method: Worku, Sabti & Kamionkowski, arXiv:2410.08267.
 *   - background and equations of motion: Sec. II.A, Eq. (eoms)
 *   - halo model: Sec. II.B, Eqs. (rhototal), (nfw); enclosed mass App. A
 *   - backward integration and Liouville map: Sec. II.C
 *   - momentum-space quadrature: Eqs. (density_integral), (localdensity) and
 *     the background density that follows them
 *   - grids and mass-independence of the orbits: Sec. II.D
 *   - halo-growth variants and G(z): Sec. IV.A, IV.B
 *
 * Conventions for every entry point:
 *   - Return value: NH_OK (0) or a negative NH_E* code.  No exception or
 *     longjmp crosses this boundary.  nh_last_error(ctx) holds a message for
 *     the last failing call on that context (thread-local per context use).
 *   - Host input arrays are read (copied) before the call returns; the caller
 *     may free or reuse them afterwards.
 *   - Output buffers belong to the caller.  "host" buffers are ordinary host
 *     memory; "device" buffers are HIP device allocations on the context's
 *     device (for example a torch tensor's data_ptr()).
 *   - Streams are hipStream_t values passed as void*; NULL is the null stream.
 *   - Units: radii in comoving kpc, velocities in km/s, masses in Msun,
 *     H0 in km/s/Mpc, temperatures in K, relic mass in eV.
 *   - All floating-point inputs must be finite.
 */
#ifndef NUHALO_H
#define NUHALO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define NH_OK          0
#define NH_EINVAL     (-1)  /* invalid request or argument; nothing was launched */
#define NH_ENOMEM     (-2)  /* host or device allocation failed */
#define NH_EDEVICE    (-3)  /* a HIP call failed; nh_last_error has HIP's text */
#define NH_ESTEPS     (-4)  /* some trajectories hit max_steps or a step underflow;
                               the profile is still written, see nh_stats */
#define NH_ENONFINITE (-5)  /* a trajectory state became non-finite; profile written */
#define NH_EBUSY      (-6)  /* serving: the request does not fit the free budget now */
#define NH_ENOTREADY  (-7)  /* serving: the ticket has not completed yet */
#define NH_ENOTFOUND  (-8)  /* serving: unknown or already collected ticket */
#define NH_ECANCELED  (-9)  /* serving: the ticket was cancelled */

/* ---- request ---------------------------------------------------------- */

/* Flat FRW background, H(z) = H0 [Om (1+z)^3 + OL]^(1/2) (Sec. II.A).
 * |Omega_m + Omega_L - 1| must be <= 1e-12 and Omega_m > 0. */
typedef struct {
    double H0_km_s_Mpc;
    double Omega_m;
    double Omega_L;
} nh_cosmology;

/* Halo mass history M(z) (Sec. II.B, IV.A). */
enum {
    NH_MASS_ZERO        = 0,  /* no halo: free streaming, n/nbar = 1 */
    NH_MASS_PAPER       = 1,  /* M0 * xi(z)^alpha, xi = clamp((z_form - z)/z_form, 0, 1) */
    NH_MASS_EXPONENTIAL = 2,  /* M0 * exp(-beta z) */
    NH_MASS_TABLE       = 3   /* sampled: halo.history.M_Msun (M0 unused) */
};
/* Concentration history c(z). */
enum {
    NH_CONC_CONSTANT = 0,     /* c0 */
    NH_CONC_POWER    = 1,     /* c0 * (1+z)^(-gamma) */
    NH_CONC_TABLE    = 2      /* sampled: halo.history.c */
};
/* Modulation of Newton's constant, G -> kappa(z) G (Sec. IV.B). */
enum {
    NH_KAPPA_NONE     = 0,    /* kappa = 1 */
    NH_KAPPA_LOG      = 1,    /* 1 + a ln(1+z) */
    NH_KAPPA_PAPER    = 2,    /* 1 + a [z/(1+z)]^b */
    NH_KAPPA_CONSTANT = 3,    /* a */
    NH_KAPPA_TABLE    = 4     /* sampled: halo.history.kappa */
};

/* Histories given as samples (any halo growth model, Sec. IV.A; any G(z),
 * Sec. IV.B).  Sample i is the value at u_i = u_min + i (0 - u_min)/(n-1),
 * u = ln a = -ln(1+z), u_min = -ln(1 + z_max); i = n-1 is z = 0.  Between
 * samples the value is the not-a-knot cubic spline through all samples (twice
 * continuously differentiable, exact for cubics; with n = 4 the single cubic
 * through them).  n >= 4, z_max >= integ.z_end.  Masses >= 0 with M(0) > 0;
 * concentrations > 0 (also between samples); kappa finite.  Arrays are read
 * only for the kinds set to *_TABLE and may be NULL otherwise. */
typedef struct {
    int           n;
    double        z_max;
    const double *M_Msun;    /* host, n */
    const double *c;         /* host, n */
    const double *kappa;     /* host, n */
} nh_history;
/* Halo geometry. */
enum {
    NH_GEOM_PAPER    = 0,     /* Sec. II.B: R from M(0) via M = (4 pi/3) R^3 rhobar_m0;
                                 fixed physical r200 = R / 200^(1/3); comoving truncation
                                 radius r200 (1+z); scale radius r200 (1+z) / c(z) */
    NH_GEOM_DELTA200 = 1      /* R(z) from M(z); truncation radius R(z)/200^(1/3) comoving */
};

/* The halo.  With compensated = 1 (Sec. II.B) the enclosed mass perturbation is
 *   M(z) [I(r/s)/I(c) - (r/R)^3]  inside the truncation radius,
 *   M(z) [1 - (r/R)^3]            out to R,  0 beyond,
 * with I(q) = ln(1+q) - q/(1+q); compensated = 0 drops the (r/R)^3 terms and
 * the cutoff (plain NFW inside, point mass outside). */
typedef struct {
    int    mass_kind;    /* NH_MASS_* */
    double M0_Msun;      /* > 0 unless NH_MASS_ZERO */
    double mass_alpha;   /* NH_MASS_PAPER: exponent of xi (1 in the base model) */
    double z_form;       /* NH_MASS_PAPER: z_i, 200^(1/3) - 1 in the base model; > 0 */
    double mass_beta;    /* NH_MASS_EXPONENTIAL: rate */
    int    conc_kind;    /* NH_CONC_* */
    double c0;           /* > 0 */
    double conc_gamma;
    int    kappa_kind;   /* NH_KAPPA_* */
    double kappa_a;
    double kappa_b;
    int    geometry;     /* NH_GEOM_*; NH_GEOM_PAPER needs z_end <= 200^(1/3) - 1 */
    int    compensated;  /* 1 (paper) or 0 */
    nh_history history;  /* samples for the *_TABLE kinds */
} nh_halo;

/* Initial (pre-halo) phase-space distribution of the relic, y = P / (k_B T). */
enum {
    NH_F0_FERMI_DIRAC = 0,    /* 1 / (1 + e^y)  (Sec. II.C) */
    NH_F0_FREEZE_IN   = 1,    /* y^(-1/2) e^(-y) (Sec. IV.B; normalisation cancels) */
    NH_F0_TABLE       = 2     /* sampled: ln f0 at ln y_i = ln_y0 + i d_ln_y, i = 0..n-1
                                 (n >= 4, d_ln_y > 0); inside the range the cubic through
                                 the four samples around ln y (stencil shifted inward at
                                 the ends), outside it continued linearly with the slope
                                 of the end interval (power-law tails, Sec. IV.B) */
};
typedef struct {
    int           kind;      /* NH_F0_* */
    double        T_K;       /* > 0; 1.95 K for the neutrino background */
    int           n;         /* NH_F0_TABLE */
    double        ln_y0;
    double        d_ln_y;
    const double *ln_f;      /* host, n, finite; the normalisation cancels */
} nh_f0;

/* Grid.  Trajectory t = (k * n_y + j) * n_mu + l starts at x0 = (r_k, 0) with
 * v0 = V_j (mu_l, sqrt(1 - mu_l^2)), V_j = y_j k_B T c / m (Sec. II.C, II.D).
 * r_kpc > 0; y > 0 strictly ascending (n_y >= 2); |mu| < 1.
 * mu == NULL: n_mu Gauss-Legendre nodes and weights on [-1, 1] (w_mu ignored).
 * The |p| weights are y_j^3 dlny_j, trapezoid in ln y with half weights at the ends. */
typedef struct {
    int           n_r;
    const double *r_kpc;     /* host, n_r */
    int           n_y;
    const double *y;         /* host, n_y */
    int           n_mu;
    const double *mu;        /* host, n_mu, or NULL */
    const double *w_mu;      /* host, n_mu, required when mu != NULL */
} nh_grid;

/* Integrator, in u = ln a from -ln(1 + z_obs) (0 for observation today) down to
 * -ln(1 + z_end). */
enum {
    NH_RK4    = 0,           /* classical RK4, n_steps equal steps */
    NH_DOPRI5 = 1            /* Dormand-Prince 5(4), adaptive */
};
enum {
    NH_FP64  = 0,            /* FP64 state and arithmetic */
    NH_FP32C = 1             /* FP32 state with compensated position / time sums;
                                FP64 tables, promoted steps and quadrature */
};
/* Dormand-Prince step control: err = RMS over (x, y, vx, vy) of E_i / sc_i with
 * sc = atol + rtol * max(|.|_n, |.|_{n+1}) (Euclidean norm of the position pair
 * for x, y and of the velocity pair for vx, vy); accept err <= 1; next step
 * h * min(5, max(0.2, 0.9 err^(-1/5))), capped at 1x right after a rejection;
 * the last step lands on u_end. */
typedef struct {
    int       method;        /* NH_RK4 | NH_DOPRI5 */
    int       n_steps;       /* NH_RK4: >= 1 */
    double    rtol;          /* NH_DOPRI5: > 0 */
    double    atol_x;        /* kpc; <= 0 means rtol * 1 kpc */
    double    atol_v;        /* km/s; <= 0 means rtol * 1 km/s */
    double    h0;            /* first trial step in u; 0 means -1e-3 */
    long long max_steps;     /* attempted-step budget per trajectory; <= 0 means 1e6 */
    double    z_end;         /* > z_obs */
    int       precision;     /* NH_FP64 | NH_FP32C (NH_FP32C needs NH_DOPRI5) */
    double    z_obs;         /* >= 0: the profile is observed at z_obs (the paper's z0, Sec. II.B):
                                integration runs from u = -ln(1+z_obs); the halo's reference
                                epoch is z_obs (NH_GEOM_PAPER: R from M(z_obs), fixed physical
                                r200 = R / ((1+z_obs) 200^(1/3)), z_end <= (1+z_obs) 200^(1/3) - 1;
                                NH_MASS_PAPER: xi = (z_form - z) / (z_form - z_obs)) */
} nh_integrator;

typedef struct {
    nh_cosmology  cosmo;
    nh_halo       halo;
    double        m_eV;      /* relic mass, > 0 */
    nh_f0         f0;
    nh_grid       grid;
    nh_integrator integ;
} nh_request;

/* Per-solve statistics. */
typedef struct {
    long long n_traj;              /* trajectories in the request */
    long long accepted_steps;      /* sum over trajectories */
    long long rejected_steps;      /* sum over trajectories */
    long long max_steps_one_traj;  /* largest accepted+rejected count of one trajectory */
    long long n_failed;            /* trajectories with a non-OK status */
    long long fp64_steps;          /* NH_FP32C: attempted steps run in FP64 */
    long long free_exits;          /* trajectories finished by the exact free-streaming exit */
    double    kernel_ms;           /* device time of the trajectory kernel(s); serving: the
                                      slices the request took part in */
    double    latency_ms;          /* serving: nh_submit -> result ready on the host; else 0 */
} nh_stats;

typedef struct nh_context nh_context;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  The context owns device tables,
 * work buffers and the serving queue; it allocates lazily and grows as
 * requests need.  One host thread at a time may use nh_solve / nh_solve_async
 * on a context. */
int nh_context_create(int device, nh_context **out);

/* Wait for outstanding work, free everything the context owns.  NULL is a no-op. */
int nh_context_destroy(nh_context *ctx);

/* Device memory (bytes) a request needs in the context beyond what every
 * request shares: tables, grids, per-trajectory results.  Validates the
 * request (NH_EINVAL).  Needs no GPU. */
int nh_footprint_bytes(const nh_request *req, size_t *bytes);

/* Context options (tuning; defaults in brackets).  Apply to later solves. */
enum {
    NH_OPT_QUEUE_ORDER   = 1,  /* persistent-kernel work order: [0] index order (a wave's
                                  lanes share radius and momentum, so their u and table
                                  reads stay close), 1 lowest momenta first, 2 momentum
                                  index fastest (lanes share radius and direction), 3 index
                                  order in 64-trajectory blocks with the blocks of each round
                                  of claims spread over the workgroups (the costly small
                                  radii then start on every CU rather than on a few) */
    NH_OPT_FREE_EXIT     = 2,  /* [1] stop a trajectory once it is beyond the compensation
                                  radius and receding (exact: the force is zero from then on);
                                  0 integrates every trajectory to z_end */
    NH_OPT_FP64_BELOW_H  = 3,  /* NH_FP32C: attempted steps with |h| below this run in FP64 [1e-6].
                                  A wavefront runs an FP64 attempt whenever one of its lanes
                                  needs one; at 1e-5 that was a quarter of all passes on the
                                  plain-at-scale halos (7 % of the time), for the same profiles */
    NH_OPT_TABLE_NODES   = 4,  /* Dormand-Prince coefficient table nodes, 64..3073, or 0 for the
                                  default [0]: 3073, or for the batched and serving forms as many
                                  as their LDS slots hold (a larger value is NH_EINVAL there) */
    NH_OPT_BLOCK_THREADS = 5,  /* Dormand-Prince threads per workgroup, a multiple of 64 in
                                  [64, 1024] (FP32C batches with two table slots use at most
                                  768), or 0 for the defaults [0]: what
                                  nh_autotune chose for that form and precision, else 768 for
                                  FP64 nh_solve (three waves per SIMD; more lanes per profile
                                  lengthen its tail), 512 for FP32C nh_solve, 1024 for batches
                                  and serving (four waves per SIMD; 768 for FP32C with two
                                  slots).  Plain solves run side by side under
                                  NH_OPT_WORKGROUPS do best at 1024. */
    NH_OPT_BATCH_SLOTS   = 6,  /* batched and serving forms: request tables per workgroup in
                                  LDS, 1 or 2, or 0 for the default [0]: what nh_autotune chose
                                  for FP32C, else 1 (3073 nodes; a workgroup drains before it
                                  changes request, and every running lane serves one request,
                                  so its parameters are scalars).  With 2 the lanes keep
                                  integrating while the next table loads, but carry their
                                  request's parameters in registers: FP32C batches at 768
                                  threads with two slots ran 21 % slower than at 1024 with
                                  one.  Two FP64 tables hold at most 2044 (constant R) or
                                  1703 nodes. */
    NH_OPT_SLICE_US      = 7,  /* serving: length of a time slice in microseconds, 200..1e6 [4000];
                                  requests are admitted and retired between slices.  While
                                  the admitted, unclaimed work would take more than four
                                  slices, a slice is stretched to a quarter of it, at most 8x */
    NH_OPT_SERVE_GRAPH   = 8,  /* serving: [1] run each slice (descriptor uploads, the slice
                                  kernel, the read-back of its queue state) as a replay of a
                                  HIP graph built once per session and table layout, with only
                                  the kernel's arguments updated; 0 issues them one by one.
                                  Taken when a serving session starts. */
    NH_OPT_TRAJECTORY_STATS = 11, /* [0] nh_solve and nh_solve_async without a ratio buffer add
                                  each trajectory's quadrature term and statistics as it
                                  finishes and store nothing per trajectory; 1 stores the
                                  speed ratios and per-trajectory statistics first (for
                                  nh_last_trajectory_stats).  Profiles are the same bits. */
    NH_OPT_FP32C_RTOL    = 10, /* NH_FP32C: tolerance floor of the FP32 attempts, in [1e-9, 1e-3]
                                  [1e-7]: they integrate at max(rtol, this).  At 1e-6 the
                                  discretisation error alone reaches 1e-4 of n/nbar for some
                                  halos; at 1e-7 the form stays within ~2e-5 of the FP64
                                  reference integration */
    NH_OPT_WORKGROUPS    = 9   /* nh_solve, nh_solve_async, nh_solve_masses, nh_solve_integrand
                                  with Dormand-Prince: at most this many workgroups per launch,
                                  1..65536, or 0 for the default [0]: as many as the device holds
                                  at once (one per CU).  Solves from several contexts on
                                  separate streams, each capped to its share of the CUs, run
                                  side by side; a profile's tail (its few longest
                                  trajectories) then idles only its own share.  Results do not
                                  depend on it. */
};
int nh_set_option(nh_context *ctx, int option, double value);

/* ---- plain solve ------------------------------------------------------ */

/* Compute n/nbar for one request and wait for it: the backward integration of
 * every trajectory (Sec. II.C) and the quadrature of Eq. (localdensity) over
 * the background density that follows it.
 * n_over_nbar: host, req->grid.n_r doubles, written in radius order.
 * stats: may be NULL.
 * Returns NH_OK, NH_ESTEPS / NH_ENONFINITE (profile written, failures counted
 * in stats), or an error with nothing written. */
int nh_solve(nh_context *ctx, const nh_request *req, double *n_over_nbar, nh_stats *stats);

/* Enqueue one request on `stream` without waiting: the backward integration of
 * every trajectory (Sec. II.C) and the quadrature of Eq. (localdensity) over
 * the background density that follows it.
 * d_out:   device, req->grid.n_r doubles, receives n/nbar.
 * d_ratio: device, n_traj doubles, or NULL; receives P_i/P0 = |v(z_end)|/|v0|
 *          of every trajectory in index order t = (k*n_y + j)*n_mu + l.
 * Without d_ratio (and NH_OPT_TRAJECTORY_STATS 0) the quadrature runs in the
 * trajectory kernels as trajectories finish and nothing is stored per
 * trajectory.  The sums are exact (fixed point), so the profile is the same
 * bits either way.
 * The context's work buffers are reused by the next call on the same context,
 * which first waits for this one.  nh_last_stats() waits and reports it. */
int nh_solve_async(nh_context *ctx, const nh_request *req, double *d_out, double *d_ratio,
                   void *stream);

/* The profile plus the relic distribution behind it (Sec. II.D, Fig. 3: the
 * phase-space distribution at each radius, whose peaks are the phase-space
 * shells of infall; the paper inspects it to choose the momentum grid).
 * d_integrand: device, n_r * n_y doubles, radius-major:
 *   d_integrand[k n_y + j] = sum_l w_mu,l f0(y_j P_i/P0 (k, j, l)),
 * the distribution at radius k and momentum node y_j integrated over the
 * direction (l in index order); far from the halo it is f0(y_j) sum_l w_mu,l.
 * n/nbar_k = sum_j w_y,j d_integrand[k n_y + j] / sum_j w_y,j f0(y_j) sum_l w_mu,l.
 * d_out, d_ratio, stream and statistics as for nh_solve_async. */
int nh_solve_integrand(nh_context *ctx, const nh_request *req, double *d_out, double *d_integrand,
                       double *d_ratio, void *stream);

/* Several relic masses from one integration (Sec. II.D: the equations of
 * motion do not involve the mass).  The request fixes the velocities: its y
 * grid at its m_eV.  For mass m_k the same trajectories carry momenta
 * y_j m_k / m_eV, and the profile is the quadrature over that grid (its
 * weights computed from the scaled grid as for any request), so mass k's
 * profile is the profile of the request with m = m_k and y scaled by
 * m_k / m_eV.  Enqueued like nh_solve_async (statistics: nh_last_stats).
 * m_eV: host, n_mass > 0 finite masses, 1 <= n_mass <= 4096.
 * d_out: device, n_mass * n_r doubles, mass-major (mass k at d_out + k n_r).
 * d_ratio: as for nh_solve_async, or NULL. */
int nh_solve_masses(nh_context *ctx, const nh_request *req, int n_mass, const double *m_eV,
                    double *d_out, double *d_ratio, void *stream);

/* Wait for the last nh_solve_async on this context and return its statistics
 * and status (NH_OK, NH_ESTEPS or NH_ENONFINITE). */
int nh_last_stats(nh_context *ctx, nh_stats *stats);

/* Per-trajectory diagnostics of the last completed solve on this context
 * (waits for it), which must have stored per-trajectory results (a ratio
 * buffer, nh_solve_masses, nh_solve_integrand, nh_solve_batch, or
 * NH_OPT_TRAJECTORY_STATS 1); NH_EINVAL otherwise.  Host arrays of `capacity`
 * entries, at least the last solve's n_traj (NH_EINVAL if fewer), each may be
 * NULL; entries in trajectory order (a batch: its requests concatenated):
 * accepted and rejected step counts, and the status word (low byte 0 ok, 1
 * max_steps, 2 step underflow, 3 non-finite; bit 8 set when the trajectory
 * left through the exact free-streaming exit). */
int nh_last_trajectory_stats(nh_context *ctx, size_t capacity, int *accepted, int *rejected, int *status);

/* ---- plain solve without memory allocation ---------------------------- */

/* For callers that cannot allocate memory (tight serving loops, harnesses that
 * forbid allocation): the plain solve of nh_solve_async, allocating nothing.
 * Its device buffers (counters, the quadrature sums, the staged tables and
 * grids of one request) live in a static device array of nh_noalloc_scratch_bytes() bytes (4 MiB) that each GPU
 * the library runs on holds until the process ends; its host staging is a
 * static array too.  The profile is the same bits as nh_solve_async's.
 * d_out: device, req->grid.n_r doubles.  Statistics: nh_last_stats.  The
 * context must exist already (nh_context_create allocates).  The inputs go
 * up by an asynchronous copy from a static pageable host array, so the call
 * is not for use under stream capture.
 * NH_EINVAL: a request whose staged inputs and sums exceed the scratch, or
 * with sampled histories (their spline set-up allocates on the host).
 * Every call on a GPU shares that GPU's scratch, which keeps the last call's
 * contents: calls that overlap on one GPU race, so a caller runs one at a time
 * per GPU (the next call on the same context waits for the previous one). */
int nh_solve_noalloc(nh_context *ctx, const nh_request *req, double *d_out, void *stream);
size_t nh_noalloc_scratch_bytes(void);

/* ---- batched solve ---------------------------------------------------- */

/* Solve n_req heterogeneous requests in one persistent launch (each request:
 * Sec. II.C integration and the quadrature of Eq. localdensity; several
 * halos, relic masses and grids at once serve the paper's rapid scans of
 * parameters, abstract and Sec. V).
 * d_out: device, sum of the requests' n_r doubles, profiles concatenated in
 * request order.  All requests must share method and precision.
 * stats: host array of n_req entries, or NULL.  Waits for completion. */
int nh_solve_batch(nh_context *ctx, int n_req, const nh_request *reqs, double *d_out,
                   nh_stats *stats, void *stream);

/* ---- serving (continuous batching) ------------------------------------ */
/* A worker thread of the context runs the slice kernel in time slices over
 * the admitted requests; in-flight trajectories are saved to device memory at
 * the end of a slice and resumed bit for bit by the next one, and requests are
 * admitted and retired between slices.  A request's profile does not depend
 * on what else is being served.  Requests must use NH_DOPRI5; one precision at
 * a time (that of the first request admitted while the server is empty).
 * Tables and slots per workgroup follow NH_OPT_TABLE_NODES / NH_OPT_BATCH_SLOTS;
 * the slice length is NH_OPT_SLICE_US.  All serving calls are thread-safe. */

/* Device-memory budget (bytes) for admitted requests (their tables, grids,
 * per-trajectory results and profile); 0 = the smaller of 80 % of the free
 * device memory and 32 GiB, taken at the first submit.  The budget is
 * allocated once, when the first request is admitted.  NH_EBUSY while
 * requests are admitted.  Needs no GPU. */
int nh_serve_set_budget(nh_context *ctx, size_t bytes);

/* Admit a request (integration, Sec. II.C, and quadrature, Eq. localdensity,
 * served between other requests for the rapid scans of the abstract and
 * Sec. V), or NH_EBUSY if its footprint (nh_footprint_bytes) does not
 * fit the free budget right now (nothing is queued then).  NH_EINVAL for an
 * invalid request, a method other than NH_DOPRI5 or another precision than
 * the one being served.  Host inputs are copied before the call returns.
 * ticket: receives an id for nh_poll / nh_cancel. */
int nh_submit(nh_context *ctx, const nh_request *req, uint64_t *ticket);

/* Collect a finished ticket: its n/nbar profile (Eq. localdensity).
 * out: host, n_r doubles.  stats: may be NULL.
 * NH_ENOTREADY while the ticket runs; NH_OK (or NH_ESTEPS / NH_ENONFINITE with
 * the profile written) once, after which the ticket is gone. */
int nh_poll(nh_context *ctx, uint64_t ticket, double *out, nh_stats *stats);

/* Cancel a ticket: its remaining trajectories are dropped and its memory
 * returns to the budget (once the next slice boundary has passed).  Polling it
 * afterwards returns NH_ECANCELED once.  NH_ENOTFOUND for an unknown ticket. */
int nh_cancel(nh_context *ctx, uint64_t ticket);

/* ---- autotuning -------------------------------------------------------- */

/* Forms that nh_autotune tunes. */
#define NH_FORM_PLAIN 0   /* nh_solve / nh_solve_async / nh_solve_masses (Dormand-Prince) */
#define NH_FORM_BATCH 1   /* nh_solve_batch and the serving loop */

typedef struct {
    int    form;            /* NH_FORM_* */
    int    precision;       /* NH_FP64 or NH_FP32C */
    int    block_threads;   /* chosen threads per workgroup */
    int    batch_slots;     /* chosen tables per workgroup (batched form), else 0 */
    int    n_tried;         /* candidate configurations timed */
    double best_ms;         /* trajectory-kernel time of the sample with the choice */
    double default_ms;      /* the same with the built-in default */
} nh_tune_result;

/* Choose the launch configuration of one form and precision by timing it.
 * Every candidate (workgroup sizes of one to four waves per SIMD; for FP32C
 * batches also one or two tables per workgroup) solves the caller's sample
 * after one untimed warm-up; the candidate with the least total trajectory-
 * kernel time (best of two passes) becomes the context's default for that
 * form and precision, used wherever NH_OPT_BLOCK_THREADS / NH_OPT_BATCH_SLOTS
 * are 0.  Results never depend on the choice (every trajectory is integrated by
 * the same arithmetic whichever lane runs it); only the time does.  The sample
 * should resemble the later work but need not be part of it.
 * reqs: host, n_req requests of one precision, all NH_DOPRI5; 1 <= n_req <= 65535
 * (NH_FORM_PLAIN solves each one in turn, NH_FORM_BATCH them as one batch).
 * result: may be NULL.  Waits for completion; the serving loop must be idle
 * (NH_EBUSY otherwise).  Allocates device memory for the outputs while it runs. */
int nh_autotune(nh_context *ctx, int form, int n_req, const nh_request *reqs, nh_tune_result *result);

/* ---- host-side helpers (need no GPU) --------------------------------------- */

/* The n-point Gauss-Legendre rule on [-1, 1] that a grid with mu == NULL uses
 * (Eq. density_integral integrates mu = cos psi over [-1, 1]).
 * x, w: host, n doubles each; nodes ascending.  1 <= n <= 4096. */
int nh_gauss_legendre(int n, double *x, double *w);

/* The u-dependent coefficients of the equations of motion as the library
 * tabulates them on the host in FP64, at n points u (u = ln a, in
 * [-ln(1+z_end), -ln(1+z_obs)]).  out: host, 6*n doubles, row i = (A, K, Kc, 1/s, c, R):
 *   dx/du = A v,   dv/du = -[K I(min(r/s, c)) / r^3 - Kc] x  for r < R, else 0,
 * A = (1+z)^2/H, K = kappa G (1+z) M / (H I(c)), Kc = kappa G (1+z) M / (H R^3),
 * s the comoving NFW scale radius, R the compensation radius (1e300 when
 * uncompensated).  Sec. II.A Eq. (eoms), Sec. II.B, App. A.  Validates req. */
int nh_coefficients(const nh_request *req, int n, const double *u, double *out);

/* ---- diagnostics ------------------------------------------------------- */

const char *nh_strerror(int code);
const char *nh_last_error(const nh_context *ctx);

/* Library version string. */
const char *nh_version(void);

/* Measured FP64 vector FMA throughput of the context's device (TFLOP/s, FMA =
 * 2 FLOP): a kernel of independent v_fma_f64 chains in every lane of every CU,
 * best of three launches.  The datasheet peak of an MI355X is 78.6 TFLOP/s;
 * this is the ceiling the trajectory kernels are measured against as well. */
int nh_fp64_fma_peak(nh_context *ctx, double *tflops);

/* The device's own values of two elementary functions of the right-hand side,
 * computed by the same inline code the trajectory kernels run, for tests of
 * their accuracy against references of higher precision:
 *   NH_FN_NFW_I       y = I(x) = ln(1+x) - x/(1+x), the NFW mass integral
 *                     (Eq. nfw, App. A), x >= 0; req is ignored (may be NULL);
 *   NH_FN_POW_FACTOR  y = the factor of K and Kc at u = x that req's tables
 *                     leave out: xi^alpha of the paper's growth model times
 *                     kappa = 1 + a [z/(1+z)]^b (Sec. IV.A, IV.B); 1 where req
 *                     has neither.  Validates req.
 * x, y: host, n doubles each (0 <= n <= 2^26).  Synchronous on the context's
 * stream.  NH_EINVAL for an unknown fn, bad sizes or pointers. */
enum { NH_FN_NFW_I = 1, NH_FN_POW_FACTOR = 2 };
int nh_device_function(nh_context *ctx, int fn, const nh_request *req, long long n, const double *x, double *y);

#ifdef __cplusplus
}
#endif

#endif /* NUHALO_H */
