/*
 * liblbm: MI355X (gfx950) D2Q9 multiple-relaxation-time lattice Boltzmann step with the local
 * curved slip boundary of Wang, Tao, Hu, Zhang and Lu, "Curved boundary conditions of the
 * lattice Boltzmann method for simulating microgaseous flows in the slip regime"
 * (arXiv:2012.14707).
 *
 * Plain C ABI: every call returns an lbm_status; nothing throws across it.  The message of the
 * last failure on the calling thread is available from lbm_last_error().
 *
 * Lattice units throughout: delta_x = delta_t = 1, c = 1, c_s^2 = 1/3.  Directions follow
 * Eq. (Eq3): 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.  Sites are row-major,
 * site = y * nx + x.
 *
 * Memory: a context owns every device buffer it allocates.  Inputs passed to lbm_create are
 * copied, so the caller may free them when it returns.  Outputs go to caller-owned buffers,
 * either host memory or device memory (flag device_ptrs), sized as documented per call.
 * A context is bound to the HIP device that was current at lbm_create and to one HIP stream;
 * all device work is queued on that stream.  A context is not thread-safe; distinct contexts
 * are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_E_INVAL (-1)    /* bad argument (null pointer, size, enum value) */
#define LBM_E_NOMEM (-2)    /* device or host allocation failed */
#define LBM_E_HIP (-3)      /* a HIP runtime call failed */
#define LBM_E_GEOMETRY (-4) /* mask / wall-link table inconsistent */
#define LBM_E_PARAM (-5)    /* physical parameters out of range (tau <= 1/2, 1 + l <= 0, r outside [0, 1]) */
#define LBM_E_UNSTABLE (-6) /* the state went non-finite */
#define LBM_E_STATE (-7)    /* call not valid in the context's current state */

/* Free parameter l of Eq. (EqNewBDSC). */
enum {
    LBM_L_PAPER = 0,             /* Eq. (Eqexlva); l := 0 where it gives l < -0.4 (end of Sec. III.B) */
    LBM_L_CLAMP_NEG = 1,         /* Eq. (Eqexlva); l := 0 where it gives l < 0 (stability fallback) */
    LBM_L_ZERO = 2,              /* l = 0 (the "previous scheme" of Sec. III.B) */
    LBM_L_GAMMA = 3,             /* l = gamma (Sec. IV comparisons) */
    LBM_L_TWO_GAMMA = 4,         /* l = 2 gamma */
    LBM_L_GAMMA2 = 5,            /* l = gamma^2 */
    LBM_L_GAMMA2_PLUS_GAMMA = 6, /* l = gamma^2 + gamma */
    LBM_L_FIXED = 7,             /* l = l_override on every link */
    LBM_L_WALL_FIT = 8           /* wall reading (LBM_DIFFUSE_WALL): l such that the Kn^2 term of the
                                    scheme's Poiseuille slip equals 8 L2 Kn^2 of Eq. (PhyscPoiSlip) with
                                    the uniform tau_q; requires LBM_R_WALL_FIT.  The near-wall relation
                                    of Eq. (NumerSana) under that reading keeps B of Eq. (CoeC) and has
                                    A = [(1+l)(1-r)(tau_s+1) + 2r(1+gamma)] / Den; along the curve of
                                    LBM_R_WALL_FIT, B is affine in 1 + l, which gives l in closed form */
};
/* Combination parameter r of Eq. (EqNewBDSC). */
enum {
    LBM_R_FROM_LEFF = 0, /* Eq. (SliCoeffrtsr) at the l actually used; equals Eq. (NSliCoertsr) where l is not clamped */
    LBM_R_PAPER = 1,     /* Eq. (NSliCoertsr) as printed, also on clamped links */
    LBM_R_FIXED = 2,     /* r = r_override on every link */
    LBM_R_WALL_FIT = 3   /* wall reading: r such that the Kn term of the slip equals 4 L1 Kn, i.e.
                            r / (1 - r) = (1 + l)(tau_s - gamma - L1 lambda) / (2 L1 lambda) with
                            lambda = Kn H of Eq. (tKnrela).  Exists only for gamma < tau_s - L1 lambda
                            and L1 > 0: lbm_create fails with LBM_E_PARAM on any other link */
};
/* Velocity of the Maxwell-diffuse equilibrium f_i^eq(rho_f, .) in Eq. (EqNewBDSC). */
enum {
    LBM_DIFFUSE_NODE = 0, /* u(x_f, t), the boundary node's half-force velocity: the reading under
                             which the analysis of Sec. III.B (Eqs. (NumerSana)-(CoeC)) holds */
    LBM_DIFFUSE_WALL = 1  /* u_b, the wall velocity (literal text of Sec. III.A) */
};
/* Population storage. */
enum {
    LBM_FP64 = 0,         /* fp64 deviations g_i = f_i - w_i rho0, fp64 collision */
    LBM_FP32_SHIFTED = 1  /* fp32 deviations, fp32 collision; fp64 precompute and reductions */
};

/* One wall link: the fluid node x_f = (x, y), dir = the D2Q9 direction from x_f toward the solid
 * node x_r (the paper's ibar, Fig. 1), q = gamma = |x_b - x_f| / |x_r - x_f| in (0, 1], and the
 * wall velocity (ubx, uby) at the crossing point x_b. */
typedef struct {
    int32_t x, y, dir, reserved;
    double q, ubx, uby;
} lbm_link;

/* Problem statement.  NaN in L1, L2 or E and values <= 0 in the *_override fields select the
 * paper's prescription. */
typedef struct {
    int32_t nx, ny;                 /* lattice size (sites) */
    int32_t periodic_x, periodic_y; /* 1 = periodic; otherwise the mask must pad that edge with solid */
    double kn, h;                   /* Knudsen number and characteristic length H (lattice units):
                                       tau_s = 1/2 + sqrt(6/pi) Kn H, Eq. (tKnrela) */
    double sigma, L1, L2;           /* slip coefficients of Eq. (PhyscSlip); NaN L1/L2 -> Sec. IV model
                                       L1 = (2 - sigma)(1 - 0.1817 sigma)/sigma, L2 = 1/pi + L1^2/2 */
    double E;                       /* constant of Eq. (Eqexlva); NaN -> min(-0.65, E_max - 0.05) with
                                       E_max the bound of Eq. (EqECond) */
    double tau_rho, tau_e, tau_eps, tau_j; /* non-hydrodynamic relaxation times (Sec. IV: 1.0, 1.1, 1.2, 1.0) */
    double tau_s_override, tau_q_override; /* > 0: use instead of Eqs. (tKnrela) / (NSliCoertstq) */
    double r_override, l_override;         /* used by LBM_R_FIXED / LBM_L_FIXED */
    int32_t l_mode, r_mode, diffuse, precision;
    double ax, ay;                  /* body acceleration a; the force density is rho a (Sec. III.B) */
    double rho0;                    /* reference density of the rest state (1) */
} lbm_params;

typedef struct {
    double tau_s, tau_q, E, E_max, L1, L2, nu; /* derived parameters; nu = (tau_s - 1/2)/3, Eq. (EqViscos) */
    int64_t n_sites, n_fluid, n_links;
    int32_t n_clamped;    /* links where the l mode reset l */
    int32_t n_nonconvex;  /* links with l outside [max(0, 2 gamma - 1), 2 gamma] (Sec. III.A) */
    int32_t precision;
    int32_t steps_per_launch; /* time steps per launch of the step kernel (see lbm_set_fusion) */
    int64_t bytes_per_step; /* algorithmic HBM bytes of one step: 18 s per fluid node (nine populations
                               in, nine out) + (5 + 5 s) per wall link (a 4-byte index, a direction
                               byte, five coefficients) + 1 mask byte per site (s = 8 or 4) */
    int64_t steps;          /* steps taken since the last initialisation */
} lbm_info;

typedef struct lbm_ctx lbm_ctx;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t lbm_version(void);

/* Message of the last failing call on this thread ("" if none).  Owned by the library. */
const char *lbm_last_error(void);

/* Fills *p with the paper's defaults: sigma = 1, L1/L2/E = NaN (derived), tau_rho = tau_j = 1,
 * tau_e = 1.1, tau_eps = 1.2 (Sec. IV), no overrides, LBM_L_PAPER, LBM_R_FROM_LEFF,
 * LBM_DIFFUSE_NODE, LBM_FP64, a = 0, rho0 = 1, non-periodic. */
lbm_status lbm_params_default(lbm_params *p);

/* Boundary schemes the paper compares against (Sec. III.B, Sec. IV), as parameter sets of the same
 * boundary rule Eq. (EqNewBDSC). */
enum {
    LBM_SCHEME_PRESENT = 0,     /* l of Eq. (Eqexlva), r of Eq. (NSliCoertsr), uniform tau_q of
                                   Eq. (NSliCoertstq): the paper's prescription (the defaults) */
    LBM_SCHEME_PREVIOUS = 1,    /* l = 0 ("previous" curved scheme): r of Eq. (SliCoeffrtsrD) and tau_q of
                                   Eq. (SliCoeffrtstqrD) evaluated at one frozen gamma */
    LBM_SCHEME_HALFWAY_DBB = 2, /* halfway diffuse bounce-back: l = 0, r of Eq. (SliCoeffHar), tau_q of
                                   Eq. (SliCoeffHata); the caller also gives q = 1/2 on every link */
    LBM_SCHEME_WALL_READING = 3 /* the present scheme re-derived for the literal reading of the diffuse
                                   part: LBM_DIFFUSE_WALL, LBM_L_WALL_FIT, LBM_R_WALL_FIT and the uniform
                                   tau_q of Eq. (NSliCoertstq) */
};

/* Sets the mode fields and the tau_q override of *p for one of the compared schemes: reads kn, h,
 * sigma, L1, L2 and tau_s_override of *p (derived as in lbm_create when unset) and writes l_mode,
 * r_mode and tau_q_override (LBM_SCHEME_WALL_READING also sets diffuse).  gamma_frozen: the gamma in (0, 1] at which LBM_SCHEME_PREVIOUS
 * evaluates Eq. (SliCoeffrtstqrD) (ignored otherwise).  LBM_E_PARAM if the resulting tau_q is not
 * above 1/2; no device work. */
lbm_status lbm_params_comparison(lbm_params *p, int32_t scheme, double gamma_frozen);

/* Creates a lattice (Sec. III.A problem statement).
 *   solid    host, uint8 [ny * nx] row-major, nonzero = solid (closed set: nodes on a wall are solid)
 *   links    host, n_links records; every (fluid node, direction) whose neighbour is solid must
 *            appear exactly once; order is free
 *   stream   hipStream_t for all device work of this context (NULL = the null stream)
 * Limits (LBM_E_INVAL): nx, ny >= 1, nx * ny < 2^31 sites and n_links <= 2^31 - 1, so that site
 * indices and link offsets fit the kernels' 32-bit indices.
 * Validation (LBM_E_GEOMETRY): x_f fluid and x_f + c_dir solid, 0 < q <= 1, finite wall velocity,
 * no duplicate, no missing link, no fluid node on a non-periodic edge, no fluid node whose eight
 * neighbours are all solid.  LBM_E_PARAM: tau_s or tau_q <= 1/2, any tau <= 1/2, 1 + l <= 0 or
 * r outside [0, 1] on some link.  On success *out owns the device state, initialised to rest
 * (f_i = w_i rho0).  On failure *out is NULL and nothing is leaked. */
lbm_status lbm_create(const lbm_params *p, const uint8_t *solid, const lbm_link *links, int64_t n_links,
                      void *stream, lbm_ctx **out);

/* Releases every device and host resource of ctx (NULL is accepted). Synchronises the stream. */
lbm_status lbm_destroy(lbm_ctx *ctx);

lbm_status lbm_get_info(const lbm_ctx *ctx, lbm_info *info);

/* Per-link boundary coefficients as computed on the device in fp64, in the caller's link order:
 * out (host) [n_links * 8] = (l_raw, l_eff, r, alpha1, alpha2, alpha3, beta, kappa) per link, where
 * Eq. (EqNewBDSC) reads f_i(x_f, t+1) = alpha1 f_ibar(x_f,t) + alpha2 f'_i(x_f,t) + alpha3 f'_ibar(x_f,t)
 * + beta rho_f + kappa f_i^eq(rho_f, u_d):  alpha1 = r(1+l-2 gamma)/(1+l), alpha2 = r l/(1+l),
 * alpha3 = r(2 gamma - l)/(1+l), beta = 2 r/(1+l) w_i c_i.u_b / c_s^2 (+ kappa w_i phi_i(u_b) under
 * LBM_DIFFUSE_WALL, where the wall equilibrium is folded into beta), kappa = 1 - r. */
lbm_status lbm_link_coeffs(lbm_ctx *ctx, double *out);

/* Rest state f_i = w_i rho0 everywhere. */
lbm_status lbm_init_rest(lbm_ctx *ctx);

/* State f_i = f_i^eq(rho, u - a/2) at fluid nodes, so that the half-force velocity of
 * Eq. (FluidMacr) equals u.  rho, ux, uy: fp64 [ny * nx], host (device_ptrs = 0) or device
 * (device_ptrs = 1); values on solid sites are ignored.  Non-finite input is accepted and is
 * reported by the next lbm_residual as LBM_E_UNSTABLE. */
lbm_status lbm_init_fields(lbm_ctx *ctx, const double *rho, const double *ux, const double *uy, int32_t device_ptrs);

/* lbm_init_fields plus a non-equilibrium part: at fluid nodes f_i = f_i^eq(rho, u - a/2) + f_i^neq with
 * f^neq = M^-1 (0, 0, 0, 0, 0, 0, 0, p_xx, p_xy) (M of Sec. II), the first-order Chapman-Enskog
 * stress of the given velocity field under the shear relaxation time tau_s of Eq. (tKnrela):
 *   p_xx = -(2/3) tau_s rho (d_x u_x - d_y u_y),   p_xy = -(1/3) tau_s rho (d_x u_y + d_y u_x).
 * Derivatives are differences over the fluid neighbours (central; one-sided next to a solid site;
 * 0 with no fluid neighbour along that axis).  A steady flow has this stress, so starting from a
 * good estimate of (rho, u) the lattice begins closer to its steady state than from f^eq alone.
 * Arguments, layout and ownership as lbm_init_fields. */
lbm_status lbm_init_fields_neq(lbm_ctx *ctx, const double *rho, const double *ux, const double *uy, int32_t device_ptrs);

/* Advances nsteps >= 0 time steps: per fluid node, collision in moment space (Eqs. (LBEColli),
 * (LBEforce), (MomentPost)) fused with streaming, and for each wall link the boundary value of
 * Eq. (EqNewBDSC).  Asynchronous on the context's stream. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* rho and the half-force velocity u (Eq. (FluidMacr)) at every site, 0 on solid sites.
 * rho, ux, uy: fp64 [ny * nx], host or device.  Synchronises the stream for host outputs. */
lbm_status lbm_moments(lbm_ctx *ctx, double *rho, double *ux, double *uy, int32_t device_ptrs);

/* Convergence residual and mass, fp64 reductions over fluid nodes in a fixed order:
 *   residual = sqrt(sum |u(t) - u(t-1)|^2 / sum |u(t)|^2), +inf if no step since initialisation,
 *   mass = sum rho.
 * Synchronises the stream.  Returns LBM_E_UNSTABLE (with the values still written) when either
 * is not finite. */
lbm_status lbm_residual(lbm_ctx *ctx, double *residual, double *mass);

/* Re-binds the context to another stream of the same device (NULL = null stream). */
lbm_status lbm_set_stream(lbm_ctx *ctx, void *stream);

/* Waits for all work queued by this context. */
lbm_status lbm_synchronize(lbm_ctx *ctx);

/* Threads per block of the step kernel: 64, 128, 256 (default), 512 or 1024.  Results do not
 * depend on it.  LBM_E_INVAL if the block's wall links would not fit the LDS staging area. */
lbm_status lbm_set_launch(lbm_ctx *ctx, int32_t block);

/* Time steps per kernel launch.  1: one launch of the fused collide-stream-boundary kernel per
 * step.  2: one launch advances two steps on 64 x rows tiles, keeping the intermediate time level
 * in LDS (temporal blocking); this halves the HBM traffic per step, and lbm_step then runs pairs
 * of steps and a single step for an odd remainder.  Results are bit-identical either way.  The
 * default is 2 where the lattice tiles, else 1.  rows: tile rows (4 or 8; 0 = the default: 4 for
 * fp32 storage and 8 for fp64, or the other where only that one fits).  LBM_E_INVAL if 2 is asked
 * and nx is not a multiple of 64, ny not a multiple of rows, or a tile's wall links do not fit the
 * LDS staging area. */
lbm_status lbm_set_fusion(lbm_ctx *ctx, int32_t steps_per_launch, int32_t rows);

/* Step launches by graph replay (on = 1, the default) or one by one (0).  With graphs, lbm_step
 * captures its launch sequence (at most 256 steps per graph, the last one recording u) once per
 * (step count, time-level parity) on a private stream of the context and replays it on the
 * context's stream, which removes the per-launch host cost that dominates small lattices.  Results
 * are bit-identical either way.  If capture is not possible the context falls back to launches
 * for good.  Changing the launch configuration or the fusion drops the captured graphs. */
lbm_status lbm_set_graphs(lbm_ctx *ctx, int32_t on);

/* Device-to-device streaming copy of `bytes` bytes (dst, src: device memory, 16-byte aligned, bytes
 * a multiple of 16, else LBM_E_INVAL), asynchronous on `stream` (hipStream_t, NULL = null stream).
 * A measurement aid, not a step of the method: its bandwidth is the practical streaming ceiling
 * that the step kernels' HBM traffic is compared with. */
lbm_status lbm_stream_copy(void *dst, const void *src, int64_t bytes, void *stream);

/* Average duration in milliseconds of the step kernel launches of the last lbm_step call,
 * measured with HIP events on the context's stream (0 if timing is off).  Timing is switched on
 * by lbm_set_timing(ctx, 1); it records one event pair per lbm_step call. */
lbm_status lbm_set_timing(lbm_ctx *ctx, int32_t on);
lbm_status lbm_last_step_ms(lbm_ctx *ctx, double *ms_total, int64_t *nsteps);

/* ------------------------------------------------------------------------------------------
 * Batches: many independent lattices of uneven sizes and parameters (e.g. a Kn / gamma /
 * geometry sweep) advanced together by one persistent kernel launch per step, captured in HIP
 * graphs.  All instances share the precision and the diffuse reading; everything else (size,
 * mask, links, Kn, H, modes, relaxation times, force) is per instance.  Each instance computes
 * exactly what a single lbm_ctx with the same inputs computes, bit for bit.
 * ------------------------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

/* Per-instance state reported by lbm_batch_solve. */
enum {
    LBM_RUNNING = 0,
    LBM_CONVERGED = 1, /* residual <= tol */
    LBM_FLOOR = 2,     /* residual stopped decreasing (rounding floor of the storage precision) */
    LBM_CAPPED = 3,    /* reached max_steps */
    LBM_DIVERGED = 4   /* residual or mass not finite */
};

/* Launch shape of the batched step. */
typedef struct {
    int32_t block;         /* threads per block = sites per tile: 128, 256, 512 or 1024 */
    int32_t graph_steps;   /* steps captured per HIP graph (even, >= 2) */
    int32_t blocks_per_cu; /* persistent grid of (compute units x blocks_per_cu) blocks; 0 = one block per tile */
    int32_t reserved;
} lbm_batch_launch;

/* Creates a batch of n_inst lattices.  params[i], solids[i], links[i] (n_links[i] records) are
 * instance i's arguments of lbm_create, with the same validation; all params[i].precision and
 * params[i].diffuse must be equal (else LBM_E_INVAL).  The batch's site space (each instance's sites
 * padded to a whole number of tiles) must stay below 2^31 sites and its wall links at most
 * 2^31 - 1 in total (else LBM_E_INVAL).  Inputs are copied.  All instances start at
 * rest and active.  stream: hipStream_t for all work (NULL: the batch creates its own stream;
 * graphs cannot be captured on the null stream). */
lbm_status lbm_batch_create(int32_t n_inst, const lbm_params *params, const uint8_t *const *solids,
                            const lbm_link *const *links, const int64_t *n_links, void *stream, lbm_batch **out);
lbm_status lbm_batch_destroy(lbm_batch *b);

/* Instance i's lbm_info (steps = steps taken by that instance). */
lbm_status lbm_batch_info(const lbm_batch *b, int32_t inst, lbm_info *info);

/* Rest state for every instance; all become active. */
lbm_status lbm_batch_init_rest(lbm_batch *b);

/* Advances every active instance by nsteps (graph replays plus eager launches for a remainder). */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Marks instances active (nonzero) or retired (0); retired instances keep their state and are
 * skipped by lbm_batch_step.  active: host [n_inst]. */
lbm_status lbm_batch_set_active(lbm_batch *b, const uint8_t *active);

/* Residual and mass (definitions of lbm_residual) of every active instance into residual[i],
 * mass[i] (host, [n_inst]); retired instances report the values of their last check.
 * Synchronises.  LBM_E_UNSTABLE if any active instance is not finite (values still written). */
lbm_status lbm_batch_residuals(lbm_batch *b, double *residual, double *mass);

/* rho, u of instance inst (layout and ownership of lbm_moments). */
lbm_status lbm_batch_moments(lbm_batch *b, int32_t inst, double *rho, double *ux, double *uy, int32_t device_ptrs);

/* Runs every instance from its current state until it retires: every check_every steps (even)
 * the residuals are computed and an instance stops as LBM_CONVERGED (residual <= tol),
 * LBM_DIVERGED (not finite), LBM_CAPPED (steps >= max_steps) or LBM_FLOOR (residual above
 * 0.995 x its value 50 checks earlier while below 1e-5).  Outputs (host, [n_inst], any may be
 * NULL): status, steps taken by the instance, last residual. */
lbm_status lbm_batch_solve(lbm_batch *b, double tol, int64_t check_every, int64_t max_steps, int32_t *status,
                           int64_t *steps, double *residual);

/* Replaces instance i's problem statement by *p, keeping its geometry (mask and wall links): p must
 * have the instance's nx, ny, periodic_x, periodic_y, precision and diffuse (else LBM_E_INVAL).  The
 * derived parameters and the per-link coefficients of Eq. (EqNewBDSC) are recomputed on the device
 * (validation of lbm_create: LBM_E_PARAM leaves the instance unchanged); the instance is reset to
 * rest (step count 0) and made active.  Synchronises.  Other instances are not touched. */
lbm_status lbm_batch_set_params(lbm_batch *b, int32_t i, const lbm_params *p);

/* lbm_batch_solve followed by the stability fallback for the paper's clamp rule (end of Sec. III.B:
 * l := 0 only where Eq. (Eqexlva) gives l < -0.4, a rule the paper motivates by stability): every
 * instance that ended LBM_DIVERGED under LBM_L_PAPER is switched to LBM_L_CLAMP_NEG (l := 0 wherever
 * l < 0) by lbm_batch_set_params, restarted from rest and solved again alone with the same tol,
 * check_every and max_steps.  Those instances keep LBM_L_CLAMP_NEG afterwards and report the status,
 * step count and residual of the re-run; fell_back[i] (host, [n_inst], may be NULL) is 1 for them and
 * 0 for every other instance, whose results are those of the first solve.  Instances are independent:
 * a diverging instance does not change the bits of any other. */
lbm_status lbm_batch_solve_fallback(lbm_batch *b, double tol, int64_t check_every, int64_t max_steps,
                                    int32_t *status, int64_t *steps, double *residual, uint8_t *fell_back);

lbm_status lbm_batch_set_launch(lbm_batch *b, const lbm_batch_launch *launch);
lbm_status lbm_batch_get_launch(const lbm_batch *b, lbm_batch_launch *launch);

/* Autotuner: times trial_steps steps of every candidate launch shape (block 128/256/512,
 * graph_steps 2/10/50, blocks_per_cu 0/2/4/8) on this batch with HIP events, keeps the fastest
 * and records it in the text file cache_path (NULL: no cache) under a key of (GPU architecture,
 * precision, total sites, instance count); a cached key is reused without timing.  Either way the
 * batch is reset to rest afterwards (lbm_batch_init_rest).  The first failing trial ends the tuning
 * with its status.  Every candidate computes identical results. */
lbm_status lbm_batch_tune(lbm_batch *b, const char *cache_path, int32_t trial_steps, lbm_batch_launch *chosen);

/* ------------------------------------------------------------------------------------------
 * Learned warm start.  A convolutional encoder-decoder predicts an initial (u, rho) from the
 * problem statement (mask, distance ratios, Kn, force direction); the lattice then starts from
 * f^eq(rho, u) (lbm_init_fields) instead of rest.  The network is not part of the paper: it only
 * changes the initial state, and the converged field is the lattice's own.
 *
 * Tensors are NHWC: element (image n, row y, column x, channel c) of a [n, h, w, C] tensor is at
 * ((n * h + y) * w + x) * C + c.  bf16 tensors (IEEE-754 binary32 with the low 16 bits dropped,
 * round to nearest even) must be 16-byte aligned and have a multiple of 8 channels.  Every
 * pointer below is device memory unless it says host.  Calls are asynchronous on `stream`
 * (hipStream_t, NULL = null stream) unless they return a host value.
 * ------------------------------------------------------------------------------------------ */

/* 'Same' convolution, ksize 1 or 3, on the matrix cores with fp32 accumulation:
 *   out[n,y,x,co] = act(bias[co] + sum_{ky,kx,ci} in[n, y+ky-k/2, x+kx-k/2, ci] w[ky*k+kx][co][ci])
 * where in[] outside the image is 0 (periodic = 0) or wraps around (periodic = 1: row y + h and
 * column x + w are row y and column x).  in bf16 [n,h,w,cin]; w bf16 [k*k][cout][cin]; bias fp32
 * [cout] or NULL; act = max(., 0) if relu.  out bf16 [n,h,w,cout] and/or out32 fp32
 * [n,h,w,cout] (either may be NULL). */
lbm_status lbm_conv2d_forward(const void *in, const void *w, const float *bias, void *out, float *out32,
                              int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout, int32_t ksize,
                              int32_t relu, int32_t periodic, void *stream);

/* Input gradient of lbm_conv2d_forward without activation:
 *   din[n,y,x,ci] = sum_{ky,kx,co} dout[n, y-ky+k/2, x-kx+k/2, co] w[ky*k+kx][co][ci]
 * (indices outside the image as in lbm_conv2d_forward with the same periodic flag)
 * dout bf16 [n,h,w,cout] -> din bf16 [n,h,w,cin].  wt: bf16 workspace of k*k*cin*cout elements
 * (overwritten with the flipped, transposed kernel). */
lbm_status lbm_conv2d_dgrad(const void *dout, const void *w, void *din, void *wt, int32_t n, int32_t h, int32_t wd,
                            int32_t cin, int32_t cout, int32_t ksize, int32_t periodic, void *stream);

/* Weight and bias gradients of lbm_conv2d_forward without activation:
 *   dw[ky*k+kx][co][ci] = sum_{n,y,x} dout[n,y,x,co] in[n, y+ky-k/2, x+kx-k/2, ci],  db[co] = sum dout[.., co]
 * fp32 outputs (db may be NULL), deterministic (fixed reduction order).  work: fp32 workspace of
 * at least *elems elements as returned by lbm_conv2d_wgrad_workspace for the same sizes (host). */
lbm_status lbm_conv2d_wgrad_workspace(int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout, int32_t ksize,
                                      int64_t *elems);
lbm_status lbm_conv2d_wgrad(const void *in, const void *dout, float *dw, float *db, float *work, int64_t work_elems,
                            int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout, int32_t ksize,
                            int32_t periodic, void *stream);

/* Network shape: level l (0 .. levels-1) works at (height >> l) x (width >> l) with
 * base_channels << l channels and two 3x3 convolutions + ReLU; levels are joined by 2x2 average
 * pooling on the way down and nearest 2x upsampling + concatenation with the same level's encoder
 * output on the way up; a 1x1 convolution gives out_channels outputs.  The input tensor has
 * in_channels rounded up to a multiple of 8 (the extra channels are zero). */
typedef struct {
    int32_t levels;        /* 1 .. 8 */
    int32_t base_channels; /* multiple of 8 */
    int32_t in_channels;   /* >= 1 */
    int32_t out_channels;  /* 1 .. 8 */
    int32_t height, width; /* multiples of 2^(levels-1) */
    int32_t max_batch;     /* images per forward/backward call */
    int32_t periodic;      /* 0: convolutions zero-pad the image edges; 1: they wrap around (doubly
                              periodic domains) */
} lbm_nn_config;

typedef struct lbm_nn lbm_nn;

/* Allocates the network (fp32 master parameters, Adam moments, bf16 copies, activations for
 * max_batch images) on the current device; parameters get a seeded He-normal initialisation and
 * zero biases.  Every call on the network runs on `stream` (hipStream_t, NULL = null stream).
 * Parameter vector layout, in this order: for each encoder level 0..levels-1 its two
 * convolutions, then for each decoder level levels-2..0 its two convolutions, then the 1x1 output
 * convolution; each convolution is its weights [k*k][cout][cin] followed by its bias [cout]; the
 * output convolution has cout = 8 (rows >= out_channels stay zero). */
lbm_status lbm_nn_create(const lbm_nn_config *cfg, uint64_t seed, void *stream, lbm_nn **out);
lbm_status lbm_nn_destroy(lbm_nn *net);
lbm_status lbm_nn_param_count(const lbm_nn *net, int64_t *count);
/* Host fp32 parameter vector in / out (set also resets the Adam state). */
lbm_status lbm_nn_set_params(lbm_nn *net, const float *host);
lbm_status lbm_nn_get_params(const lbm_nn *net, float *host);
/* Host fp32 gradient of the last lbm_nn_backward, parameter layout. */
lbm_status lbm_nn_get_grads(const lbm_nn *net, float *host);

/* Forward pass of `batch` images: in bf16 [batch, height, width, ceil8(in_channels)];
 * out fp32 [batch, height, width, out_channels] (NULL: kept inside for lbm_nn_backward). */
lbm_status lbm_nn_forward(lbm_nn *net, const void *in, float *out, int32_t batch);

/* Loss and gradients of the last forward pass (same batch):
 *   loss = sum_{p: mask[p] != 0, c < out_channels} (out[p,c] - target[p,c])^2 / (count * out_channels)
 * with count = number of nonzero mask pixels; target fp32 [batch, height, width, out_channels],
 * mask uint8 [batch, height, width].  Writes every parameter gradient; *loss (host) on return.
 * Synchronises the stream. */
lbm_status lbm_nn_backward(lbm_nn *net, const float *target, const uint8_t *mask, int32_t batch, double *loss);

/* One Adam step on every parameter from the last gradients (bias-corrected, step count kept by
 * the network), then refreshes the bf16 copies. */
lbm_status lbm_nn_adam_step(lbm_nn *net, float lr, float beta1, float beta2, float eps);

/* Input features of one lattice (the network's 12 inputs, channels 12 .. channels-1 zero):
 *   0      1 on fluid sites, 0 on solid sites
 *   1..8   on fluid sites: q of the wall link in D2Q9 direction d (1 = E, 2 = N, 3 = W, 4 = S,
 *          5 = NE, 6 = NW, 7 = SW, 8 = SE), 1 where direction d has no wall link; 0 on solid sites
 *   9      kn_feature, 10 ax_feature, 11 ay_feature (constant over the image)
 * solid uint8 [ny * nx] (nonzero = solid); links: n_links records of lbm_link in device memory,
 * records outside the grid or with dir outside 1..8 are skipped (duplicates: one of them is kept).
 * out bf16 [ny, nx, channels], channels a multiple of 8 and >= 16. */
lbm_status lbm_nn_features(const uint8_t *solid, const lbm_link *links, int64_t n_links, int32_t nx, int32_t ny,
                           float kn_feature, float ax_feature, float ay_feature, void *out, int32_t channels,
                           void *stream);

/* Initial fields from one image of network output pred fp32 [ny * nx, stride] (channels: u_x, u_y,
 * delta rho, normalised).  The three channels are taken on fluid sites (0 on solid sites) and
 * smoothed smooth_iters times, each pass replacing the value at a fluid site by the mean over the
 * fluid sites of its 3 x 3 neighbourhood (wrapping around the edges if periodic, else bounded by
 * them); then on fluid sites ux = u_scale t0, uy = u_scale t1, rho = rho0 + rho_scale (t2 - mean
 * of t2 over fluid sites), so that the total mass equals that of the rest state; solid sites get
 * rho0 and 0.  rho, ux, uy: fp64 [ny * nx].  *n_bad (host) = number of fluid sites with a
 * non-finite value after smoothing (the caller falls back to rest if > 0).  Allocates and frees
 * 48 bytes of device memory per site; synchronises the stream. */
lbm_status lbm_nn_fields(const float *pred, int32_t stride, const uint8_t *solid, int32_t nx, int32_t ny,
                         int32_t smooth_iters, int32_t periodic, double u_scale, double rho_scale, double rho0,
                         double *rho, double *ux, double *uy, int64_t *n_bad, void *stream);

/* lbm_nn_fields without any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * results as lbm_nn_fields; its scratch (two sets of three fp64 planes and a count) lives in a fixed
 * device array of the library, sized for nx * ny <= 262144 sites (12.6 MB, held by every GPU the
 * library runs on until the process ends).  Larger lattices: LBM_E_INVAL before any device work.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race, so the caller serialises them.  No call here allocates or frees device memory. */
lbm_status lbm_nn_fields_noalloc(const float *pred, int32_t stride, const uint8_t *solid, int32_t nx, int32_t ny,
                                 int32_t smooth_iters, int32_t periodic, double u_scale, double rho_scale,
                                 double rho0, double *rho, double *ux, double *uy, int64_t *n_bad, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
