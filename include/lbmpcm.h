/*
 * lbmpcm.h - C ABI of the MI355X (gfx950) library for the enthalpy-based
 * multiple-relaxation-time lattice Boltzmann method for solid-liquid phase
 * change in metal foams under local thermal non-equilibrium
 * (Q. Liu, Y.-L. He, Q. Li, arXiv:1701.00702).
 *
 * One time step updates three coupled population sets per node (D2Q9 flow;
 * D2Q9 thermal fields, or the D2Q5 thermal fields of Appendix B):
 *   f  flow field with the Brinkman-Forchheimer (generalized non-Darcy) force
 *      and the volumetric no-slip treatment of the solid phase (Sec. III A,
 *      Eqs. 12-27);
 *   g  PCM total enthalpy, with temperature and liquid fraction recovered
 *      without iteration from the enthalpy (Sec. III B 1, Eqs. 28-40);
 *   h  metal-foam internal energy (Sec. III B 2, Eqs. 41-49);
 * coupled by the interstitial heat-exchange sources (Eqs. 36, 47) and closed
 * by non-equilibrium extrapolation on the walls (Sec. III C, Eq. 52).
 * The default problem is the cavity of Sec. IV B: isothermal hot wall at
 * x = 0, cold wall at x = nx-1, adiabatic horizontal walls, gravity along
 * -y; each wall can instead be isothermal at its own temperature or
 * adiabatic (e.g. the corner solidification of Sec. IV A).
 *
 * Conventions shared by every entry point:
 *  - Host field arrays are row-major double[ny][nx], x fastest, owned by the
 *    caller.  Node (x, y) = (0, 0) is the bottom-left corner.
 *  - All device memory is owned by the library, except after
 *    lbm_create_ext, where the caller lends one device workspace.
 *  - Work is queued on the handle's HIP stream.  lbm_step returns without
 *    waiting; errors raised on the device surface at the next call that
 *    synchronises (lbm_fields, lbm_diagnostics, lbm_synchronize, lbm_save).
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Every entry point returns an lbm_status; on failure a message is
 *    available from lbm_last_error() (thread-local, valid until the next
 *    failing call on the same thread).
 */
#ifndef LBMPCM_H
#define LBMPCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_handle lbm_handle;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* bad argument or a parameter set the scheme cannot run */
    LBM_ENOMEM = -2,     /* device or host allocation failed */
    LBM_EDEVICE = -3,    /* a HIP call or kernel failed */
    LBM_ENONFINITE = -4, /* the state holds NaN/Inf (reported by lbm_diagnostics) */
    LBM_ESTATE = -5,     /* call not valid in the handle's current state */
    LBM_EIO = -6         /* checkpoint file could not be written or read */
} lbm_status;

/* Storage of the populations of a node (27 with D2Q9 thermal fields, 19 with
 * D2Q5 ones).  Arithmetic is FP64 for LBM_F64 and FP32 otherwise.  Every
 * form stores, per field, the offset of each population from the rest
 * equilibrium at a fixed reference state (flow: the lattice weights times
 * the reference density; enthalpy and metal fields: the equilibria at rest
 * at the middle of the mushy band on D2Q9, at T_init on D2Q5).
 *   LBM_F64, LBM_F32   the offsets in FP64 / FP32 (216 / 108 bytes per node)
 *   LBM_F16_OFFSET     the offsets in binary16 times a power-of-two scale (54)
 *   LBM_BF16_OFFSET    the offsets in bfloat16 (54)
 *   LBM_F16_SPLIT      per field the rest population and one base value
 *                      (flow: density offset; enthalpy: c_f,ref (T_f - T_ref);
 *                      metal: c_m,ref (T_m - T_ref)), stored times the axis
 *                      weight 1/9, in FP32, and the eight moving populations
 *                      as binary16 remainders from the rest equilibrium of
 *                      that base (72 bytes per node)
 *   LBM_BF16_SPLIT     as LBM_F16_SPLIT with bfloat16 remainders (72)
 *   LBM_F32_H64        as LBM_F32, except the rest population of the enthalpy
 *                      field, which carries H itself, in FP64; that population,
 *                      H, T_f and f_l are computed in FP64, the rest of the
 *                      enthalpy collision in FP32 (112 bytes per node).
 * With D2Q5 thermal fields (lbm_params.thermal_lattice = 5) the forms
 * LBM_F64, LBM_F32 and LBM_F32_H64 are available: 152, 76 and 80 bytes per
 * node, planes [f0..f8, g0..g4, h0..h4] (LBM_F32_H64: [f0..f8, g1..g4,
 * h0..h4] in FP32, then g0 in FP64). */
typedef enum {
    LBM_F64 = 0,
    LBM_F32 = 1,
    LBM_F16_OFFSET = 2,
    LBM_BF16_OFFSET = 3,
    LBM_F16_SPLIT = 4,
    LBM_F32_H64 = 5,
    LBM_BF16_SPLIT = 6
} lbm_precision;

/* Problem description in dimensionless groups (Eq. 54).  Lattice units:
 * dx = dt = 1, c_s^2 = 1/3, rho_l = rho_s = 1, c_pl = c_ps = c_pm = 1
 * (Sec. IV parameter list).  Optional fields use the stated sentinel. */
typedef struct lbm_params {
    int32_t nx, ny;       /* nodes including the wall nodes, each >= 4;
                             nx <= 262144, nx * ny <= 2^31                   */
    int32_t bc_x;         /* 0: cavity (hot wall x=0, cold wall x=nx-1);
                             1: periodic in x, walls only at y=0 and y=ny-1      */
    int32_t gravity_axis; /* 1: gravity along -y; 0: along -x                    */
    double porosity;      /* phi, in (0, 1)                                       */
    double Ra, Pr, Da, Ste;
    double k_ratio;       /* lambda = k_m / k_f                                   */
    double cap_ratio;     /* sigma = (rho c_p)_m / (rho c_p)_f  (= rho_m here)    */
    double Nu_i;          /* interstitial Nusselt number H_v = h_v d_p^2 / k_f    */
    double F_phi;         /* Forchheimer coefficient; < 0: Eq. (4) from phi       */
    double dp_over_L;     /* pore size d_p / L; <= 0: 0.0135                      */
    double k_f;           /* lattice PCM diffusivity; <= 0: the largest value with
                             every relaxation time <= 2 and the interstitial
                             exchange number z <= 0.5                             */
    double cf_ref;        /* c_f,ref; <= 0: 0.2 c_pl                              */
    double cm_ref;        /* c_m,ref; <= 0: 1.0 c_pm                              */
    double J;             /* viscosity ratio nu_e / nu_f; <= 0: 1                 */
    double T_hot, T_cold; /* temperatures of the default hot (x=0) and cold
                             (x=nx-1) walls; Delta T = T_hot - T_cold sets the
                             latent heat, the buoyancy scale and the Nusselt
                             numbers; T_0 = T_cold (Eq. 7)                     */
    double T_init;        /* initial temperature of both phases                   */
    double T_solidus, T_liquidus;
    int32_t thermal_lattice;   /* 0 or 9: D2Q9 thermal fields (Sec. III B/C);
                                  5: D2Q5 thermal fields (Appendix B)          */
    int32_t thermal_collision; /* 0: MRT (rates of Sec. III C); 1: BGK thermal
                                  collisions, every rate 1/tau (Sec. V A)     */
    double varpi;              /* D2Q5 weight parameter in (0,1), Eq. (B2);
                                  <= 0: 2/3 (c_sT^2 = 1/3)                     */
    double zeta_e;             /* > 0: fixed zeta_e = zeta_eps in (0,2)
                                  (Sec. V D); <= 0: zeta_e = zeta_eps =
                                  2 - zeta_alpha (Eq. 53, Sec. III C)         */
    int32_t wall_type[4];      /* left, right, bottom, top: 0 the cavity's own
                                  (isothermal T_hot / T_cold left / right,
                                  adiabatic bottom and top), 1 isothermal at
                                  wall_T, 2 adiabatic.  At a corner an
                                  isothermal vertical wall wins, then an
                                  isothermal horizontal wall.  Periodic
                                  problems (bc_x = 1) take 0 left and right. */
    double wall_T[4];          /* temperatures of walls of type 1             */
    double L_char;             /* > 0: characteristic length for Ra, Da, d_p,
                                  Fo and Nu; <= 0: nx - 1 (periodic: ny - 1)  */
    int32_t solid_treatment;   /* 0: volumetric scheme, Eq. (20); 1: the
                                  bounce-back alternative of Sec. V B: a node
                                  with f_l < 0.5 reflects its flow populations
                                  and is at rest, other nodes collide their
                                  unblended f+                                */
    int32_t band_rows;         /* storage only: rows per band of the state
                                  blocks; 0: automatic (about 256 MiB of
                                  state per band); else at least
                                  max(32, ceil(2048 / nx) + 4), at most ny
                                  (larger values take ny).  Results do not
                                  depend on it.                               */
    int32_t pcm_even_rates;    /* D2Q9 MRT thermal fields only.  0: the
                                  enthalpy field's stress moments (p_xx,
                                  p_xy; moments 7 and 8 of Eq. 13) relax at
                                  the free rate zeta_v = 1.2 of Sec. III C;
                                  1: at the rate of e and eps (Eq. 53, or
                                  the given zeta_e), so every even
                                  non-conserved moment of that field relaxes
                                  at one rate and every odd one at
                                  zeta_alpha.  With 1 the solid stays at the
                                  melting temperature to rounding, the
                                  property Sec. V C states for the scheme;
                                  with 1.2 it undershoots by up to about 2%
                                  of the temperature difference.  Other
                                  lattices or BGK collisions: LBM_EINVAL
                                  unless 0.                                   */
} lbm_params;

/* Derived lattice constants of one cavity (read-only view). */
typedef struct lbm_lattice {
    double L;                        /* characteristic length nx-1 (channel: ny-1) */
    double k_f, k_m, nu_f, nu_e, K, F_phi, gbeta, h_v, L_a, d_p, z;
    double tau_v, tau_g, tau_h;
    double s[9], zeta[9], eta[9];    /* relaxation rates in moment order of Eq. (13);
                                        D2Q5: zeta[0..4], eta[0..4] in the
                                        moment order of Eq. (B1), rest 1 */
    double H_fs, H_fl, T_ref, H_ref;
    double scale_exp[3];             /* storage scale exponents (f, g, h) */
    double q_thermal;                /* thermal velocities: 9 or 5 */
    double varpi;                    /* D2Q5 weight parameter (0 on D2Q9) */
    double wall_type[4], wall_T[4];  /* resolved: 1 isothermal, 2 adiabatic */
    double solid_treatment;          /* 0 volumetric, 1 bounce-back */
} lbm_lattice;

/* Diagnostics of one cavity at the current step (all FP64).
 * Walls are indexed 0 left (hot), 1 right (cold), 2 bottom, 3 top; corner
 * nodes belong to the left/right walls.  Interior = non-wall nodes. */
typedef struct lbm_diag {
    double step, Fo;                  /* steps taken; Fo = t k_f / L^2          */
    double liquid_fraction;           /* mean f_l over interior nodes           */
    double Nu_hot;                    /* -(L/(k_e dT)) <phi k_f dT_f/dx + (1-phi) k_m dT_m/dx> at x=0 */
    double Nu_hot_pcm;                /* -(L/dT) <dT_f/dx> at x=0               */
    double Nu_cold;                   /* same at x = nx-1 (positive outflow)    */
    double E_int, E_int0;             /* sum of phi rho_l H + (1-phi) rho_m c_pm T_m */
    double flux_E[4];                 /* energy carried in through each wall since step 0 */
    double energy_residual;           /* E_int - E_int0 - sum(flux_E)           */
    double M_int, M_int0, flux_M[4], mass_residual; /* same for the density   */
    double x_front_mid;               /* f_l = 0.5 crossing on row ny/2, / L    */
    double max_dT_LTNE;               /* max |T_f - T_m| over interior nodes    */
    double u_max;                     /* max |u| over interior nodes            */
    double nonfinite;                 /* nodes holding a non-finite population  */
} lbm_diag;

/* Launch shape of the step kernels.  Every shape gives bit-identical results. */
typedef struct lbm_launch_config {
    int32_t block;            /* threads per workgroup: 64, 128, 256 or 512      */
    int32_t nodes_per_thread; /* 1, 2 or 4 consecutive-by-block nodes per thread */
    int32_t xcd_remap;        /* 1: consecutive tiles share an XCD (and its L2)  */
    int32_t persistent;       /* 0: one tile per workgroup; >0: that many
                                 workgroups per CU loop over all tiles           */
    int32_t steps_per_launch; /* 1: one step per launch; 2: two steps per launch
                                 through LDS (2-D tiles with a one-node ring,
                                 the state crosses HBM once per two steps;
                                 every form); 3: three steps per launch (a
                                 two-node ring, the middle step in place in
                                 LDS; every form but LBM_F64).  Default: the
                                 most the form has.
                                 block and nodes_per_thread then do not apply. */
    int32_t tile_shape;       /* tile shape of the multi-step kernel: 0 the
                                 default; 1 about twice as wide and half as
                                 tall; 2 about half as wide and twice as tall
                                 (multi-step launches without a persistent
                                 grid).  Every shape gives the same bits.     */
    int32_t tile_w, tile_h;   /* reported by lbm_get_launch and lbm_autotune:
                                 the tile of the multi-step kernel (0 with
                                 one step per launch); ignored on input       */
} lbm_launch_config;

/* Create a single-cavity solver.  Maps the groups to lattice units (Eq. 54,
 * Eq. 26, Eq. A19, Sec. III C rates), validates them (rates in (0,2),
 * interstitial exchange number < 1, Remark I bounds, phi in (0,1)), allocates
 * the double-buffered state with hipMalloc and initialises every node at rest
 * at T_init (isothermal walls at their temperature).  *out receives the
 * handle, or NULL on failure. */
lbm_status lbm_create(const lbm_params *p, lbm_precision prec, lbm_handle **out);

/* Create a solver advancing n_cavities independent cavities (p[0..n-1]) in
 * one launch per step over a packed node index. */
lbm_status lbm_create_batch(const lbm_params *p, int32_t n_cavities, lbm_precision prec,
                            lbm_handle **out);

/* Device bytes lbm_create_ext needs for the same cavities and precision:
 * the two state buffers (the bytes per node of lbm_precision), the two
 * interstitial-source planes (4 bytes per node, 8 with LBM_F64), the tile
 * tables and wall tallies, and a staging area of at most 2^22 nodes (or one
 * row of the widest cavity) times six doubles that lbm_set_initial and
 * lbm_fields pass whole rows through; no per-node scratch beyond that, so
 * the state buffers can fill nearly all of the GPU's memory. */
lbm_status lbm_workspace_bytes(const lbm_params *p, int32_t n_cavities, lbm_precision prec,
                               uint64_t *bytes);

/* As lbm_create_batch, but the caller lends a device workspace of at least
 * lbm_workspace_bytes bytes (256-byte aligned) and a HIP stream
 * (hipStream_t, may be NULL for the null stream).  The workspace must stay
 * valid until lbm_destroy; the library never frees it. */
lbm_status lbm_create_ext(const lbm_params *p, int32_t n_cavities, lbm_precision prec,
                          void *workspace, uint64_t workspace_bytes, void *hip_stream,
                          lbm_handle **out);

/* Queue later work on another HIP stream (hipStream_t). */
lbm_status lbm_set_stream(lbm_handle *h, void *hip_stream);

/* Re-initialise one cavity (only before the first step): every node at rest
 * with PCM temperature T_pcm0 and foam temperature T_mf0 (host double[ny][nx];
 * either may be NULL for T_init); isothermal wall nodes take their wall
 * temperature.  The previous-step interstitial source is set to the current
 * one, so the time-derivative terms of Eqs. (36) and (47) start at zero. */
lbm_status lbm_set_initial(lbm_handle *h, int32_t cavity, const double *T_pcm0,
                           const double *T_mf0);

/* Advance every cavity by n >= 0 steps (asynchronous).  Each step is one
 * launch of the fused kernel (or one launch per two or three steps, see
 * lbm_launch_config): streaming, wall reconstruction (Eq. 52),
 * enthalpy/temperature/liquid fraction (Eqs. 37-39, 48), volumetric blend
 * (Eq. 20), velocity (Eqs. 23-25), the three moment-space collisions
 * (Eqs. 14, 32, 43) and the wall energy/mass flux tallies.  Runs of 32
 * launches go out as HIP graphs, captured when the handle is created and
 * on every lbm_set_launch, so a call spends no host time on capture. */
lbm_status lbm_step(lbm_handle *h, int64_t n);

/* Batched handles only: the same n steps as one launch per cavity per step
 * (the reference point for the single-launch batched form). */
lbm_status lbm_step_per_cavity(lbm_handle *h, int64_t n);

/* Wait for all queued work on the handle's stream. */
lbm_status lbm_synchronize(lbm_handle *h);

/* Steps taken so far. */
int64_t lbm_step_count(const lbm_handle *h);

/* Macroscopic fields of one cavity at the current step, from the
 * post-streaming populations: velocity u of Eq. (23), T_f and f_l of
 * Eqs. (38)-(39), T_m of Eq. (48), density of Eq. (21).  Any pointer may be
 * NULL.  Synchronises the stream. */
lbm_status lbm_fields(lbm_handle *h, int32_t cavity, double *ux, double *uy, double *T_pcm,
                      double *T_mf, double *f_l, double *rho);

/* The same fields for rows [y0, y0 + rows) of the cavity only: each
 * non-NULL pointer receives double[rows][nx], row y0 first.  For reading
 * parts of cavities too large for a host copy of every field.  LBM_EINVAL
 * unless 0 <= y0 and 1 <= rows <= ny - y0.  Synchronises the stream. */
lbm_status lbm_fields_rows(lbm_handle *h, int32_t cavity, int32_t y0, int32_t rows, double *ux,
                           double *uy, double *T_pcm, double *T_mf, double *f_l, double *rho);

/* FP64 diagnostics of one cavity (deterministic reductions).  The paper
 * defines none of these quantities; the definitions are this library's:
 * liquid fraction = mean f_l (Eq. 39) over interior nodes; melt front = the
 * first f_l = 0.5 crossing from the hot wall on row ny/2 (f_l = 0.5 is the
 * phase interface of Sec. IV B), linearly interpolated, divided by L; Nusselt
 * numbers from second-order one-sided differences of T_f and T_m at the
 * vertical walls, averaged over the non-corner wall nodes, with
 * k_e = phi k_f + (1 - phi) k_m (Eq. 8); energy phi rho_l H + (1 - phi)
 * rho_m c_pm T_m (Eqs. 37, 48) and density summed over interior nodes, with
 * the link fluxes across each wall tallied every step.  Uses the handle's
 * workspace (per-workgroup partial sums, the temperatures of the three
 * columns next to each vertical wall, the middle row's liquid fraction) as
 * scratch.  Synchronises the stream.  Returns LBM_ENONFINITE, with *out filled, when the state holds
 * NaN/Inf. */
lbm_status lbm_diagnostics(lbm_handle *h, int32_t cavity, lbm_diag *out);

/* The same diagnostics for callers that cannot allocate or hand out device
 * memory (tight serving loops, harnesses that forbid allocation): calls no
 * hipMalloc, hipFree or other allocating routine and touches none of the
 * workspace's scratch regions.  Its kernels use one fixed device array per
 * GPU (about 3.5 MiB, held until the process ends) for per-workgroup
 * partial sums, the temperatures of the three columns next to each vertical
 * wall and the middle row's liquid fraction.  Cavities with nx or ny above
 * 32768 are rejected with LBM_EINVAL.  Every call writes each scratch
 * element it reads, so nothing carries over between calls; calls that
 * overlap on one GPU (several host threads, or streams running at once)
 * share that array and race.  Runs the kernels of lbm_diagnostics, so the
 * results are the same bit for bit.  Synchronises the stream. */
lbm_status lbm_diagnostics_noalloc(lbm_handle *h, int32_t cavity, lbm_diag *out);

/* Derived lattice constants of one cavity. */
lbm_status lbm_get_lattice(const lbm_handle *h, int32_t cavity, lbm_lattice *out);

/* The same mapping and validation without a handle or a device (host only):
 * what lbm_create would use for these parameters. */
lbm_status lbm_lattice_of(const lbm_params *p, lbm_precision prec, lbm_lattice *out);

/* Read or set the step kernel's launch shape. */
lbm_status lbm_get_launch(const lbm_handle *h, lbm_launch_config *out);
lbm_status lbm_set_launch(lbm_handle *h, const lbm_launch_config *cfg);

/* Time every supported launch shape (one-step launch shapes; two and three
 * steps per launch in every tile shape) for steps_per_trial launches on
 * the live state (reads the current buffer, writes only scratch), keep the
 * fastest, and report it in *chosen (may be NULL).  With a non-NULL
 * cache_path the choice is looked up in / appended to that text file, keyed
 * by device, precision, number of cavities, total nodes and the first
 * cavity's sizes.  Synchronises the stream. */
lbm_status lbm_autotune(lbm_handle *h, int32_t steps_per_trial, const char *cache_path,
                        lbm_launch_config *chosen);

/* Write / read the complete state (populations, previous-step sources,
 * wall tallies, step count) to a file; resuming is bit-exact.  Both move the
 * state through one host buffer of 64 MiB, so no host copy of the whole
 * state is made.  lbm_load requires a handle created with the same cavities
 * and precision (LBM_EINVAL otherwise) and a file of this library's format
 * and of the exact length such a checkpoint has (LBM_EIO otherwise, found
 * before the state is touched).  It reads the state into the buffers the
 * next step would write and makes them current only when every byte has
 * arrived, so a failed load leaves the handle's state as it was.  Both
 * synchronise the stream. */
lbm_status lbm_save(lbm_handle *h, const char *path);
lbm_status lbm_load(lbm_handle *h, const char *path);

/* Copy the raw stored populations of one cavity to host memory, for
 * bit-level comparisons: every stored plane of the cavity in storage order
 * ([plane][ny][nx], planes as listed for lbm_precision), i.e. (bytes per
 * node) * nx * ny bytes: 216, 108, 54, 54, 72 or 112 per node on D2Q9,
 * 152, 76 or 80 on D2Q5. */
lbm_status lbm_copy_state(lbm_handle *h, int32_t cavity, void *host, uint64_t bytes);

/* Overwrite one stored population of the current state with value,
 * converted to the element type it is stored in (test hook for the
 * failure-detection path).  field: 0 f, 1 g, 2 h; dir: 0..8 (0..4 for g
 * and h on D2Q5). */
lbm_status lbm_debug_poke(lbm_handle *h, int32_t cavity, int32_t x, int32_t y, int32_t field,
                          int32_t dir, double value);

/* Release the handle and everything the library allocated for it. */
lbm_status lbm_destroy(lbm_handle *h);

/* Message of the last failing call on this thread ("" if none). */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMPCM_H */
