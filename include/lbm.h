/*
 * lbm.h -- C ABI of the MI355X (gfx950) porous-media lattice Boltzmann library.
 *
 * The library advances the one-domain lattice Boltzmann scheme of Gusev & Karlin,
 * "Monolithic kinetic algorithm for heterogeneous porous media systems using a continuous
 * one-domain approach" (arXiv 2606.29619), on the D2Q9 and D3Q27 lattices (Sec. 3.1):
 * the product-form porosity-scaled equilibrium (Sec. 3.2), the Relax-to-Force shifted
 * equilibrium with the extended-equilibrium and bulk-viscosity corrections (Sec. 3.2), the
 * collide-and-stream update with per-cell relaxation beta (Sec. 3.3, eq. dicrete_scheme), the
 * closed-form Darcy-Forchheimer velocity solve and the variable-porosity viscous correction
 * (Sec. 3.3, eqs. v_(0), v_(1), v_final, accel, porosity_correction), in one code path for
 * free-fluid and porous cells.
 *
 * Geometry.  Cells are indexed n = x + nx*(y + ny*z) (x fastest).  Every axis wraps
 * periodically; walls are layers of solid cells (mask = 1), which reflect populations by
 * halfway (link-wise) bounce-back.  The porosity is read on every cell, solid cells included;
 * its derivatives are central differences.  Derivatives of moment fields become one-sided next
 * to solid cells (Sec. 3.5, last paragraph).  Consequence: the porosity given to a solid cell
 * enters grad eps and the Hessian of eps at its fluid neighbours, and through them the
 * RT grad eps force of eqs. (v_(0), accel) and Delta_nu (eq. porosity_correction_expanded) of
 * the first fluid layer.  Give solid cells a smooth continuation of the fluid porosity (for a
 * flat wall, the value of the adjacent fluid cell) unless a porosity jump at the wall is meant;
 * analytic derivatives (lbm_params.grad_eps, hess_eps) avoid the question.
 *
 * Conventions common to every entry point:
 *   - every function returns LBM_OK (0) or a negative LBM_ERR_* code and never throws;
 *   - lbm_last_error() returns a description of the calling thread's last failure;
 *   - device pointers are HIP device addresses on the device that was current at lbm_create;
 *   - all device work is enqueued on the stream given to lbm_create, in order, and is
 *     asynchronous unless a function says it synchronises;
 *   - a solver handle must not be used from two threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_API __attribute__((visibility("default")))

/* Return codes. */
#define LBM_OK 0
#define LBM_ERR_INVALID_ARG -1   /* a parameter, field value or pointer is out of its domain */
#define LBM_ERR_UNSUPPORTED -2   /* a valid combination this library does not implement */
#define LBM_ERR_WORKSPACE -3     /* the device workspace is too small or misaligned */
#define LBM_ERR_HIP -4           /* a HIP runtime call or kernel launch failed */
#define LBM_ERR_NONFINITE -5     /* the state holds NaN or Inf (reported by lbm_residual) */
#define LBM_ERR_STATE -6         /* a call out of order (e.g. on a destroyed handle) */

/* Lattices (Sec. 3.1): the value is Q. */
#define LBM_D2Q9 9
#define LBM_D3Q27 27

/*
 * Storage of the populations.  LBM_F64 and LBM_F32 store f-bar and compute in that type
 * (static fields and moments too).  The shifted 16-bit forms store, per population,
 * (f-bar_i - sigma_i) * 2^12 / w_i in FP16 or BF16 (w_i: lattice weight, the rest state of
 * the product-form equilibrium, eq. prod_form), with sigma_i chosen by lbm_params.shift; every
 * value is decoded to FP32, collided in FP32 and re-encoded (round to nearest even); static
 * fields and moment records are FP32, statistics FP64.
 */
#define LBM_F64 0
#define LBM_F32 1
#define LBM_F16_SHIFTED 2
#define LBM_BF16_SHIFTED 3

/*
 * Shift sigma_i of the 16-bit storage forms.
 * LBM_SHIFT_WEIGHTS: sigma_i = rho0 w_i, the lattice weights.
 * LBM_SHIFT_POROUS:  sigma_i = rho0 eps(src) w_i, src being the cell whose collision produced
 *   the value (the upstream cell x - c_i, or x itself after a bounce-back).  A porous cell at
 *   rest holds eps rho0 w_i (eq. prod_form with v = 0), so this shift removes the porosity
 *   from the stored deviation.
 */
#define LBM_SHIFT_WEIGHTS 0
#define LBM_SHIFT_POROUS 1

/*
 * Time-stepping scheme.
 * LBM_SCHEME_TWO_PASS follows Sec. 3.5 as written: every step first takes the moments and the
 *   corrected velocity of all cells (pass one), then forces, collides and streams (pass two).
 * LBM_SCHEME_LAGGED fuses both into one pass over the populations: a cell's own moments,
 *   velocity correction and forcing use its current populations, while the neighbour values
 *   inside the stencils of Delta_nu, Phi^ext and Phi^eta are the previous step's.  A steady
 *   state of either scheme is one of the other; transients differ by O(dt).  The first step
 *   after lbm_create uses the initial fields as the previous step; the first step after
 *   lbm_set_populations is a two-pass step.
 */
#define LBM_SCHEME_TWO_PASS 0
#define LBM_SCHEME_LAGGED 1

/*
 * Wet-node boundaries (Sec. 3.4).  A boundary node is a fluid cell whose outward neighbour
 * along each of its outward normals is solid (mask = 1).  Under LBM_SCHEME_LAGGED the boundary
 * density and velocity come from the current step's moments, while the acceleration of the
 * rebuild, like the bulk correction and forcing, takes its neighbours' values from the
 * previous step; such a step runs as separate passes.
 *   Face nodes (one normal): the inward neighbour must be a bulk fluid cell.
 *   Edge and corner nodes (two or three normals, Sec. 3.4.1): velocity nodes only; the two
 *     cells x_b + d and x_b + 2d along the inward diagonal d = -(sum of the normals) must be
 *     bulk fluid cells.
 * Node types (lbm_params.bc_type):
 *   LBM_NODE_VELOCITY: superficial velocity v_b prescribed.  Density under
 *     LBM_BC_RHO_CONTINUITY: on faces from mass continuity, eq. (bc_density_impermWall), with
 *     a_b,perp of eq. (accel_approx_boundary), viscous term included (evaluated from the
 *     drag-solved velocities v^(1) of the bulk cells and the boundary velocities of the nodes at
 *     that point of the step); on edges and corners, where that relation does not apply,
 *     extrapolated from the bulk, rho_b = 2 rho(x_b + d) - rho(x_b + 2d).  Under
 *     LBM_BC_RHO_BOUNCE_BACK: eq. (bc_density_BounceBack) everywhere (meant for solid walls;
 *     an inflow boundary needs the continuity rule).  All populations rebuilt by
 *     lbm_params.bc_scheme;
 *   LBM_NODE_PRESSURE (faces only): intrinsic density rho_b prescribed, tangential velocity zero,
 *     normal velocity from the same continuity relation (a_b,perp without the viscous term);
 *     populations rebuilt by bc_scheme;
 *   LBM_NODE_OUTFLOW (faces only): zero-gradient outflow, eq. (f_bar_outflow_BC).
 * Schemes: LBM_BC_EQUILIBRIUM (eq_bc_f_bar), LBM_BC_NEEM (NEEM_bc_f_bar, zeta_beta_NEEM; on edges
 * and corners the inner node is x_b + d), LBM_BC_TMS (Sec. 3.4.4, f_i_neq_TMS; the unknown set
 * P- holds every population that enters through one of the node's faces).  Links of bulk cells
 * into solid cells keep halfway bounce-back.
 * bc_normal: LBM_NORMAL_XM .. LBM_NORMAL_ZP for one normal, LBM_NORMAL_AXES(sx, sy, sz) with
 * s in {-1, 0, 1} per axis for any number (sz = 0 in 2D).
 */
#define LBM_NODE_BULK 0
#define LBM_NODE_VELOCITY 1
#define LBM_NODE_PRESSURE 2
#define LBM_NODE_OUTFLOW 3
#define LBM_NORMAL_XM 0   /* outward normal -x */
#define LBM_NORMAL_XP 1
#define LBM_NORMAL_YM 2
#define LBM_NORMAL_YP 3
#define LBM_NORMAL_ZM 4
#define LBM_NORMAL_ZP 5
#define LBM_NORMAL_SIGN_(s) ((s) < 0 ? 1 : ((s) > 0 ? 2 : 0))
#define LBM_NORMAL_AXES(sx, sy, sz) \
    (64 + LBM_NORMAL_SIGN_(sx) + 4 * LBM_NORMAL_SIGN_(sy) + 16 * LBM_NORMAL_SIGN_(sz))
#define LBM_BC_EQUILIBRIUM 0
#define LBM_BC_NEEM 1
#define LBM_BC_TMS 2
#define LBM_BC_RHO_CONTINUITY 0
#define LBM_BC_RHO_BOUNCE_BACK 1

/* Workgroup tiles (lbm_params.tiles). */
#define LBM_TILES_AUTO 0
#define LBM_TILES_RECTANGULAR 1

/* Kernels of a two-pass step (lbm_params.passes). */
#define LBM_PASSES_AUTO 0
#define LBM_PASSES_SEPARATE 1
#define LBM_PASSES_FUSED 2

/* Output element type for lbm_moments / lbm_get_populations / lbm_set_populations. */
#define LBM_DTYPE_F64 0
#define LBM_DTYPE_F32 1

/* Velocity returned by lbm_moments. */
#define LBM_VELOCITY_SUPERFICIAL 0   /* v (Sec. 2: the superficial or Darcy velocity) */
#define LBM_VELOCITY_INTRINSIC 1     /* u = v / eps */

/*
 * Run description.  Host arrays are read during lbm_create only (the library copies them);
 * the caller keeps ownership.  Arrays hold N = nx*ny*nz values in cell order; vector arrays
 * are [D][N] (component-major).
 */
typedef struct lbm_params {
    int lattice;          /* LBM_D2Q9 or LBM_D3Q27 */
    int storage;          /* LBM_F64, LBM_F32, LBM_F16_SHIFTED or LBM_BF16_SHIFTED */
    int scheme;           /* LBM_SCHEME_TWO_PASS or LBM_SCHEME_LAGGED */
    int shift;            /* LBM_SHIFT_WEIGHTS or LBM_SHIFT_POROUS (16-bit storage only) */
    int nx, ny, nz;       /* >= 1; nz must be 1 for D2Q9 */
    double RT;            /* lattice temperature RT > 0 (1/3 is the lattice reference); FP32
                             arithmetic uses 1 - fl(1 - fl(RT)), whose complement is exact
                             (for 1/3: 1.2e-7 relative above it), so that the equilibria of a
                             cell at rest sum to its mass */
    double nu_f;          /* fluid viscosity in the Darcy coefficient mu_D = eps nu_f / kappa
                             (eq. mu_D_Ergun_perm) */
    double nu_eff_ref;    /* effective shear viscosity nu_eff(eps) = nu_eff_ref * eps^nu_eff_pow > 0;
                             beta follows from eq. (nu_eff_def) with dt = 1 */
    int nu_eff_pow;       /* -1, 0 or 1 */
    double eta_eff;       /* effective bulk viscosity entering Phi^eta (eq. eta_corr);
                             NaN leaves Phi^eta out, which fixes eta = 2 nu_eff / D
                             (eq. eta_0_no_corr) */
    double b[3];          /* body acceleration (b[2] ignored for D2Q9) */
    double rho0;          /* initial intrinsic density where rho_init is NULL, > 0 */
    const double *eps;    /* [N] porosity in (0, 1] on every cell (solid cells included: their
                             values enter the differenced derivatives of the neighbouring fluid
                             cells, see Geometry above) */
    const double *kappa;  /* [N] permeability > 0 on fluid cells; +inf means free fluid */
    const double *forch;  /* [N] Forchheimer coefficient C_F >= 0 on fluid cells, so that
                             mu_F = eps C_F (eq. mu_F_Ergun_perm with C_F = F_eps/sqrt(kappa)) */
    const uint8_t *mask;  /* [N] 1 = solid cell, 0 = fluid; NULL = no solid cells */
    const double *rho_init; /* [N] initial intrinsic density > 0, or NULL (uniform rho0) */
    const double *v_init;   /* [D][N] initial superficial velocity, or NULL (zero) */
    const uint8_t *bc_type;     /* [N] LBM_NODE_*, or NULL (no wet-node boundaries) */
    const uint8_t *bc_normal;   /* [N] LBM_NORMAL_* or LBM_NORMAL_AXES() of each node */
    const double *bc_velocity;  /* [D][N] v_b of velocity nodes, or NULL (zero) */
    const double *bc_density;   /* [N] rho_b of pressure nodes, or NULL (rho0) */
    int bc_scheme;              /* LBM_BC_EQUILIBRIUM, LBM_BC_NEEM or LBM_BC_TMS */
    int bc_rho_rule;            /* LBM_BC_RHO_CONTINUITY or LBM_BC_RHO_BOUNCE_BACK */
    int picard_iters;           /* 0..64: Picard iterations of the second-order velocity
                                   evaluation (App. F) after the one-shot correction, two-pass
                                   scheme only; each is one stencil pass over the moment records
                                   (and, with boundaries, their records fixed again) */
    double picard_omega;        /* under-relaxation omega in (0, 1] of the iterations */
    /* Analytic porosity derivatives (Sec. 3.5: Delta_nu is best evaluated from analytic
     * derivatives of eps when eps(x) is known in closed form).  Both NULL: central differences
     * of eps.  Otherwise both are required, FP64, host memory, read only during lbm_create:
     *   grad_eps [D][N]         d eps / d x_a, a = x, y (, z);
     *   hess_eps [D(D+1)/2][N]  the Hessian's upper triangle row by row: xx, xy, yy (D2Q9) or
     *                           xx, xy, xz, yy, yz, zz (D3Q27).
     * They replace every derivative of eps in the step (the RT grad eps force of v_(0),
     * Delta_nu, and the wall-normal gradient at pressure and velocity nodes); values on solid
     * cells are never read.  They cost D + D(D+1)/2 extra values per cell of workspace and of
     * traffic in the passes that evaluate Delta_nu.  Only one of the two given, or a value
     * that is not finite on a fluid cell: LBM_ERR_INVALID_ARG. */
    const double *grad_eps;
    const double *hess_eps;
    /* Workgroup tiles of the cell passes: LBM_TILES_AUTO picks rows of 256, 128 or 64 cells and,
     * for an x extent that is not a multiple of 64 (16-bit storage: D3Q27 runs whose rows would
     * leave at least 30 % of the lanes idle), packed rows (256
     * consecutive cells of a plane, wrapping from row to row); LBM_TILES_RECTANGULAR never
     * packs.  The tiles decide only which thread updates which cell: results are bitwise the
     * same. */
    int tiles;
    /* Kernels of a two-pass step.  LBM_PASSES_FUSED corrects the velocity inside the
     * collision pass (two kernels per step, the corrected velocities shared through LDS)
     * where the run allows it: D3Q27, no solid cells, no wet-node boundaries, no Picard
     * iterations, no analytic porosity derivatives, nx a multiple of 64 and ny of 8 (4 for FP64
     * storage); LBM_PASSES_AUTO does so where, in addition, the grid is
     * large enough for z-chunks of at least 16 planes (about 2^21 cells); every other run, and
     * LBM_PASSES_SEPARATE, uses the separate correction pass.  All give bitwise the same
     * results. */
    int passes;
} lbm_params;

/* Global statistics of the current state, accumulated in FP64 on the device. */
typedef struct lbm_stats {
    double mass;          /* sum over fluid cells of sum_i f-bar_i (= sum eps rho) */
    double momentum[3];   /* sum over fluid cells of rho v */
    double vmax;          /* max |v| over fluid cells */
    double dv2;           /* sum |v - v_prev|^2, v_prev = v at the previous lbm_residual call */
    double v2;            /* sum |v_prev|^2 */
    double residual;      /* sqrt(dv2 / v2): the relative L2 change of v (Sec. 4.2's steady-state
                             measure, taken between consecutive lbm_residual calls); +inf when
                             v2 = 0 */
    int64_t nonfinite;    /* number of fluid cells whose populations or velocity are not finite */
    int64_t step;         /* time steps taken since creation */
} lbm_stats;

typedef struct lbm_solver lbm_solver;

/*
 * Bytes of device workspace lbm_create needs for these parameters (pure host computation, no
 * device work).  Only lattice, storage, scheme, shift, nx, ny, nz, whether mask is non-NULL and
 * the number of boundary nodes in bc_type are read.
 * Errors: LBM_ERR_INVALID_ARG for NULL pointers or bad lattice, storage or dimensions.
 */
LBM_API int lbm_footprint(const lbm_params *p, size_t *workspace_bytes);

/*
 * Validate the run, carve the caller-owned device workspace (>= lbm_footprint bytes,
 * 256-byte aligned) into populations, static fields and moment buffers, upload and precompute
 * the per-cell coefficients (mu_D, mu_F, nu_eff, beta from eqs. mu_D_Ergun_perm,
 * mu_F_Ergun_perm, nu_eff_def) and write the initial populations of eq. (eq_bc_f_bar) with
 * a_0, Phi^ext_0, Phi^eta_0 from the initial fields (the flowchart's initialisation).
 * hip_stream is a hipStream_t (NULL = the null stream); the workspace and the stream are
 * borrowed for the handle's lifetime.  Synchronises the stream before returning.
 * Errors: LBM_ERR_INVALID_ARG (field values out of range, dimensions, pointers),
 * LBM_ERR_UNSUPPORTED, LBM_ERR_WORKSPACE, LBM_ERR_HIP.  On error *out is NULL.
 */
LBM_API int lbm_create(const lbm_params *p, void *dev_workspace, size_t workspace_bytes,
                       void *hip_stream, lbm_solver **out);

/*
 * Enqueue n >= 0 time steps (Sec. 3.5, collide-and-stream loop).  A two-pass step runs the
 * moment pass (eqs. transformed_density_moment, transformed_momentum_moment, v_(0), v_(1)), the
 * velocity correction (eq. v_final) and the fused forcing-collide-stream pass (eqs. accel,
 * ex_corr, eta_corr, prod_form, dicrete_scheme) with halfway bounce-back and periodic wrap; a
 * lagged step runs all of it in one kernel (LBM_SCHEME_LAGGED).
 * Asynchronous; kernel faults surface at the next synchronising call.
 */
LBM_API int lbm_step(lbm_solver *h, int64_t n);

/*
 * As lbm_step, and also measures each kernel class with HIP events on the handle's stream;
 * synchronises.  kernel_ms[0..2] receive the summed durations (ms) of the moment, velocity
 * correction and collide-stream kernels over the n steps (lagged steps count their single
 * kernel under collide-stream; a two-pass step whose correction runs inside the collision pass,
 * see lbm_params.passes, reports 0 for the correction and the fused kernel under
 * collide-stream).
 */
LBM_API int lbm_step_timed(lbm_solver *h, int64_t n, double kernel_ms[3]);

/*
 * Write the macroscopic fields of the current state: intrinsic density rho [N] and the
 * corrected velocity [D][N] (eqs. v_(0), v_(1), v_final), superficial v or intrinsic u = v/eps
 * per velocity_kind, as LBM_DTYPE_F64 or LBM_DTYPE_F32 into caller device buffers (either
 * pointer may be NULL).  Solid cells get 0.  Under LBM_SCHEME_LAGGED the correction takes its
 * neighbour values from the previous step, as the next step will.  Asynchronous.
 */
LBM_API int lbm_moments(lbm_solver *h, void *rho_dev, void *v_dev, int dtype, int velocity_kind);

/*
 * Compute the global statistics of the current state (lbm_stats) with deterministic FP64
 * reductions on the device, copy them to *out and remember the current v for the next call.
 * Synchronises.  Returns LBM_ERR_NONFINITE (with *out filled) if any fluid cell is not finite.
 */
LBM_API int lbm_residual(lbm_solver *h, lbm_stats *out);

/*
 * Statistics for callers that cannot allocate device memory or synchronise: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The same statistics as
 * lbm_residual (same kernels, same order of summation, so the values are bitwise those of
 * lbm_residual on the same state), enqueued on the handle's stream without synchronising:
 * stats_dev (device memory on the handle's device, caller-owned) receives 8 doubles in the
 * slot order mass, momentum x, y, z, max|v|, sum |v - v_prev|^2, sum |v_prev|^2, number of
 * non-finite fluid cells (the residual is sqrt(slot 5 / slot 6)); the current v becomes v_prev
 * of the next statistics call, as in lbm_residual.  No device memory is allocated: the
 * per-block partial sums go to a file-scope device array of the library (at most 1024 rows of 8
 * doubles, 64 KiB per device, kept until the process ends), whose address is looked up once per
 * device on the first call there.  Every call on a GPU shares that GPU's array, so calls that
 * overlap on one GPU (other streams, other threads) race; nothing in it needs clearing.
 * Errors: LBM_ERR_INVALID_ARG (NULL pointer), LBM_ERR_UNSUPPORTED (a device index above 63),
 * LBM_ERR_HIP; a non-finite state is reported in slot 7, not as an error.
 */
LBM_API int lbm_stats_noalloc(lbm_solver *h, double *stats_dev);

/*
 * Copy the populations f-bar_i(x) of the current state in natural layout [Q][N] (the value
 * that streamed into cell x along c_i) into a caller device buffer of dtype.  Solid cells get
 * 0; the incoming populations of outflow nodes are their zero-gradient copies.  With
 * lbm_set_populations this is the checkpoint of the state.  Asynchronous.
 */
LBM_API int lbm_get_populations(lbm_solver *h, void *dev_out, int dtype);

/*
 * Replace the state by populations in natural layout [Q][N] from a caller device buffer of
 * dtype and set the step counter to step.  Asynchronous.
 */
LBM_API int lbm_set_populations(lbm_solver *h, const void *dev_in, int dtype, int64_t step);

/* Time steps taken so far. */
LBM_API int lbm_get_step(const lbm_solver *h, int64_t *step);

/*
 * The library's lattice numbering: c_out receives Q*3 integers (c_ix, c_iy, c_iz), opp_out Q
 * opposite indices.  D2Q9 follows the paper's wall example (Sec. 3.4.1): 0 rest, 1 +x, 2 +y,
 * 3 -x, 4 -y, 5 (+,+), 6 (-,+), 7 (-,-), 8 (+,-).  D3Q27: rest, the six faces, twelve edges,
 * eight corners, opposite pairs adjacent.  Returns Q, or LBM_ERR_INVALID_ARG.
 */
LBM_API int lbm_lattice_info(int lattice, int *c_out, int *opp_out);

/* ------------------------------------------------------------------------------------------
 * Request server: continuous batching of many independent runs on one GPU.
 *
 * Requests (each an lbm_params run with a steady-state tolerance) queue on submission and are
 * admitted in arrival order as memory of the caller's device pool frees up: a request whose
 * workspace (lbm_footprint) does not fit lets later, smaller ones pass (backfill) until it has
 * waited 64 rounds, after which admission waits for it.  Admitted requests keep their
 * populations resident and advance together in rounds of check_every steps: every pass of a
 * round is one kernel launch over the tiles of all active runs that share a lattice, storage,
 * solids flag, scheme and AA phase (kernel boundaries are the per-request step barriers), so
 * small runs fill the GPU together.  After each round the server takes each run's statistics
 * (lbm_residual's FP64 reductions) and retires runs whose relative L2 change of v over the
 * round fell below tol (converged), whose residual stopped falling (at the rounding floor of
 * their storage, when the caller asks for that rule), that reached max_steps (censored) or that
 * hold non-finite values (failed).  Each run's arithmetic is that of lbm_step, so its result is bitwise the same
 * alone and in any mix.  All work is enqueued on the server's stream; progress synchronises it
 * once per round.  A server handle must not be used from two threads at once.
 * ------------------------------------------------------------------------------------------ */
typedef struct lbm_server lbm_server;

#define LBM_REQ_QUEUED 0
#define LBM_REQ_ACTIVE 1
#define LBM_REQ_CONVERGED 2
#define LBM_REQ_CENSORED 3   /* reached max_steps before tol */
#define LBM_REQ_FAILED 4     /* creation failed or the state became non-finite */
#define LBM_REQ_FLOOR 5      /* the residual stopped falling above tol (see lbm_server_submit) */

typedef struct lbm_request_info {
    int64_t id;
    int state;               /* LBM_REQ_* */
    int64_t steps;           /* time steps taken */
    double residual;         /* relative L2 change of v over the last round (+inf before two) */
    double t_submit;         /* seconds since lbm_server_create (steady clock) */
    double t_admit;          /* -1 until admitted */
    double t_done;           /* -1 until converged, censored or failed */
    int64_t cells;           /* nx * ny * nz */
    size_t workspace_bytes;  /* lbm_footprint of the run */
} lbm_request_info;

typedef struct lbm_server_stats {
    int64_t rounds;          /* rounds run */
    int64_t submitted, admitted, finished;
    int64_t queued, active;  /* now */
    double cell_updates;     /* sum over admitted runs of cells x steps */
    size_t pool_bytes;       /* size of the device pool */
    size_t pool_used;        /* bytes held by admitted, unreleased runs */
    size_t pool_peak;        /* maximum of pool_used */
} lbm_server_stats;

/*
 * Create a server on the caller's device pool (>= 1 MiB, 256-byte aligned; borrowed until
 * lbm_server_destroy) and stream.  check_every >= 2 is the round length in steps (even, so
 * that every run starts each round in the natural AA layout); max_active caps the number of
 * resident runs (0: only memory and the limit of 4096 bound it).
 * Errors: LBM_ERR_INVALID_ARG, LBM_ERR_WORKSPACE.
 */
LBM_API int lbm_server_create(void *dev_pool, size_t pool_bytes, int64_t check_every,
                              int max_active, void *hip_stream, lbm_server **out);

/*
 * Queue a run.  The params and every host array they point to are copied, so the caller may
 * free them on return.  tol > 0 is the steady-state threshold on the relative L2 change of v
 * over one round (Sec. 4.2's measure, eq. SS_convergence_L2, taken over check_every steps);
 * max_steps >= check_every caps the run.  floor_checks > 0 adds a retirement rule for storage
 * whose rounding keeps the residual above tol: the state keeps changing by rounding noise
 * about the steady state, so the residual stops falling at a floor set by the precision (FP32
 * and the 16-bit forms stay far above 1e-7); a run whose residual has made no new minimum (1 %
 * below the previous one) for floor_checks rounds retires as LBM_REQ_FLOOR with its residual
 * reported.  0 leaves the rule off.  *id receives the request id (ids count from 0 in
 * submission order).  Runs with wet-node boundaries (bc_type), Picard iterations or analytic
 * porosity derivatives are served too, each stepped with its own launches (as lbm_step) in
 * every round instead of sharing the batched ones.  Errors: those of lbm_footprint,
 * LBM_ERR_INVALID_ARG, LBM_ERR_WORKSPACE (the run can never fit in the pool).
 */
LBM_API int lbm_server_submit(lbm_server *s, const lbm_params *p, double tol, int64_t max_steps,
                              int floor_checks, int64_t *id);

/*
 * Run up to max_rounds rounds (admission, check_every steps of every active run, statistics,
 * retirement); returns early when nothing is active or queued.  The ids of runs that finished
 * during the call are written to finished_ids (room for max_finished; more are still counted
 * in *n_finished, which may be NULL).  Synchronises the stream.
 */
LBM_API int lbm_server_progress(lbm_server *s, int64_t max_rounds, int64_t *finished_ids,
                                int max_finished, int *n_finished);

/* Current state of a request. */
LBM_API int lbm_server_info(const lbm_server *s, int64_t id, lbm_request_info *out);

/*
 * Solver handle of an active or finished, unreleased request, for lbm_moments,
 * lbm_get_populations and lbm_residual on the server's stream.  Valid until the request is
 * released; stepping it directly is not allowed.
 */
LBM_API int lbm_server_solver(lbm_server *s, int64_t id, lbm_solver **out);

/* Release a finished request's workspace back to the pool (its info stays available). */
LBM_API int lbm_server_release(lbm_server *s, int64_t id);

LBM_API int lbm_server_get_stats(const lbm_server *s, lbm_server_stats *out);

/* Destroy the server (NULL is a no-op); the pool and the stream remain the caller's. */
LBM_API int lbm_server_destroy(lbm_server *s);

/* Release the host-side handle (NULL is a no-op).  The workspace remains the caller's. */
LBM_API int lbm_destroy(lbm_solver *h);

/* Description of the calling thread's last error ("" if none); valid until the next call. */
LBM_API const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
