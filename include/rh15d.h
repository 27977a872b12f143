/*
 * rh15d.h - C ABI of the MI355X per-column MALI library (librh15d.so).
 *
 * The method (paper Sec. 2.1): multi-level accelerated Lambda iteration in
 * the Rybicki & Hummer (1992) formalism with a local (diagonal) approximate
 * Psi operator, preconditioned rate equations and overlapping transitions,
 * solved independently for every atmosphere column (Sec. 2.2, the 1.5D
 * approach), with Ng acceleration, a choice of start solutions and a
 * per-column convergence test on the maximum relative population change
 * (Sec. 2.3).  The only emergent spectra are the vertical ones (Sec. 2.2).
 *
 * Conventions
 *   - SI units throughout; wavelengths in metres.
 *   - Every call returns int: RH15D_OK (0) or a negative error code; the
 *     text of the last failure of the calling thread is rh15d_last_error().
 *     Nothing aborts the process.  Non-convergence of a column is not an
 *     error: it is that column's status.
 *   - Device pointers are HIP device pointers on the current device;
 *     host pointers are marked HOST.  The caller owns every buffer it
 *     passes; the library owns only the atom handle.
 *   - Columns are ragged: column c spans depth rows
 *     depth_offset[c] .. depth_offset[c+1]-1 of every per-depth array,
 *     ordered from the top (largest z) down.
 */
#ifndef RH15D_H
#define RH15D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RH15D_OK = 0,
    RH15D_EINVAL = -1,   /* bad argument: null pointer, bad size, bad option */
    RH15D_EIO = -2,      /* atom file missing or malformed */
    RH15D_ENOMEM = -3,   /* workspace too small or device allocation failed */
    RH15D_EDEVICE = -4   /* HIP runtime error */
};

enum { RH15D_FP64 = 0, RH15D_FP32 = 1 };
enum { RH15D_START_LTE = 0, RH15D_START_ZERO_RADIATION = 1, RH15D_START_PROVIDED = 2, RH15D_START_ESCAPE = 3 };
enum { RH15D_SCHED_CHUNKED = 0, RH15D_SCHED_SLOTS = 1 };

/* Per-column status codes written to rh15d_outputs.status. */
enum {
    RH15D_CONVERGED = 0,    /* max relative change fell below tol */
    RH15D_MAX_ITER = 1,     /* iteration limit reached */
    RH15D_NONFINITE = 2,    /* a population became non-finite or non-positive */
    RH15D_SINGULAR = 3,     /* a rate matrix had a zero pivot */
    RH15D_BAD_INPUT = 4     /* the column's data cannot be used (a non-finite or
                               non-positive T, n_e or n_H, a non-finite velocity,
                               a negative microturbulence, or z not strictly
                               decreasing): no iteration, n_iter = 0, its
                               populations, history, spectrum and Psi* are NaN;
                               the other columns are unaffected (Sec. 2.2: a
                               problematic column is dealt with on its own) */
};

#define RH15D_MAX_LEVELS 8
#define RH15D_MAX_MU 16
#define RH15D_MAX_DEPTH 1024

typedef struct rh15d_atom rh15d_atom;

typedef struct {
    int n_levels;        /* L, the last level may be a continuum (higher stage) */
    int n_lines;
    int n_continua;
    int n_transitions;   /* lines first, then continua */
    int n_lambda;        /* size of the union wavelength grid */
} rh15d_atom_info;

/* Load a model atom in the project's text format (see the atom-file
 * description in the package's synthetic-input module).  Builds the union
 * wavelength grid of all transitions (sorted, exact duplicates merged),
 * each transition's active wavelengths and trapezoid frequency weights,
 * and the Einstein coefficients from the oscillator strengths.  Overlapping
 * transitions (Sec. 2.1) are found here.  *out receives a handle owned by
 * the library (free with rh15d_free_atom); it is immutable and may be
 * shared by threads and streams.  Returns RH15D_EIO for a missing or
 * malformed file, RH15D_EINVAL for more than RH15D_MAX_LEVELS levels. */
int rh15d_load_atom(const char *path, rh15d_atom **out);
void rh15d_free_atom(rh15d_atom *atom);
int rh15d_atom_get_info(const rh15d_atom *atom, rh15d_atom_info *info);
/* Copy the union wavelength grid (HOST, n_lambda doubles, metres). */
int rh15d_atom_lambda(const rh15d_atom *atom, double *lambda_host);

typedef struct {
    int64_t n_columns;
    const int64_t *depth_offset;  /* HOST [n_columns+1], offset[0] = 0,
                                     2 <= N_d <= RH15D_MAX_DEPTH per column */
    const double *z;              /* DEVICE [total_depth] height, m, strictly
                                     decreasing within a column */
    const double *T;              /* DEVICE [total_depth] temperature, K, > 0 */
    const double *n_e;            /* DEVICE [total_depth] electron density, m^-3, > 0 */
    const double *n_H;            /* DEVICE [total_depth] hydrogen density, m^-3, > 0 */
    const double *v_z;            /* DEVICE [total_depth] vertical velocity, m/s,
                                     positive upward (towards an observer at mu = 1) */
    const double *v_turb;         /* DEVICE [total_depth] microturbulence, m/s, >= 0
                                     (the device values are checked per column on
                                     the device: a column that breaks one of these
                                     conditions gets status RH15D_BAD_INPUT) */
    const double *init_pops;      /* DEVICE [total_depth][n_levels] start populations
                                     (read only when start = RH15D_START_PROVIDED) */
    /* Magnetic field, read only for the Stokes spectrum (rh15d_outputs.stokes):
       all three NULL (no field) or all three DEVICE [total_depth]; a column
       with a non-finite value gets a NaN Stokes spectrum. */
    const double *B;              /* field strength, T */
    const double *B_incl;         /* inclination to the vertical (the line of sight), rad */
    const double *B_azim;         /* azimuth of the field's horizontal part, rad (the reference
                                     direction of Stokes Q is azimuth 0) */
} rh15d_columns;

typedef struct {
    int precision;      /* RH15D_FP64: everything in FP64.  RH15D_FP32: formal
                           solution and rate accumulation in FP32; rate
                           matrices, Ng and the convergence test in FP64 */
    int n_mu;           /* Gauss-Legendre angles on (0,1), 1..RH15D_MAX_MU */
    double tol;         /* converged when max_{i,k} |n_new - n_old| / n_new < tol */
    int max_iter;       /* iteration limit, >= 0 */
    int ng_order;       /* 0 (off) or 2 */
    int ng_delay;       /* first iteration whose solution enters Ng's history */
    int ng_period;      /* iterates collected between Ng attempts (>= ng_order+2) */
    int start;          /* RH15D_START_* (Sec. 2.3, starting solutions) */
    double coll_scale;  /* constant multiplier of collision rates (1 = physical;
                           Sec. 2.3, collisional-radiative switching) */
    int scheduler;      /* RH15D_SCHED_CHUNKED: fixed chunks of columns iterated
                           together; RH15D_SCHED_SLOTS: resident slots, converged
                           columns retired and refilled */
    int batch_columns;  /* columns resident at once; 0 = automatic */
    int profile;        /* 1: time the kernels with HIP events and count the
                           algorithmic work (see rh15d_last_stats) */
    int sweep_mc;       /* angles carried by one lane of the formal-solution
                           kernel: 1, 3 or 5 dividing n_mu; 0 = automatic */
    int sweep_pack;     /* wavelengths per wavefront: 1 = one set of active
                           transitions per wavefront, 2 = mixed sets;
                           0 = automatic */
    double crs_f0;      /* collisional-radiative switching (Sec. 2.3,
                           Hummer & Voels 1988): the collision rates of
                           iteration it (1, 2, ...) are multiplied by
                           crs_f0 / 10^(it-1) while that exceeds 1, formed
                           by repeated division by 10; no column converges
                           and no iterate enters Ng's history while the
                           factor exceeds 1.  <= 1 (default 1): off */
    double tol_fp;      /* > 0: a column converges only when, besides the change
                           test of tol, the distance to the fixed point that its
                           last two changes imply is below tol_fp: with
                           r = Delta_k / Delta_{k-1} < 1 the remainder of a
                           linear iteration Delta_k r / (1 - r), tested as
                           Delta_k^2 < tol_fp (Delta_{k-1} - Delta_k).  There is
                           no ratio at the first iteration or after an applied
                           Ng extrapolation (then only Delta_k = 0 passes).
                           0 (default): the change test alone (Sec. 2.3) */
    int esc_iter;       /* RH15D_START_ESCAPE: statistical-equilibrium iterations
                           from LTE with the spontaneous rate of every transition
                           times the escape probability (1 - e^-tau)/tau of its
                           vertical optical depth tau from the top at the line
                           centre (rest frame) or continuum edge, no other
                           radiative rates (Sec. 2.3, starting solutions);
                           0..100, default 3 */
    int prd;            /* 1: lines the atom marks PRD emit with the angle-averaged
                           partial-redistribution profile psi = rho phi
                           (Sec. 2.1; rho from the angle-averaged R_II of
                           Hummer 1962 after every iteration, see
                           rh15d_solve_columns); 0 (default): every line in
                           complete redistribution.  Forces one angle per lane
                           (sweep_mc must be 0 or 1) */
    double prd_eps0;    /* PRD switching (Sec. 2.3, Eq. 1): the rho update after
                           iteration n is rho eps + (1 - eps), eps = min(1,
                           prd_eps0 n^2); <= 0 (default): off */
} rh15d_options;

/* Measurements of the calling thread's last rh15d_solve_columns.  The
 * times and work counts are filled with options.profile = 1 (zero
 * otherwise); they come from HIP events recorded on the caller's stream
 * around the library's own launches.  graph_launches is filled on every
 * call. */
typedef struct {
    int64_t sweep_launches;     /* formal-solution launches (rate mode) */
    double sweep_ms;            /* their summed duration */
    double se_ms, converge_ms;  /* rate-equation solves; convergence test + Ng */
    double prep_ms;             /* column preparation (start populations included) */
    double final_ms;            /* emergent spectrum and Psi* */
    double total_ms;            /* first to last event of the call */
    int64_t column_iterations;  /* sum over columns of the iterations performed */
    int64_t ray_steps;          /* formal-solution ray-steps of the rate launches */
    double sweep_flops;         /* algorithmic flops of the rate launches */
    double sweep_bytes;         /* algorithmic HBM bytes of the rate launches */
    int64_t graph_launches;     /* iterations replayed as a captured HIP graph
                                   (slot scheduler on a non-default stream with
                                   profile = 0); 0 when every iteration was
                                   launched kernel by kernel */
} rh15d_stats;

int rh15d_last_stats(rh15d_stats *stats);

typedef struct {
    double *pops;       /* DEVICE [total_depth][n_levels] final populations, m^-3 */
    double *history;    /* DEVICE [n_columns][max_iter] max relative change per
                           iteration, NaN after the last one; may be NULL */
    int32_t *n_iter;    /* DEVICE [n_columns] iterations performed */
    int32_t *status;    /* DEVICE [n_columns] RH15D_CONVERGED, ... */
    double *spectrum;   /* DEVICE [n_columns][n_lambda] emergent vertical intensity
                           at the top, W m^-2 Hz^-1 sr^-1; may be NULL */
    double *psi_star;   /* DEVICE [total_depth][n_transitions] Psi* = Lambda* over chi of the
                           final populations averaged over each transition's rays
                           (weights W phi for lines, W / sum W for continua), m;
                           may be NULL */
    double *stokes;     /* DEVICE [n_columns][n_lambda][4] emergent vertical Stokes vector
                           (I, Q, U, V) at the top, W m^-2 Hz^-1 sr^-1, with the
                           Zeeman effect of the columns' magnetic field; may be NULL.
                           Sec. 2.1 (the full Stokes vector from Zeeman splitting).
                           Populations are unpolarised: the field enters only this
                           final formal solution, computed in FP64 in both
                           precisions from the final populations (and the final
                           rho of PRD lines).  Lines whose two levels the atom file
                           gives J and a Lande factor (section ZEEMAN) are split
                           into their anomalous Zeeman pattern (components of
                           strength normalised per q = M_l - M_u, shifted by
                           (g_u M_u - g_l M_l) e B / (4 pi m_e)); each contributes
                           the absorption matrix
                             eta_I = [phi_0 sin^2 t + (phi_+1 + phi_-1)(1 + cos^2 t)/2]/2,
                             eta_Q, eta_U = [phi_0 - (phi_+1 + phi_-1)/2] sin^2 t (cos, sin)(2 a)/2,
                             eta_V = (phi_+1 - phi_-1) cos t / 2,
                           rho_Q, rho_U, rho_V alike from the dispersion profiles
                           (phi + i psi = w(v + i a) / sqrt(pi), w the Faddeeva
                           function), times the line's scalar absorption
                           coefficient, and the emission vector of the same
                           combinations times its emission coefficient (t the
                           inclination, a the azimuth); other transitions and the
                           background are unpolarised.  The transfer equation is
                           integrated upward with DELO and a linear effective
                           source function (Rees, Durrant & Murphy 1989) on the
                           depth points; the bottom enters as (B_nu + dB_nu/dtau,
                           0, 0, 0).  With no field it equals (spectrum, 0, 0, 0). */
    double *psi_ray;    /* DEVICE [total_depth][n_lambda][n_mu][2] Psi* = Lambda* / chi of every
                           ray of the final formal solution (the diagonal of the local
                           approximate operator, Sec. 2.1), per depth point, wavelength,
                           angle and direction (0 downward, 1 upward), m; 0 at a ray's
                           boundary point and where no transition is active at the
                           wavelength; NaN for a column with status RH15D_BAD_INPUT.
                           8 n_lambda n_mu 2 bytes per depth point: for small problems
                           (tests, single columns); may be NULL */
} rh15d_outputs;

/* Fill *opt with the defaults: FP64, 5 angles, tol 1e-4, tol_fp 0, 200
 * iterations, Ng order 2 / delay 5 / period 4, LTE start (esc_iter 3),
 * coll_scale 1, crs_f0 1, chunked, no profiling, automatic sweep shape,
 * complete redistribution (prd 0, prd_eps0 0). */
int rh15d_default_options(rh15d_options *opt);

/* Device workspace needed by rh15d_solve_columns for these columns and
 * options, in bytes (HOST *bytes).  The size depends on the sweep shape
 * (its number of rate sums): with sweep_mc = sweep_pack = 0 it follows the
 * shape rh15d_autotune has chosen for this device, so query it after
 * tuning. */
int rh15d_workspace_size(const rh15d_atom *atom, const rh15d_columns *cols,
                         const rh15d_options *opt, size_t *bytes);

/* Solve every column to convergence (or its iteration limit), in order:
 * column preparation (LTE populations, collisions, background, normalised
 * line profiles), start populations, then per iteration the formal
 * solution of every (wavelength, angle, direction) ray with the diagonal
 * Psi* and the preconditioned rate accumulation, the statistical-
 * equilibrium solve per depth, the convergence test and Ng; finally the
 * vertical emergent spectrum and Psi*.  With options.prd, after the
 * convergence test of every iteration each PRD line's
 * rho(j) = 1 + gamma n_l B_lu / (n_u P_u) [sum_j' g(j, j') J(j') - Jbar]
 * is recomputed from that iteration's intensities and the new populations
 * (J the angle-averaged, Jbar the profile-weighted mean intensity, P_u the
 * total rate out of the upper level, gamma = P_u / (P_u + c_el n_H) the
 * coherent fraction, g the redistribution weights of the angle-averaged
 * R_II normalised per output frequency), switched (prd_eps0) and
 * normalised so that the emission profile integrates to 1; the next
 * formal solution and the emergent spectrum use psi = rho phi for
 * spontaneous and stimulated emission (Uitenbroek 2001, angle-averaged
 * PRD; a reading of its discretisation).  Work is enqueued on hip_stream
 * (NULL = the default stream); the call returns after the iteration loop
 * has finished on the device (it reads a done-counter back each iteration),
 * and all outputs are valid once the stream is synchronised.  workspace is
 * a DEVICE buffer of at least rh15d_workspace_size bytes (caller-owned,
 * 256-byte aligned); if NULL the library allocates and frees its own.
 * Errors: RH15D_EINVAL for a bad argument (checked before any launch),
 * RH15D_ENOMEM if workspace_bytes is too small, RH15D_EDEVICE on a HIP
 * error. */
int rh15d_solve_columns(const rh15d_atom *atom, const rh15d_columns *cols,
                        const rh15d_options *opt, const rh15d_outputs *out,
                        void *workspace, size_t workspace_bytes, void *hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): rh15d_solve_columns with
 * its workspace in a fixed device region of the library,
 * rh15d_static_workspace_bytes() bytes (64 MiB) per device, held from the
 * library's load until the process ends.  Arguments, outputs, per-column
 * statuses and results are those of rh15d_solve_columns with workspace =
 * NULL; results are bit for bit the same.  The call allocates nothing: no
 * device, pinned-host or graph memory, no streams or events (the sweep's
 * kernel classes run one after another on hip_stream; iterations are not
 * captured as a graph).  It reads the done-counter back into a host buffer
 * of the calling thread.  Requirements: the atom's device tables for this
 * device, options.n_mu and sweep shape exist (any earlier
 * rh15d_solve_columns or rh15d_workspace_size of the atom with the same
 * options built them), else
 * RH15D_EINVAL; options.profile = 0, else RH15D_EINVAL; as many columns
 * stay resident as the region holds (options.batch_columns, if set, must
 * fit), and if not even one column and the depth offsets fit, RH15D_ENOMEM
 * with the size needed.  Every call on a device uses the same region: the
 * solve clears what it needs at its start (nothing carries over between
 * calls), and calls that overlap on one device race. */
size_t rh15d_static_workspace_bytes(void);
int rh15d_solve_columns_static(const rh15d_atom *atom, const rh15d_columns *cols, const rh15d_options *opt,
                               const rh15d_outputs *out, void *hip_stream);

/* ------------------------------------------------------------------------
 * Grid optimisation (Sec. 2.3, "Grid optimisation"): every column is
 * re-interpolated onto a new depth grid that puts more points where
 * temperature, vertical velocity or optical depth change fast; each column
 * gets its own grid and may get its own number of points.  The paper gives
 * no formula; this reading gives the interval between input points k-1
 * and k the length
 *   d_k = sqrt((w_z dz_k / H)^2 + (w_T d ln T_k)^2 + (w_v dv_z,k)^2
 *              + (w_tau d ln(tau_k + 1e-5))^2),
 * H the column's height range and tau the optical depth from the top in
 * the atom's background law at its reference wavelength (trapezoid rule in
 * z; zero if the atom has no background), and spreads the new points at
 * equal steps of the summed length.  The first and last input points are
 * kept exactly; inside an interval z, v_z and v_turb are interpolated
 * linearly in the length, T, n_e and n_H linearly in their logarithms.
 * ------------------------------------------------------------------------ */
#define RH15D_GRID_MAX_INPUT 8192
typedef struct {
    double w_z;     /* weight of the height step, in units of the column's height range */
    double w_T;     /* weight of the step in ln T */
    double w_v;     /* weight of the step in v_z, s/m */
    double w_tau;   /* weight of the step in ln(tau + 1e-5) */
} rh15d_grid_options;

typedef struct {
    const int64_t *depth_offset;  /* HOST [n_columns+1] rows of each new column, offset[0] = 0,
                                     2..RH15D_MAX_DEPTH rows per column */
    double *z, *T, *n_e, *n_H, *v_z, *v_turb;  /* DEVICE [offset[n_columns]] the new columns, top down */
    int32_t *status;              /* DEVICE [n_columns] 0, or RH15D_BAD_INPUT for a column with fewer
                                     than 2 points, a non-finite value, a non-positive T, n_e or n_H,
                                     z not strictly decreasing, or zero summed length; its new
                                     values are NaN */
} rh15d_grid_output;

/* Defaults: w_z = 1, w_T = 2, w_v = 2e-4 s/m (5 km/s weigh as much as the
 * height range), w_tau = 0.2. */
int rh15d_default_grid_options(rh15d_grid_options *opt);

/* Re-grid the columns in (init_pops and the magnetic field are ignored: a
 * caller with a field interpolates it onto the new heights itself; input
 * columns may have up to RH15D_GRID_MAX_INPUT points) into out.  Output buffers are caller-owned
 * and must not overlap the input.  The depth offsets are uploaded before
 * the call returns (the call waits for work queued earlier on hip_stream);
 * the re-gridding itself is asynchronous on hip_stream.  Errors:
 * RH15D_EINVAL for a null pointer, a weight that is negative or not finite,
 * all weights zero, or a column count outside the limits (checked before
 * any launch); RH15D_EDEVICE on a HIP error. */
int rh15d_optimize_grid(const rh15d_atom *atom, const rh15d_columns *in, const rh15d_grid_options *opt,
                        const rh15d_grid_output *out, void *hip_stream);

/* Autotuner of the formal-solution kernel's shape.  Columns are
 * independent, so a pool of workers can take them in any grouping (Sec. 3.1,
 * pool mode); on the GPU the grouping of rays into wavefronts is free too.
 * For every candidate shape (sweep_mc in {1, 3, 5} dividing n_mu, times
 * sweep_pack in {1, 2}) this solves the given columns twice with the other
 * options of opt (the second solve timed with HIP events on hip_stream)
 * and keeps the fastest for this device, opt->n_mu and opt->precision:
 * later solves of the atom with sweep_mc = sweep_pack = 0 use it.  Results
 * do not depend on the shape beyond the order of floating-point sums.
 * Allocates its own device buffers and synchronises the stream; the
 * columns should be a representative sample (a few thousand columns). */
#define RH15D_TUNE_MAX 6
typedef struct {
    int sweep_mc, sweep_pack;                       /* the chosen shape */
    int n_candidates;
    int cand_mc[RH15D_TUNE_MAX], cand_pack[RH15D_TUNE_MAX];
    double ms[RH15D_TUNE_MAX];                      /* timed solve of each candidate */
} rh15d_tune_result;

int rh15d_autotune(rh15d_atom *atom, const rh15d_columns *cols, const rh15d_options *opt, void *hip_stream,
                   rh15d_tune_result *result);

/* ------------------------------------------------------------------------
 * Learned start solution.  The start populations decide how many MALI
 * iterations a column needs (Sec. 2.3, "Different starting solutions").
 * A small network predicts each depth point's natural-log departure
 * coefficients ln(n_i / n*_i) from the local thermodynamic stencil; the
 * prediction only seeds the iteration (start = RH15D_START_PROVIDED), MALI
 * still decides convergence.  The dense layers run on the matrix cores
 * with BF16 weights and FP32 accumulation (forward activations as two BF16
 * terms, backward operands in BF16); master weights, gradients and Adam
 * moments are kept in FP32 on the device.
 * ------------------------------------------------------------------------ */

/* Departure coefficients ln(n_i / n*_i) of the populations pops (DEVICE
 * [total_depth][n_levels]) against the Saha-Boltzmann populations of the
 * columns' T, n_e, n_H; written to log_b (DEVICE float [total_depth][n_levels]).
 * Asynchronous on hip_stream. */
int rh15d_departures(const rh15d_atom *atom, const rh15d_columns *cols, const double *pops, float *log_b,
                     void *hip_stream);

/* Start populations from departure coefficients: n_i = exp(l_i) n*_i,
 * renormalised to the point's total population (DEVICE in/out as above),
 * where l_i = sign(x) max(|x| - shrink, 0) and x = log_b_i clamped to
 * [-50, 50], or 0 (LTE) if log_b_i is not finite.  shrink >= 0 moves
 * predictions smaller than the network's error toward LTE. */
int rh15d_pops_from_departures(const rh15d_atom *atom, const rh15d_columns *cols, const float *log_b,
                               double shrink, double *pops, void *hip_stream);

typedef struct rh15d_mlp rh15d_mlp;

/* Network of 36 inputs (9-point depth stencil at k + {-128, -32, -8, -2, 0,
 * 2, 8, 32, 128}, clamped at the column ends, of ln T, ln n_e, ln n_H and
 * v_z / 10 km/s, in that order per stencil point), n_layers hidden
 * layers of n_hidden SiLU units and n_out linear outputs.  Weights are
 * He-uniform from a splitmix64 stream seeded by seed, biases zero.  The
 * handle (device buffers on the current device) is owned by the library. */
int rh15d_mlp_create(int n_hidden, int n_layers, int n_out, uint64_t seed, rh15d_mlp **out);
void rh15d_mlp_free(rh15d_mlp *mlp);

/* Parameters as one FP32 vector (HOST): for each layer the weight matrix
 * [fan_in][fan_out] row-major, then its bias [fan_out]. */
int rh15d_mlp_n_params(const rh15d_mlp *mlp, int64_t *n);
int rh15d_mlp_get_params(const rh15d_mlp *mlp, float *host);
int rh15d_mlp_set_params(rh15d_mlp *mlp, const float *host);   /* also resets Adam */
int rh15d_mlp_get_grads(const rh15d_mlp *mlp, float *host);    /* of the last gradient call */

/* Feature scaling (HOST [36] each): inputs enter as (x - mean) / std. */
int rh15d_mlp_get_normalization(const rh15d_mlp *mlp, float *mean, float *std_);
int rh15d_mlp_set_normalization(rh15d_mlp *mlp, const float *mean, const float *std_);
/* Fit the scaling to n raw feature rows (DEVICE float [n][36]); synchronises. */
int rh15d_mlp_fit_normalization(rh15d_mlp *mlp, const float *features, int64_t n, void *hip_stream);

/* Raw features of n sample points given by global depth index (DEVICE
 * int64 [n], or NULL for every point in order) into features (DEVICE float
 * [n][36]).  Asynchronous. */
int rh15d_mlp_features(const rh15d_columns *cols, const int64_t *samples, int64_t n, float *features,
                       void *hip_stream);

/* Outputs (DEVICE float [n][n_out]) of n feature rows.  Asynchronous. */
int rh15d_mlp_forward(rh15d_mlp *mlp, const float *features, int64_t n, float *out, void *hip_stream);

/* Mean squared error against target (DEVICE float [n][n_out]) and its
 * gradient with respect to every parameter (kept in the handle); *loss
 * (HOST, may be NULL) synchronises the stream.  1 <= n <= 262144. */
int rh15d_mlp_gradients(rh15d_mlp *mlp, const float *features, const float *target, int64_t n, float *loss,
                        void *hip_stream);

/* rh15d_mlp_gradients, then one Adam step (beta 0.9 / 0.999, eps 1e-8) with
 * learning rate lr. */
int rh15d_mlp_train_step(rh15d_mlp *mlp, const float *features, const float *target, int64_t n, float lr,
                         float *loss, void *hip_stream);

/* n_batches Adam steps, the same as rh15d_mlp_train_step on rows
 * [b batch, (b + 1) batch) of features (DEVICE float [n_batches batch][36])
 * and target (DEVICE float [n_batches batch][n_out]) with learning rate
 * lr[b] (HOST float [n_batches], >= 0), b = 0 .. n_batches - 1 in order,
 * and bitwise the same parameters.  One step is captured as a HIP graph on
 * a stream of the handle and replayed once per batch (one launch per step
 * instead of one per kernel); the replays are ordered after the work on
 * hip_stream and hip_stream after them.  losses (DEVICE float [n_batches],
 * may be NULL) receives each step's loss.  The captured step is kept for
 * the next call with the same features, target, batch and losses; the
 * call waits for the previous call's replays.  1 <= batch <= 262144. */
int rh15d_mlp_train_batches(rh15d_mlp *mlp, const float *features, const float *target, int64_t batch,
                            int n_batches, const float *lr, float *losses, void *hip_stream);

/* Text of the calling thread's last failure ("" if none). */
const char *rh15d_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RH15D_H */
