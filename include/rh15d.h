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
enum { RH15D_START_LTE = 0, RH15D_START_ZERO_RADIATION = 1, RH15D_START_PROVIDED = 2 };
enum { RH15D_SCHED_CHUNKED = 0, RH15D_SCHED_SLOTS = 1 };

/* Per-column status codes written to rh15d_outputs.status. */
enum {
    RH15D_CONVERGED = 0,    /* max relative change fell below tol */
    RH15D_MAX_ITER = 1,     /* iteration limit reached */
    RH15D_NONFINITE = 2,    /* a population became non-finite or non-positive */
    RH15D_SINGULAR = 3      /* a rate matrix had a zero pivot */
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
    const double *v_turb;         /* DEVICE [total_depth] microturbulence, m/s */
    const double *init_pops;      /* DEVICE [total_depth][n_levels] start populations
                                     (read only when start = RH15D_START_PROVIDED) */
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
} rh15d_options;

/* Measurements of the calling thread's last rh15d_solve_columns made with
 * options.profile = 1 (all zero otherwise).  Times come from HIP events
 * recorded on the caller's stream around the library's own launches. */
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
} rh15d_outputs;

/* Fill *opt with the defaults: FP64, 5 angles, tol 1e-4, 200 iterations,
 * Ng order 2 / delay 5 / period 4, LTE start, coll_scale 1, chunked,
 * no profiling, automatic sweep shape. */
int rh15d_default_options(rh15d_options *opt);

/* Device workspace needed by rh15d_solve_columns for these columns and
 * options, in bytes (HOST *bytes). */
int rh15d_workspace_size(const rh15d_atom *atom, const rh15d_columns *cols,
                         const rh15d_options *opt, size_t *bytes);

/* Solve every column to convergence (or its iteration limit), in order:
 * column preparation (LTE populations, collisions, background, normalised
 * line profiles), start populations, then per iteration the formal
 * solution of every (wavelength, angle, direction) ray with the diagonal
 * Psi* and the preconditioned rate accumulation, the statistical-
 * equilibrium solve per depth, the convergence test and Ng; finally the
 * vertical emergent spectrum and Psi*.  Work is enqueued on hip_stream
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

/* Text of the calling thread's last failure ("" if none). */
const char *rh15d_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RH15D_H */
