/*
 * chhs.h -- C ABI of the MI355X (gfx950) solver for one time step of the
 * second-order convex-splitting scheme for Cahn-Hilliard-Hele-Shaw
 * (Chen, Feng, Liu, Wang, Wise, arXiv 1611.02967).
 *
 * Problem (Section 2, scheme (2.4)-(2.7)): on a cell-centred grid of one
 * spacing h over a box, given (phi^{m-1}, phi^m) find (phi^{m+1}, mu^{m+1/2},
 * p^{m+1/2}) with homogeneous Neumann data (App. A.1, eqn:nbc1-3) such that
 *
 *   phi - s div(M(a) grad mu) - s div(a grad p) = phi^m                        (2.5)
 *   mu - chi(phi, phi^m) + 3/4 eps^2 Lap phi    = -phi_* - 1/4 eps^2 Lap phi^{m-1}   (2.6)
 *   s Lap p + s gamma div(a grad mu)            = 0        (2.7, times s)
 *
 * with phi_* = 3/2 phi^m - 1/2 phi^{m-1}, a = A_h phi_*, M(a) = 1 + gamma a^2,
 * chi(x, y) = (x^2 + y^2)(x + y)/4 (2.4), the operators of App. A.2.  p is
 * fixed to mean zero.  The system is solved by nonlinear multigrid (full
 * approximation scheme, Section 5) with V(nu1, nu2) cycles down to a 2^d
 * coarsest grid until the residual norm is <= tol.
 *
 * Residual norm: ||R|| = (||R_phi||^2 + ||R_mu||^2 + ||R_p||^2)^(1/2) with the
 * discrete l2 norm of App. A.2 (weights h^d), R = f - N(u) for the three rows
 * above (the pressure row as written, i.e. multiplied by s).
 *
 * Layout: every cell-centred field is a dense FP64 array of nx*ny*nz values,
 * x fastest (index (k*ny + j)*nx + i), interior cells only (no ghost layer).
 * Batches of independent instances are packed one after another in instance
 * order.  All field pointers below are DEVICE pointers owned by the caller.
 *
 * Streams: all device work is enqueued on the stream given to chhs_init, or,
 * when that is NULL, on a stream the context creates (with default flags, so
 * that it stays ordered with the legacy null stream, which cannot be captured
 * into a graph).  Calls that return host results synchronise that stream
 * before returning.
 *
 * Errors: every int-returning call returns CHHS_OK (0) or a negative code;
 * no call aborts or throws.  chhs_strerror gives a static message.
 *
 * Thread safety: a context may be used by one host thread at a time.
 */
#ifndef CHHS_H
#define CHHS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CHHS_OK = 0,
    CHHS_E_INVAL = -1,     /* bad sizes or parameters                          */
    CHHS_E_NOMEM = -2,     /* workspace smaller than chhs_workspace_bytes      */
    CHHS_E_HIP = -3,       /* a HIP runtime call failed                        */
    CHHS_E_NOCONV = -4,    /* max_vcycles reached above tol; state not advanced */
    CHHS_E_NONFINITE = -5, /* residual norm became NaN or Inf; state not advanced */
    CHHS_E_STATE = -6      /* call order violated (e.g. a V-cycle before setup) */
};

/* One instance: dim = 2 or 3 (nz = 1 for 2D); h = L/N in every direction
 * (Section 2: one spacing for all directions); eps, gamma > 0 of (1.2)-(1.4)
 * (gamma = 0 allowed: no flow); dt = the time step s.  Extents must halve
 * together: nx = cx 2^k, ny = cy 2^k (, nz = cz 2^k) with the same k >= 1.
 * Size limits of the 32-bit indexing: fewer than 2^29 cells per instance (an
 * FP64 field below 4 GiB) and at most 2^31 - 1 cells over a batch; larger
 * problems are rejected (chhs_workspace_bytes returns 0, chhs_init
 * CHHS_E_INVAL) before anything is allocated or launched. */
typedef struct chhs_problem {
    int32_t dim, nx, ny, nz;
    double h, eps, gamma, dt;
} chhs_problem;

/* Solver options.  Defaults (chhs_default_opts): nu1 = nu2 = 2, tol = 1e-10,
 * max_vcycles = 100, coarse_sweeps = 4 (smoothing steps on the coarsest grid),
 * precision 0 = FP64 throughout, 1 = FP32 smoothing/transfer inside FP64
 * residual + correction (iterative refinement), use_graph = 1 (default) replays each
 * V-cycle as a captured HIP graph (contexts with timing != 0 launch directly),
 * timing = 1 brackets every launch of every
 * kernel class with HIP events (see chhs_get_timing); any other nonzero value
 * is a mask of classes, bit (class + 1) set for each class to time.  Each
 * event pair delays the next launch by a few microseconds.  smoother selects
 * the 2D smoothing kernels of the levels above the single-workgroup tail:
 * 0 = default (row-streaming strips on the finest level, square LDS tiles on
 * coarser ones), 1 = tiles everywhere, 2 = strips on every level (including
 * the explicit smoothing calls on tail levels).  On 3D levels above the tail:
 * 0 = the fused z-marching step on levels whose z segments hold at least 16
 * planes, per-cell red-black kernels (one launch per color) on the others,
 * 3 = per-cell kernels on every level, 4 = the fused step on every level
 * (3D second-order scheme only).  All kernels perform the same red-black
 * updates (results agree to rounding).
 * tile_threads = 0 (default) gives tiled levels 1024-thread blocks when they
 * have at most 256 tiles and 256-thread blocks otherwise; 256, 512 or 1024
 * fixes the block size of every tiled level (the same arithmetic per cell).
 * tile_rows = 0 (default) cuts coarse tiled levels into 64 x 8 tiles when they
 * have at most 128 tiles of 64 x 16 (over the batch) and into 64 x 16 tiles
 * otherwise; 16, 8 or 4 fixes the tile height of every coarse tiled level
 * (the finest level has 64 x 16 tiles); 32 (precision = 1 only) gives the
 * finest level of the FP32 hierarchy 64 x 32 tiles (fewer halo cells
 * recomputed per cell) and leaves the coarse levels at their default.
 * autotune = 1 (smoother = 0, second-order scheme): chhs_init times, on the
 * problem at hand, each level's smoothing launches and keeps the fastest per
 * level (the choice then depends on the device; results agree to rounding).
 * 2D (nu1, nu2 >= 1): tiles of 256, 512 and 1024 threads (on coarse levels
 * each with 16, 8 and 4 rows; on the FP32 finest level also 64 x 32 tiles of
 * 512 and 1024 threads; the pre- and post-smoothing launches of a tile
 * height each take their fastest block size) and strips of 1/4, 1/2, 1, 2
 * and 4 times the default segment height.  3D: the fused step or the
 * per-cell kernels.
 * order = 2 (default; 0 means the same) solves the second-order scheme
 * (2.4)-(2.7).  order = 1 solves instead the first-order convex-splitting step
 * that Remark 2.2 names as a way to obtain phi^1 from phi^0 (its form is cited,
 * not written, in the paper; the reading here): the same three rows with
 * phi_* := phi^m, the convex part of chi fully implicit, chi(phi) = phi^3, the
 * whole eps^2 Lap phi implicit (kap = eps^2/h^2) and f_mu = -phi^m; phi_prev
 * is not read.  order = 1 needs precision = 0 and smooths every level with the
 * per-cell red-black kernels.
 * nu1_coarse, nu2_coarse: smoothing steps before / after the coarse
 * correction on the levels between the finest and the coarsest (0 = nu1,
 * nu2 as on the finest level; Section 5 uses V(2,2) on every level).
 * prolong = 0 (default) prolongs the coarse correction by piecewise-constant
 * injection, 1 by cell-centred bi/trilinear interpolation (3/4, 1/4 along each
 * axis, continued evenly across the boundary); Section 5 leaves the transfer
 * operators open, and both converge to the same solution (Theorem 2.1).
 * inner_cycles (precision = 1; 0 means 1, at most 8): FP32 correction-form
 * V-cycles per FP64 refinement (residual, stopping test and update).  With
 * more than one the stopping test runs every inner_cycles FP32 cycles, and
 * chhs_stats.vcycles counts refinements; the converged solution is the same
 * (to the tolerance). */
typedef struct chhs_opts {
    int32_t nu1, nu2, max_vcycles, coarse_sweeps;
    double tol;
    int32_t precision;
    int32_t use_graph;
    int32_t timing;
    int32_t smoother;
    int32_t autotune;
    int32_t order;
    int32_t tile_threads;
    int32_t tile_rows;
    int32_t nu1_coarse, nu2_coarse;
    int32_t prolong;
    int32_t inner_cycles;
} chhs_opts;

/* Kernel classes of chhs_timing. */
enum {
    CHHS_K_PRE0 = 0,       /* finest-level pre-smoothing launches (2D: nu1 steps
                              fused with residual + restriction)                */
    CHHS_K_POST0 = 1,      /* finest-level post-smoothing launches (2D: fused
                              with prolongation and the residual norm)          */
    CHHS_K_TRANSFER0 = 2,  /* standalone transfer kernels at the finest level   */
    CHHS_K_COARSE = 3,     /* every launch on coarser levels (incl. the tail)   */
    CHHS_K_NORM = 4,       /* standalone residual-norm reductions and p shift   */
    CHHS_K_SETUP = 5,      /* per-step setup and energy reductions              */
    CHHS_K_REFINE = 6,     /* mixed precision: the FP64 refinement launch on the
                              finest level (u += e, residual, FP32 right-hand
                              side and base state, norm partials)               */
    CHHS_K_COUNT = 8
};

/* Device time per kernel class accumulated while opts.timing = 1. */
typedef struct chhs_timing {
    double ms[CHHS_K_COUNT];
    int64_t launches[CHHS_K_COUNT];
} chhs_timing;

/* Per-instance statistics of the last step (or of the current system). */
typedef struct chhs_stats {
    int32_t vcycles;       /* V-cycles taken by the last step                 */
    int32_t status;        /* CHHS_OK / CHHS_E_NOCONV / CHHS_E_NONFINITE      */
    int32_t total_vcycles; /* V-cycles summed over the steps of the call      */
    int32_t steps_done;    /* steps applied by the call                       */
    double res[3];         /* ||R_phi||, ||R_mu||, ||R_p|| at exit            */
    double res_norm;       /* combined residual norm at exit                  */
    double res0;           /* combined residual norm of the initial guess     */
    double mass;           /* (phi^{m+1}, 1)                                  */
    double E_h;            /* E_h(phi^{m+1}), (2.8)                           */
    double F_h;            /* F_h(phi^{m+1}, phi^m), (2.9)                    */
    double diss_mu;        /* s ||grad_h mu||^2                               */
    double diss_u;         /* (s/gamma) ||u||^2, u = -grad p - gamma a grad mu */
    double max_abs_phi;    /* max |phi^{m+1}|                                 */
} chhs_stats;

typedef struct chhs_ctx chhs_ctx;

/* Fills *o with the defaults listed above. */
void chhs_default_opts(chhs_opts* o);

/* Bytes of device workspace chhs_init needs for n_inst instances p[0..n_inst-1]
 * under options o; 0 if the arguments are invalid. */
size_t chhs_workspace_bytes(const chhs_problem* p, int32_t n_inst, const chhs_opts* o);

/* Creates a context.  workspace_dev: caller-owned device memory of ws_bytes
 * >= chhs_workspace_bytes(...), 256-byte aligned, kept alive until
 * chhs_destroy.  hip_stream: a hipStream_t (NULL = a stream of the context's
 * own, ordered with the null stream).  The context itself (host memory,
 * pinned staging, captured graphs, that stream) is owned by the library.
 * Returns CHHS_E_INVAL, CHHS_E_NOMEM or CHHS_E_HIP on failure, with
 * *out = NULL. */
int chhs_init(const chhs_problem* p, int32_t n_inst, const chhs_opts* o,
              void* workspace_dev, size_t ws_bytes, void* hip_stream, chhs_ctx** out);

/* Advances nsteps time steps of (2.4)-(2.7).  phi_prev, phi_cur (device,
 * in/out): (phi^{m-1}, phi^m) on entry, (phi^{m+n-1}, phi^{m+n}) on success;
 * pass identical contents for the first step (phi^{-1} := phi^0, Remark 2.2).
 * mu, p (device, in/out): initial guess in, mu^{m+n-1/2}, p^{m+n-1/2} (mean
 * zero) out.  stats_host: n_inst records of the last step, or NULL (the
 * energies are those of the last step only; chhs_step_log gives every step's).  On
 * CHHS_E_NOCONV / CHHS_E_NONFINITE the failing step is not applied: the four
 * arrays hold the state before that step. */
int chhs_step(chhs_ctx* c, double* phi_prev, double* phi_cur, double* mu, double* p,
              int32_t nsteps, chhs_stats* stats_host);

/* chhs_step with the post-step reductions of every step (discrete mass (phi,1)
 * of Section 4, E_h (2.8), F_h (2.9) and the two dissipation terms of the energy
 * law of Theorem 2.1): per_step_host (host, nsteps * n_inst records, record
 * m * n_inst + i = step m of instance i; required when nsteps > 0) receives for
 * every step its cycle count, residuals and energies.  The reductions are
 * enqueued on the stream after each step's solve and read back once, at the end
 * of the call (the context keeps pinned host memory for nsteps records,
 * allocated on the first call that needs more).  On CHHS_E_NOCONV /
 * CHHS_E_NONFINITE the record of the failing step carries its status and
 * residuals, later records stay zero (steps_done = 0), and the state holds the
 * last step that succeeded. */
int chhs_step_log(chhs_ctx* c, double* phi_prev, double* phi_cur, double* mu, double* p,
                  int32_t nsteps, chhs_stats* per_step_host);

/* Loads the system of one step (setup of (2.4)-(2.7): phi_*, right-hand side,
 * cell averages on all levels) from (phi_prev, phi_cur) and the initial guess
 * (phi_cur, mu, p), without solving.  Device pointers, read only. */
int chhs_setup_step(chhs_ctx* c, const double* phi_prev, const double* phi_cur,
                    const double* mu, const double* p);

/* One FAS V(nu1, nu2) cycle on the loaded system (p normalised to mean zero
 * afterwards); writes the residual norm after the cycle to res_norm_host
 * [n_inst] (host memory). */
int chhs_fas_vcycle(chhs_ctx* c, double* res_norm_host);

/* Residual norms of the current iterate of the loaded system:
 * out_host[n_inst][4] = ||R_phi||, ||R_mu||, ||R_p||, combined. */
int chhs_residual_norms(chhs_ctx* c, double* out_host);

/* Copies the current iterate (phi, mu, p) of the loaded system into caller
 * device arrays (any may be NULL). */
int chhs_get_solution(chhs_ctx* c, double* phi, double* mu, double* p);

/* Discrete mass, E_h(phi) (2.8) and F_h(phi, phi_prev) (2.9) of caller device
 * arrays: out_host[n_inst][3] = mass, E_h, F_h.  eps and h of each instance
 * are those given to chhs_init. */
int chhs_energy_mass(chhs_ctx* c, const double* phi, const double* phi_prev, double* out_host);

/* The mass, E_h and F_h of chhs_energy_mass for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops): no
 * context, no hipMalloc / hipFree or other allocating call.  p[0..n_inst-1]:
 * the instances (dim 2 or 3, one dim for all, extents >= 1, h > 0, eps > 0;
 * only these fields are read), at most 32 instances, fewer than 2^29 cells
 * each and at most 2^31 - 1 in all; CHHS_E_INVAL otherwise.  phi, phi_prev:
 * device arrays packed instance after instance as everywhere in this ABI.
 * out_dev: DEVICE memory, [n_inst][3] = mass, E_h, F_h, written on
 * hip_stream (NULL = the null stream) when the work enqueued there runs; the
 * call returns after enqueuing and does not synchronise.  The partial sums live
 * in a fixed 512 KiB device array of the library (one per GPU, held until the
 * process ends); calls that overlap on one GPU race for it and must be
 * ordered by the caller (one stream, or events).  CHHS_E_HIP if a launch
 * fails. */
int chhs_energy_mass_noalloc(const chhs_problem* p, int32_t n_inst, const double* phi,
                             const double* phi_prev, double* out_dev, void* hip_stream);

/* Level-by-level access for kernel-level tests.  field: 0 phi, 1 mu, 2 p,
 * 3 f_phi, 4 f_mu, 5 f_p, 6 phi_*, 7 phi^m (psi).  dir 0: level -> dev,
 * dir 1: dev -> level.  Single-instance contexts only.  On the finest level
 * the kernels take f_phi = phi^m and f_p = 0, as the step's setup writes them
 * (the fields themselves are not read there). */
int chhs_level_count(chhs_ctx* c, int32_t* levels);
int chhs_level_shape(chhs_ctx* c, int32_t level, int32_t* nxyz3);

/* The smoothing kernel the V-cycle uses on level `level` (counted from the
 * finest) of the batch: out3[0] = 0 square tiles (out3[1] = threads per block
 * of the pre-smoothing launches; the autotuner may give the post-smoothing
 * launches another block size), 1 row-streaming strips (out3[1] = rows per segment), 2 per-cell kernels (one
 * launch per color), 3 inside the one-workgroup coarse tail for every instance
 * (out3[1] = 0), 4 fused 3D steps by z marching (out3[1] = planes per segment);
 * out3[2] = blocks per launch (0 for the tail).  Reflects the autotuner's
 * choice.  Any batch size; CHHS_E_INVAL for a level no instance has. */
int chhs_level_kernel(chhs_ctx* c, int32_t level, int32_t* out3);
int chhs_copy_field(chhs_ctx* c, int32_t level, int32_t field, double* dev, int32_t dir);

/* How the counted cycles run: *graphs = the number of cycle graphs captured
 * and instantiated so far (0 before the first step, 2 for the plain FP64
 * loop, 1 or 2 for mixed precision), 0 when they launch directly
 * (use_graph = 0, timing != 0, or a capture that failed, which disables
 * graphs for the context).  CHHS_E_INVAL for a null argument. */
int chhs_graph_count(chhs_ctx* c, int32_t* graphs);

/* One smoothing step (red then black collective cell update) on one level,
 * and the restriction + FAS coarse right-hand side from level to level+1.
 * Single-instance contexts only; for kernel-level tests.  chhs_smooth runs
 * the FP64 kernels: CHHS_E_INVAL on a 2D level cut into 64 x 32 tiles (a
 * mixed-precision context with tile_rows = 32 or an autotuned one). */
int chhs_smooth(chhs_ctx* c, int32_t level, int32_t nsweeps);
int chhs_restrict(chhs_ctx* c, int32_t level);

/* Copies the accumulated kernel timing into *out (host); reset != 0 zeroes it.
 * Synchronises the stream.  All zero unless opts.timing = 1. */
int chhs_get_timing(chhs_ctx* c, chhs_timing* out, int32_t reset);

/* Replaces opts.timing (same meaning; >= 0) from the next launch on, for
 * example to time only one class in a measured stretch.  Captured cycle
 * graphs are dropped when the mask changes (they are captured again when
 * timing is 0).  CHHS_E_INVAL for a negative mask. */
int chhs_set_timing(chhs_ctx* c, int32_t timing);

/* Chooses the sweeps per level and the prolongation (and, in mixed precision,
 * the FP32 cycles per refinement) by time to tolerance:
 * on the system of the step from (phi_prev, phi_cur) with initial guess (mu,
 * p) (device arrays, read only; the state is not advanced), solves the step
 * to tol for each of a fixed set of candidates (nu1, nu2 on the finest
 * level, nu1_coarse, nu2_coarse below it, prolong; the context's own options
 * first; then, for precision = 1, inner_cycles 1, 2 and 3 with the kept
 * cycle), times the solve (setup and cycles; the best of three after one
 * untimed solve that captures the cycle graphs) and keeps the fastest in the
 * context's options, replacing the given ones only if it is more than 2%
 * faster.  Candidates that do not reach tol within max_vcycles are skipped.  The solution is the same to tol for
 * every candidate (Theorem 2.1: one solution per step); only the time and the
 * cycle count differ.  choice_out (host, 6 values, or NULL): the kept nu1,
 * nu2, nu1_coarse, nu2_coarse, prolong, inner_cycles.  CHHS_E_NOCONV if no
 * candidate converges (options unchanged). */
int chhs_tune_sweeps(chhs_ctx* c, const double* phi_prev, const double* phi_cur, const double* mu,
                     const double* p, int32_t* choice_out);

/* The context's options as they are now (after chhs_tune_sweeps or
 * chhs_set_timing). */
int chhs_get_opts(chhs_ctx* c, chhs_opts* out);

/* Releases the context (not the caller's workspace).  NULL is ignored. */
void chhs_destroy(chhs_ctx* c);

/* Static text for a return code. */
const char* chhs_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* CHHS_H */
