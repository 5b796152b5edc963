/*
 * lo.h -- C ABI of an MI355X (gfx950) implementation of the fully discrete
 * Lax--Oleinik scheme for separable Hamilton--Jacobi equations
 *     d_t u + K(grad u) + V(t, x) = 0,   K(p) = sum_a K_a(p_a)
 * of Bouillard, Faou and Zavidovique, "Fast weak-KAM integrators for
 * separable Hamiltonian systems" (arXiv:1210.4090).
 *
 * One time step (Section 2.3, eq. eqconvol, split axis by axis as in
 * Remark rk28, on the periodic grid of Section 3.3 / Remark rk282):
 *     w_0 = u
 *     w_{a+1}(x) = min over lifted grid sources y on the line of x along a of
 *                  fl( w_a(y) + tau K*_a((x_a - y_a) / tau) ),   a = 0..d-1
 *     u+(x) = fl( w_d(x) - fl(tau V(t_n, x)) )
 * and N steps compose as in eq. uN with t_n = t0 + n tau.
 *
 * Conventions
 *  - Grids: ndim in {1,2,3}; axis a has n[a] points, spacing dx_a =
 *    period[a] / n[a]; arrays are FP64, row-major with axis 0 fastest:
 *    index = i0 + n0 (i1 + n1 i2).
 *  - Kinetic cost of a displacement of s cells (target minus source) along
 *    axis a: for the mechanical Hamiltonian K_a(p) = (p + P_a)^2 / 2
 *    (eq. HPV, Lagrangian v^2/2 - P_a v of Section 2.1) it is evaluated as
 *        d = s * dx_a;  k = ((0.5 * d) * d) / tau - P_a * d
 *    in IEEE binary64 with no contraction; or it is read from a caller table
 *    of tau K*_a(s dx_a / tau) (hypothesis (i): the table must be discretely
 *    convex; displacements outside the table cost +inf).
 *  - Argmin offsets are e = source - target in cells along the axis, on the
 *    lifted line (so |e| may exceed n[a]/2); among equal minima the smallest
 *    e is reported.  They are int16: a call that requested argmins and met an
 *    offset beyond +-32767 returns LO_ERR_UNSUPPORTED (its stored offsets are
 *    then unusable).
 *  - Pointers documented "device" are HIP device memory owned by the caller;
 *    "host" pointers are read during the call only.  Streams are hipStream_t
 *    passed as void* (NULL = default stream).  A plan is used from one
 *    stream at a time.
 *  - Every entry point returns lo_status and never aborts.  Errors found on
 *    the device (a window that exceeded the plan's capacity, an argmin that
 *    hit a fixed window's edge) are latched in the plan and returned by the
 *    next call that synchronises (lo_run, lo_step, lo_backward, lo_last_diag).
 */
#ifndef LO_H
#define LO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lo_plan_s* lo_plan_t;

typedef enum {
    LO_OK = 0,
    LO_ERR_INVALID = 1,      /* bad descriptor, argument or non-convex table */
    LO_ERR_UNSUPPORTED = 2,  /* valid request this build does not implement */
    LO_ERR_OOM = 3,          /* device allocation failed */
    LO_ERR_HIP = 4,          /* a HIP runtime call failed */
    LO_ERR_WINDOW = 5        /* window saturated or exceeded capacity: result untrusted */
} lo_status;

typedef enum {
    LO_BRUTE = 0,   /* windowed exhaustive minimum: bit-exact with the definition */
    LO_FAST = 1     /* claim (lower-envelope) kernels: each source claims the targets where it
                       beats its neighbours.  O(1) per point for the mechanical cost, the
                       minimum within 1e-12; O(log window) per point for a caller's convex
                       table (crossings by bisection), the minimum and argmins exact */
} lo_method;

/* flags */
#define LO_FLAG_NO_GRAPH 1u   /* lo_run: launch kernels directly, no HIP graph */
#define LO_FLAG_AUTOTUNE 2u   /* LO_FAST: the first lo_run advances a copy of its input 60 steps
                                 (past the wide windows of the first steps), times each fast
                                 sweep's launch shapes (points per thread of a row sweep, tile
                                 length of the last axis's tile sweep; other tile axes keep a
                                 length that follows the window) over 8 steps from there
                                 (twice, alternately) and keeps, per axis, one
                                 more than 3% faster than the default; the choice is kept for
                                 later plans of the same grid in the process, and in the file
                                 named by the environment variable LO_TUNE_CACHE when it is set
                                 (LO_TUNE_LOG, when set, prints each timing to stderr).
                                 Results do not depend on the shape.  lo_effective_H applies
                                 it to each batch. */

typedef struct {
    int32_t ndim;              /* 1..3 */
    int64_t n[3];              /* grid points per axis, each >= 3 */
    double period[3];          /* torus period per axis (> 0) */
    double tau;                /* time step (> 0) */
    double P[3];               /* rotation vector of K_a(p) = (p + P_a)^2/2 */
    const double* kstar_tab[3];/* host, optional: tau K*_a(s dx_a/tau) for s in
                                  [-kstar_half[a], kstar_half[a]]; NULL = mechanical */
    int64_t kstar_half[3];
    int32_t window[3];         /* 0 = rigorous window computed on the device every step;
                                  > 0 = fixed half-width, swept by the exhaustive (brute) kernels
                                  whatever the method (a minimiser on or past the edge
                                  raises LO_ERR_WINDOW) */
    int32_t method;            /* lo_method */
    uint32_t flags;            /* LO_FLAG_* */
    double t0;                 /* time of step 0 */
} lo_desc;

/*
 * Potential V(t, x) on the grid, one of:
 *  - table != NULL: static V, device [npts], copied at plan time;
 *  - nmodes > 0, basis != NULL (device [nmodes][npts], must outlive the plan):
 *      coef  (host [nmodes])        static V = sum_m coef[m] basis[m], summed in m order;
 *      tcoef (host [ntcoef][nmodes]) V(t_n) = sum_m tcoef[n][m] basis[m] (steps n < ntcoef);
 *  - all NULL / 0: V = 0.
 */
typedef struct {
    const double* table;
    int32_t nmodes;
    const double* basis;
    const double* coef;
    const double* tcoef;
    int64_t ntcoef;
} lo_potential;

/* Build a plan: validates the descriptor (Section 2.1 hypotheses (i); grid
 * sizes), builds the kinetic tables and tau*V on the device.  Synchronous. */
lo_status lo_plan(const lo_desc* desc, const lo_potential* V, lo_plan_t* out);

lo_status lo_plan_destroy(lo_plan_t plan);

/* Replace the static coefficients of a basis potential (host [nmodes]) and
 * rebuild tau*V (used by the differentiable front end).  Synchronous. */
lo_status lo_set_coef(lo_plan_t plan, const double* coef);

/* One step n (time t0 + n tau), in place on u (device [npts]).  argmin:
 * NULL or device int16 [ndim][npts] receiving the offsets of every axis
 * sweep.  Synchronises on return. */
lo_status lo_step(lo_plan_t plan, double* u, int64_t n, int16_t* argmin, void* stream);

/* Steps n0 .. n0+nsteps-1 in place on u (device [npts]) -- eq. uN.
 * If ckpt_every > 0 and ckpt != NULL, ckpt (device [ceil(nsteps/ckpt_every)][npts])
 * receives u before steps n0 + k*ckpt_every.  Synchronises on return. */
lo_status lo_run(lo_plan_t plan, double* u, int64_t n0, int64_t nsteps,
                 int64_t ckpt_every, double* ckpt, void* stream);

/*
 * Discrete effective Hamiltonian (Proposition prop:klm) of ninst independent
 * problems in one persistent launch.  descs[i] / V[i] describe instance i
 * (2-D, static potential, 1/tau an integer so that (dx, tau) is rational as
 * in Section 3.3); every instance starts from u0 = 0 and runs T/tau steps.
 * With D = u(T) - u(T-1), hbar_out (host [ninst][3]) receives
 * {-max D, -(max D + min D)/2, -min D}: a bracket of the effective
 * Hamiltonian and its midpoint.  Synchronous.
 */
lo_status lo_effective_H(int32_t ninst, const lo_desc* descs, const lo_potential* V, double T,
                         double* hbar_out, void* stream);

/*
 * Adjoint of the N-step map u0 -> u^N = T^N u0 for the plan's static
 * potential.  ckpt: device [ceil(nsteps/ckpt_every)][npts] as written by
 * lo_run(n0 = 0), may be NULL when nsteps = 0; grad_uT: device [npts] = dL/du^N.  Outputs (each may be
 * NULL): grad_u0 device [npts] = dL/du0; grad_coef host [nmodes] = dL/dc
 * for a basis potential.  Segments of ckpt_every steps are recomputed from
 * the checkpoints with int16 argmins and the upstream gradient is scattered
 * onto the argmin sources axis by axis in reverse.  Synchronous.
 */
lo_status lo_backward(lo_plan_t plan, const double* ckpt, int64_t nsteps, int64_t ckpt_every,
                      const double* grad_uT, double* grad_u0, double* grad_coef, void* stream);

/* Forward run that records every sweep's argmins, for an adjoint without
 * recomputation: steps n0 .. n0+nsteps-1 on u (device [npts]) as lo_run, and
 * argmins (device int16 [nsteps][ndim][npts], caller-owned) receives every
 * step's offsets as lo_step reports them.  Trades 2 ndim bytes a point a step
 * (2 GB for 500 steps of a 1024^2 grid) for the segment recompute of
 * lo_backward.  Errors as lo_run; LO_ERR_UNSUPPORTED if an offset exceeds
 * int16.  Synchronous. */
lo_status lo_run_record(lo_plan_t plan, double* u, int64_t n0, int64_t nsteps, int16_t* argmins, void* stream);

/* Adjoint of the nsteps-step map from argmins recorded by lo_run_record
 * (steps 0 .. nsteps-1, device int16 [nsteps][ndim][npts]): gradients as
 * lo_backward's, without recomputing any step (the same argmins, scattered in
 * the same order, give the same gradients).  Same arguments and errors as
 * lo_backward otherwise. */
lo_status lo_backward_recorded(lo_plan_t plan, const int16_t* argmins, int64_t nsteps, const double* grad_uT,
                               double* grad_u0, double* grad_coef, void* stream);

const char* lo_status_string(lo_status s);

/* Diagnostics of the last lo_step/lo_run/lo_backward (host arrays [ndim],
 * each may be NULL): the largest |argmin offset| seen per axis (only when
 * argmins were produced, else -1), and the widest window used.  Returns
 * LO_ERR_WINDOW when that call's window saturated. */
lo_status lo_last_diag(lo_plan_t plan, int32_t* max_abs_offset, int32_t* window_used);

/* Copy the plan's kinetic cost for displacements s0 .. s0+count-1 of one
 * axis into a host array (for checking the table against an independent
 * evaluation).  Displacements outside the plan's range give +inf. */
lo_status lo_kinetic_table(lo_plan_t plan, int32_t axis, int64_t s0, int64_t count, double* out);

/* Measurement aid: runs steps n0 .. n0+nsteps-1 on u (device [npts]) like
 * lo_run but without a graph, with a pair of HIP events on `stream` around
 * every axis sweep (the steps run back to back; the host reads the events
 * every 30 steps); ms (host [ndim]) receives the mean interval of each axis'
 * pair in milliseconds: the kernel's duration plus the events' own cost, so
 * never less than a profiler's kernel duration.  Synchronous. */
lo_status lo_time_kernels(lo_plan_t plan, double* u, int64_t n0, int64_t nsteps, double* ms, void* stream);

/* Comparison path: the paper's own fast algorithm (Section 4) on a 1-D plan.
 * Each step splits the lifted line into convex and concave pieces (a convex
 * piece continues while its slopes drop by at most eta, a concave one while
 * they rise by at most eta: Section 4.3's tolerance; eta = 0 is exact),
 * convolves each piece with the kinetic cost restricted to offsets
 * [-window, window] in linear time (Theorem th:convex; Theorem th:ccc and
 * Lemma lm:simplif for concave pieces), takes the minimum over the pieces and
 * subtracts tau V(t_n).  Runs steps n0 .. n0+nsteps-1 on u (device [n[0]]).
 * window = 0 takes the plan's whole cost table; a window that holds every
 * minimiser with eta = 0 gives the definition's result (every value is a
 * genuine candidate; near-ties may pick one a few ulps off).  pieces / breaks
 * (host, may be NULL) receive the pieces convolved over the run and the
 * breaks between pieces of different type (pieces also end at the borders of
 * the 64-source segments that GPU threads take).  LO_ERR_UNSUPPORTED unless
 * the plan is 1-D and not batched; LO_ERR_INVALID for eta < 0, window < 0 or
 * above the plan's table, or steps beyond a time-dependent potential's
 * schedule.  Synchronous; allocates its scratch in the plan on first use. */
lo_status lo_run_decomp(lo_plan_t plan, double* u, int64_t n0, int64_t nsteps, double eta, int32_t window,
                        int64_t* pieces, int64_t* breaks, void* stream);

/* The first discrete semigroup (Section 2.2, eq. cost1, composed as in
 * eq. compo) on a 1-D plan with a static potential (or none): each step is
 *     u+(x) = min over lifted y in [x - window, x + window] of
 *             fl( fl(u(y) + k(x - y)) - I(y, x) ),
 * k the plan's kinetic cost and I the time integral of V along the straight
 * path from y to x, by the trapezoid rule over the grid points the path
 * crosses, on hv = fl(tau V): I = hv(x) when y = x, else
 * (hv(y)/2 + hv(y+d) + ... + hv(x-d) + hv(x)/2) / m, m = |x - y|, d = sign(x - y).  The potential is inside the cost (no separate potential
 * step).  Path sums come from prefix sums of hv, so values agree with the
 * path-order definition to rounding (about N eps max|tau V|), not bit for
 * bit.  window = 0 takes the plan's whole cost table.  Runs nsteps steps on
 * u (device [n[0]]).  LO_ERR_WINDOW when a minimiser reached |x - y| = window
 * (the result may then miss farther minimisers); LO_ERR_UNSUPPORTED unless
 * the plan is 1-D, not batched and its potential static; LO_ERR_INVALID for
 * window < 0 or above the plan's table.  Synchronous; allocates its scratch in
 * the plan on first use. */
lo_status lo_run_semigroup1(lo_plan_t plan, double* u, int64_t nsteps, int32_t window, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lo_step
 * without a plan, allocating nothing.  One step n (time t0 + n tau) in place on
 * u (device [npts]) for the mechanical cost of desc (kstar_tab must be NULL:
 * LO_ERR_UNSUPPORTED otherwise); tau_v: NULL (no potential) or device [npts]
 * holding fl(tau V(t_n, x)), read only; argmin: NULL or device int16
 * [ndim][npts] as in lo_step.  desc->flags is ignored.  Values and argmins
 * equal lo_step's for the same descriptor and potential.
 * Work memory: one static device array of about 34 MiB (kinetic tables, a
 * second grid array of LO_NOALLOC_MAX_POINTS doubles, statistics, flags),
 * which each GPU that runs this call holds until the process ends.  Grids of
 * more than LO_NOALLOC_MAX_POINTS points return LO_ERR_UNSUPPORTED before any
 * device work.  Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (other threads, other streams) race and must be
 * serialised by the caller.  Runs on the current device; the stream must
 * belong to it.  Synchronises on return; errors as lo_step. */
#define LO_NOALLOC_MAX_POINTS 4194304
lo_status lo_step_noalloc(const lo_desc* desc, const double* tau_v, double* u, int64_t n, int16_t* argmin,
                          void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LO_H */
