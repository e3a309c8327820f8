/*
 * lbm.h -- C ABI of the MI355X lattice Boltzmann engine with the single-node
 * second-order boundary scheme of Zhao & Yong, "A family of single-node
 * second-order boundary schemes for the lattice Boltzmann method".
 *
 * One time step (paper, Section 2) is
 *   collision   f'_i(x,t) = f_i(x,t) + Omega_i(x,t)                 Eq. (22a)
 *   advection   f_i(x+e_i, t+1) = f'_i(x,t)                          Eq. (22b)
 * with the MRT collision of the Appendix (equilibrium Eq. (42)), and on
 * every cut link (x_f, i) -- x_f fluid, x_f - e_i solid, wall at
 * x_b = x_f - gamma e_i, gamma in (0,1] -- the single-node scheme
 *   f_i(x_f,t+1) = (1-b) f_i(x_f,t) + b [ (1+l-2g)/(1+l) f_ibar(x_f,t)
 *                 + l/(1+l) f'_i(x_f,t) + (2g-l)/(1+l) f'_ibar(x_f,t)
 *                 + 2/(1+l) * 3 w_i rho0 e_i.phi(x_b,t) ]                Eq. (213)
 * (Eq. (210) when b = 1), l = l(gamma) inside the band of Eq. (212).
 *
 * Units: lattice units, h = dt = c = 1, c_s^2 = 1/3.
 * Layout: node index n = x + nx*(y + ny*z), x fastest; 2D lattices have
 * nz = 1.  Distributions are handled as deviations from the rest state,
 * delta f_i = f_i - w_i rho0, stored on the GPU in blocks of 2048 nodes that
 * each hold their Q direction runs; host arrays use planes [Q][N].
 *
 * Conventions for every call:
 *  - Return value: LBM_OK (0) or a negative LBM_E* code; the message is
 *    available from lbm_last_error().  No C++ exception crosses the ABI.
 *  - Host input arrays are copied during the call; the caller keeps them.
 *    Host output arrays are caller-allocated with the stated sizes.
 *    Pointers named *_dev are device memory owned by the caller.
 *  - A handle is not thread-safe; separate handles are independent.
 *  - lbm_step, lbm_run_checkpointed and lbm_adjoint only enqueue work on the
 *    handle's stream; calls that return host data synchronise that stream.
 *    A kernel fault surfaces as LBM_EDEVICE at the next synchronising call.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm lbm_t;

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* bad argument value */
    LBM_EGEOM = -2,       /* solid mask and cut links are inconsistent */
    LBM_ESTATE = -3,      /* call out of order (e.g. step before geometry) */
    LBM_ENOMEM = -4,      /* device or host allocation failed */
    LBM_EDEVICE = -5,     /* HIP runtime error */
    LBM_ENONFINITE = -6   /* a reduction met a NaN or infinity */
};

/* lattices: velocity orderings are reported by lbm_lattice_info().
 * D2Q9 and D3Q15 are ordered as in the paper's Appendix (D3Q15: rest, the
 * six axis vectors, then the eight corner vectors, with the Appendix's
 * transformation matrix); D3Q19 is rest, the six axis vectors
 * (+x,-x,+y,-y,+z,-z), then the twelve edge vectors. */
enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1, LBM_D3Q15 = 2 };

/* precision: FP64 stores and computes delta f in double; FP32 stores and
 * computes delta f in float.  In both, the per-link coefficients are
 * computed in double (and stored in the populations' precision), and the
 * boundary combination, reductions and gradient sums are double. */
enum { LBM_FP64 = 0, LBM_FP32 = 1 };

/* l(gamma) rules; the first five are the paper's Section 3 choices, ZERO is
 * Remark (5)'s nonconvex member, MIN = max(0, 2 gamma - 1) is the lower edge
 * of Eq. (212) and the only convex rule listed that reproduces half-way
 * bounce-back (Eq. (26)) at gamma = 1/2.  Default: LBM_L_MIN. */
enum {
    LBM_L_GAMMA = 0, LBM_L_1P5GAMMA = 1, LBM_L_2GAMMA = 2, LBM_L_GAMMA2 = 3,
    LBM_L_GAMMA2_PLUS_GAMMA = 4, LBM_L_ZERO = 5, LBM_L_MIN = 6
};

/* x boundary: y and z are always periodic.
 * PERIODIC: periodic x.
 * PRESSURE: periodic x with a density jump drho: a population that crosses
 *   from x = nx-1 to x = 0 gains w_i*drho, one crossing the other way loses
 *   w_i*drho (a pressure drop c_s^2*drho per period).
 * OUTFLOW: column x = 0 must be solid; at x = nx-1 a population moving in
 *   -x is read from (nx-1, y-e_y, z-e_z) (zero x-gradient). */
enum { LBM_X_PERIODIC = 0, LBM_X_PRESSURE = 1, LBM_X_OUTFLOW = 2 };

/* objectives for the adjoint: J = mean over steps t in [t_begin, t_end) of
 * FORCE_X: x component of the momentum-exchange force on the links with the
 *   given tag during step t -> t+1,
 *   sum_links (e_ibar)_x (f'_ibar(x_f,t) + f_i(x_f,t+1));
 * MEAN_UX: mean of u_x(x,t) over the fluid nodes;
 * PRESSURE_DROP: p_in(t) - p_out(t), p = c_s^2 rho = rho / 3 the pressure of
 *   the incompressible model (Eq. (42) and the pressure of Section 3.2),
 *   p_in and p_out its means over the fluid nodes of the cross-sections
 *   x = x_in and x = x_out (lbm_set_objective_planes; default 0 and nx-1). */
enum { LBM_OBJ_NONE = 0, LBM_OBJ_FORCE_X = 1, LBM_OBJ_MEAN_UX = 2, LBM_OBJ_PRESSURE_DROP = 3 };

/* Create a solver.  s: Q relaxation rates in the row order of the lattice's
 * moment matrix (rows for conserved moments -- density and momentum -- are
 * ignored because their non-equilibrium part vanishes); each other rate in
 * (0, 2).  rho0 > 0 is the mean density of Eq. (42).  g: body force per unit
 * mass (D values) or NULL; it enters the collision as 3 w_i rho0 e_i.g.
 * Allocates the distribution arrays on the current HIP device.
 * Errors: EINVAL (lattice, precision, sizes, rates), ENOMEM, EDEVICE. */
int lbm_create(lbm_t **out, int lattice, int precision, int64_t nx,
               int64_t ny, int64_t nz, const double *s, double rho0,
               const double *g);

/* Choose l(gamma) and b of Eq. (213); b in (0, 1].  Must precede
 * lbm_set_geometry.  Errors: EINVAL, ESTATE (geometry already set). */
int lbm_set_scheme(lbm_t *h, int l_rule, double b);

/* Use the two-node scheme Eq. (211) of Remark (2) instead of Eq. (210)
 * (on != 0): the time-lagged f_ibar(x_f, t) is replaced by its advected
 * value f'_ibar(x_f + e_i, t), which the next step's pull brings to x_f; a
 * link whose neighbour x_f + e_i is solid keeps Eq. (210).  With b < 1 the
 * bracket of Eq. (213) is modified the same way.  Must precede
 * lbm_set_geometry.  Errors: ESTATE. */
int lbm_set_two_node(lbm_t *h, int on);

/* Time-dependent wall data of the separable form phi(x_b, t) =
 * phi(x_b, 0) * lambda^t (t in steps): the step from t to t+1 uses the wall
 * term of Eq. (210)/(213) scaled by lambda^t (phi at time t, as in Eq. (210)).
 * The Taylor-Green vortex of Section 3.2 has such data, lambda =
 * exp(-8 pi^2 nu dt).  The adjoint applies the same factor, so dwall_u of
 * lbm_grad is the gradient with respect to phi(x_b, 0).  lambda = 1 (the
 * default) is constant data; any other value disables lbm_step's graph
 * replay.  EINVAL unless lambda is finite and positive. */
int lbm_set_wall_decay(lbm_t *h, double lambda);

/* Choose the x boundary (see above); drho is used by LBM_X_PRESSURE only.
 * Must precede lbm_set_geometry.  Errors: EINVAL, ESTATE. */
int lbm_set_x_boundary(lbm_t *h, int kind, double drho);

/* Set the obstacle geometry.
 * solid: N bytes (1 = solid, 0 = fluid).
 * n_links cut links (x_f, i), sorted by (node, dir) or not (they are sorted
 * here): node[k] the fluid node x_f, dir[k] the direction i with x_f - e_i
 * solid, q[k] = gamma in (0, 1], wall_u[k*D + a] = phi(x_b) (NULL = 0),
 * tag[k] >= 0 an obstacle label for forces and objectives (NULL = 0).
 * A fluid direction whose pull source is solid must be listed, once, and a
 * listed direction must have a solid pull source.  The coefficients of
 * Eq. (213) are computed here in double and checked against Eq. (212).
 * Errors: EINVAL (q, rule violates Eq. (212), more than 2^26 links),
 * EGEOM (inconsistent mask/links, fluid at x = 0 with OUTFLOW), ENOMEM. */
int lbm_set_geometry(lbm_t *h, const uint8_t *solid, int64_t n_links,
                     const int64_t *node, const int8_t *dir, const double *q,
                     const double *wall_u, const int32_t *tag);

/* Replace the per-link gamma and wall velocity of the current geometry (same
 * links, same order as given to lbm_set_geometry); recomputes coefficients.
 * Either pointer may be NULL to keep the current values. */
int lbm_update_links(lbm_t *h, const double *q, const double *wall_u);

/* Collision operators of Remark (1) (the boundary scheme does not depend on
 * the collision): every row of the moment matrix is even or odd under
 * e -> -e, so the two-relaxation-time operator (TRT) -- relaxing the halves
 * (f_i + f_ibar)/2 at s_plus and (f_i - f_ibar)/2 at s_minus -- is exactly the
 * MRT operator with rate s_plus on the even rows and s_minus on the odd ones;
 * BGK is s_minus = s_plus.  For TRT, s_plus = s_nu and s_minus follows from
 * (1/s_plus - 1/2)(1/s_minus - 1/2) = magic (magic > 0; 3/16 is the common
 * choice).  The conserved rows get s_nu too (their non-equilibrium part is
 * zero, so any value is equivalent). */
enum { LBM_COLLISION_BGK = 1, LBM_COLLISION_TRT = 2 };

/* The Q rates of such an operator, in the lattice's moment-row order, into
 * s_out (no GPU needed).  s_nu in (0, 2); magic is ignored for BGK.
 * Errors: EINVAL. */
int lbm_collision_rates(int lattice, int kind, double s_nu, double magic, double *s_out);

/* Set the rates of a handle to those of lbm_collision_rates() (as
 * lbm_set_parameters() would).  Errors: EINVAL. */
int lbm_set_collision(lbm_t *h, int kind, double s_nu, double magic);

/* Replace the relaxation rates (Q values, same rules as lbm_create) or the
 * body force (D values); either pointer may be NULL.  Takes effect at the
 * next step; the state is kept.  Errors: EINVAL. */
int lbm_set_parameters(lbm_t *h, const double *s, const double *g);

/* Initial state f(x,0) = f^eq(rho(x), u(x)) of Eq. (42) at fluid nodes.
 * rho: N values or NULL (rho0); u: N*D values, u[n*D + a], or NULL (0).
 * Resets the time counter to 0.  With LBM_X_OUTFLOW, the outlet column's
 * -x populations are represented through the zero-gradient rule (exact for
 * x-uniform initial fields there).  Errors: ESTATE, ENOMEM, EDEVICE. */
int lbm_init(lbm_t *h, const double *rho, const double *u);

/* Initial state given as deviations df[i*N + n] = f_i(n,0) - w_i rho0
 * (solid entries ignored).  Resets the time counter to 0. */
int lbm_init_deviation(lbm_t *h, const double *df);

/* Enqueue n >= 0 time steps.  On domains of at most 2^20 nodes, runs of 64
 * steps outside an objective window are replayed from a captured HIP graph
 * (launch-bound sizes); results are identical to single launches.  The
 * graph is rebuilt after any change of parameters, links, geometry or
 * stream. */
int lbm_step(lbm_t *h, int64_t n);

/* Current time (number of steps taken since init or set_state). */
int64_t lbm_time(const lbm_t *h);

/* Macroscopic fields at the current time t, from f(x,t):
 * rho[n] = rho0 + sum_i delta f_i, u[n*D + a] = sum_i e_ia f_i / rho0.
 * Solid nodes get NaN.  Either pointer may be NULL.  Synchronises. */
int lbm_moments(lbm_t *h, double *rho, double *u);

/* Pre-collision deviations df[i*N + n] = f_i(n,t) - w_i rho0 at the current
 * time (NaN at solid nodes).  Synchronises. */
int lbm_get_distribution(lbm_t *h, double *df);

/* Totals at the current time over fluid nodes, summed in double:
 * mass = sum rho, mom[a] = sum rho0 u_a.  ENONFINITE if either is not
 * finite.  Synchronises. */
int lbm_reduce(lbm_t *h, double *mass, double *mom);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * totals of lbm_reduce(), same outputs and errors, computed without any
 * allocation.  The per-block partial sums go to a fixed device array of
 * 2^19 doubles (4 MiB) that the library holds on each device until the
 * process ends; EINVAL when the domain needs more partial sums than that
 * (above 33,554,176 nodes for D3Q19/D3Q15, 44,738,816 for D2Q9).  Every
 * call on one device uses the same array: calls that overlap on one device
 * (separate threads or streams) race.  Synchronises. */
int lbm_reduce_noalloc(lbm_t *h, double *mass, double *mom);

/* Momentum-exchange force of the most recent step t-1 -> t on each tag:
 * force[tag*D + a] = sum over the tag's links of
 * (e_ibar)_a (f'_ibar(x_f,t-1) + f_i(x_f,t)), absolute (not deviation)
 * values, for tags 0 .. n_tags-1.  ESTATE before the first step. */
int lbm_force(lbm_t *h, int32_t n_tags, double *force);

/* Device state: the post-collision array and the link slots; together with
 * lbm_time() they determine every later step.  dst/src are device buffers
 * of lbm_state_bytes() bytes owned by the caller. */
int64_t lbm_state_bytes(const lbm_t *h);
int lbm_get_state(lbm_t *h, void *dst_dev);
int lbm_set_state(lbm_t *h, const void *src_dev, int64_t time);

/* Objective of the adjoint (see LBM_OBJ_*); resets its accumulator.  The
 * accumulation happens during later lbm_step / lbm_run_checkpointed calls
 * whose steps fall in [t_begin, t_end). */
int lbm_set_objective(lbm_t *h, int kind, int32_t tag, int64_t t_begin,
                      int64_t t_end);

/* Cross-sections x = x_in and x = x_out (0 <= x < nx) of the PRESSURE_DROP
 * objective; read by the next lbm_set_objective(), which fails with EINVAL
 * when either plane has no fluid node.  Errors: EINVAL. */
int lbm_set_objective_planes(lbm_t *h, int64_t x_in, int64_t x_out);

/* Pressure drop at the current time t, from f(x,t): *dp = p_in - p_out with
 * p = rho / 3 averaged over the fluid nodes of the planes x = x_in and
 * x = x_out, summed in double.  Errors: EINVAL (plane outside [0, nx) or
 * without fluid), ESTATE, ENONFINITE.  Synchronises. */
int lbm_pressure_drop(lbm_t *h, int64_t x_in, int64_t x_out, double *dp);

/* Value of the objective accumulated so far.  Synchronises. */
int lbm_objective(lbm_t *h, double *J);

/* Run n steps from the current state keeping a snapshot every `every` steps
 * in library-owned device memory, so that lbm_adjoint() can later replay
 * each segment (sqrt(n) checkpointing when every ~ sqrt(n); every = 1 keeps
 * every state and needs no replay).  A snapshot is taken by exchanging
 * buffers with the current state, without a copy, and the snapshot buffers
 * are kept for the next run with the same snapshot count.  Memory: ceil(n /
 * every) snapshots, plus `every` replay states and two adjoint arrays
 * allocated by lbm_adjoint(), all of lbm_state_bytes().
 * With the rate gradients off the reverse sweep reads step records instead
 * of states (see lbm_set_rate_gradient): the run records the last step of
 * every segment, lbm_adjoint() replays each segment through two states
 * recording its other steps, and every = 1 records every step and keeps no
 * snapshot (no replay at all).  A record is D values per node plus 3 per
 * cut link, in the handle's precision; memory ceil(n / every) records, plus
 * every - 1 records and two states for the replay when every > 1 (and, with
 * Eq. (211), two more runs of one value per link).  The objective
 * accumulates as in lbm_step.  Errors: ESTATE, EINVAL, ENOMEM. */
int lbm_run_checkpointed(lbm_t *h, int64_t n, int64_t every);

/* Reverse sweep over the last lbm_run_checkpointed() run: for each segment
 * from the last, replay it from its snapshot as far as the adjoint reads it
 * (every state but the segment's last; Eq. (211) also reads the next
 * snapshot), and run the adjoint steps backwards, accumulating in double
 * the gradients of the objective.  The wall-data factor of
 * lbm_set_wall_decay applies at each step's time.  Leaves the forward state
 * at the end of the run; can be called again on the same run.  Errors:
 * ESTATE (no run), ENOMEM, EDEVICE. */
int lbm_adjoint(lbm_t *h);

/* The same reverse sweep in pieces: n more adjoint steps backwards (fewer
 * when the sweep reaches the run's first step; n = 0 only starts it).  The
 * first call after lbm_run_checkpointed() starts a sweep from the run's end
 * (zeroing the gradient sums); lbm_adjoint() always starts a new one.
 * Between calls lbm_get_adjoint() returns lambda at the sweep's current
 * time and lbm_grad() the sums so far; the whole sweep in any number of
 * pieces gives the same values, bit for bit, as lbm_adjoint().  Changing
 * links, parameters or the objective before the sweep ends makes it
 * inconsistent with the recorded run.  Errors: as lbm_adjoint, EINVAL for
 * n < 0. */
int lbm_adjoint_step(lbm_t *h, int64_t n);

/* Steps the current reverse sweep still has to go (0 when it has reached
 * the run's first step), or -1 when no sweep has started. */
int64_t lbm_adjoint_remaining(const lbm_t *h);

/* Choose whether lbm_adjoint() accumulates dJ/ds for the relaxation rates
 * (a block reduction of Q extra sums per step; default on).  When off,
 * lbm_grad() reports zeros for ds, and the reverse sweep reads, for each
 * forward step, a record of the velocity u of the state it starts from (the
 * equilibrium's Jacobian depends on u alone) and of the three forward values
 * of each cut link's gradient, f_ibar(x_f, t), f'_i(x_f, t) and
 * f'_ibar(x_f, t), instead of the states (see lbm_run_checkpointed; the
 * gradients are the same).  Takes effect at the next lbm_run_checkpointed();
 * a sweep over a run that kept records only (every = 1) while the rate
 * gradients are on fails with ESTATE, and so does any sweep after the
 * boundary scheme (Eq. (210)/(213) or Eq. (211)) was changed since the
 * run. */
int lbm_set_rate_gradient(lbm_t *h, int on);

/* Gradients of J from the last lbm_adjoint(), in double: dq[k] = dJ/dgamma_k
 * (l follows gamma through the rule), dwall_u[k*D + a] = dJ/dphi_k,a,
 * dg[a] = dJ/dg_a, ds[k] = dJ/ds_k for the relaxation rates.  Any pointer
 * may be NULL.  Synchronises. */
int lbm_grad(lbm_t *h, double *dq, double *dwall_u, double *dg, double *ds);

/* The same gradients with the per-link ones left on the device: dq_dev
 * (n_links doubles) and dwall_u_dev (n_links * D doubles, link-major) are
 * device memory owned by the caller, written in the caller's link order by
 * a kernel enqueued on the handle's stream (no host transfer; the caller
 * orders its own use after that stream).  dg and ds are host arrays as in
 * lbm_grad(); when both are NULL the call does not synchronise.  Any
 * pointer may be NULL. */
int lbm_grad_device(lbm_t *h, void *dq_dev, void *dwall_u_dev, double *dg, double *ds);

/* Adjoint state lambda(t0) = dJ/df(x, t0) at the start of the last run,
 * lam[i*N + n] (0 at solid nodes).  Synchronises. */
int lbm_get_adjoint(lbm_t *h, double *lam);

/* Use a caller-provided HIP stream (hipStream_t as void*; NULL = the
 * library's own default-priority stream). */
int lbm_set_stream(lbm_t *h, void *hip_stream);

/* Lattice tables for cross-checks: Q, D, e[i*D + a], w[i], M[k*Q + i]
 * (moment matrix).  Any output pointer may be NULL.  No GPU needed. */
int lbm_lattice_info(int lattice, int32_t *Q, int32_t *D, int8_t *e,
                     double *w, double *M);

/* Counts after lbm_set_geometry: fluid nodes and cut links. */
int lbm_counts(const lbm_t *h, int64_t *n_fluid, int64_t *n_links);

/* Average duration in milliseconds of the step kernel over the last
 * lbm_step() call of n >= 1 steps, from HIP events on the handle's stream
 * (timing enabled by lbm_set_timing(h, 1)). */
int lbm_set_timing(lbm_t *h, int on);
int lbm_last_step_ms(lbm_t *h, double *ms_per_step);

const char *lbm_last_error(const lbm_t *h);
int lbm_destroy(lbm_t *h);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
