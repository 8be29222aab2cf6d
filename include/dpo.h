/*
 * dpo.h — C ABI of libdpo.so, the MI355X (gfx950) semi-Lagrangian dynamic
 * programming library for planar low-thrust orbit transfer.
 *
 * Method: "Dynamic Programming Techniques for Planar Orbital Transfer of LEO
 * Satellites" (arXiv 2407.14675), Section 3.  The library computes the fixed
 * point of the semi-Lagrangian scheme eq:schema
 *
 *     v_j = min_f { dt*l(x_j,f) + exp(-lambda*dt) * I[V](x_j + dt*Phi(x_j,f)) }
 *
 * on a closed uniform 4-D grid, with I[V] the Q1 (multilinear) interpolation
 * and I[V](z) = M for feet outside the domain (state-constraint penalty,
 * paragraph "Grid and polar coordinates"), by value iteration and by policy
 * iteration (eq:p_eval, eq:p_impr), and evaluates the feedback eq:feed.
 *
 * Conventions (all entry points):
 *  - Every function returns int: DPO_OK (0), DPO_ENOCONV (1, output valid but
 *    the stop rule was not met), or a negative error.  Nothing aborts or
 *    throws across the ABI.  dpo_last_error() gives the message.
 *  - Array arguments are DEVICE pointers unless marked "host".  They are owned
 *    by the caller, must be contiguous and must stay valid until the work
 *    queued on `stream` has finished.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Sweeps are asynchronous on it; solvers synchronise it at residual checks.
 *  - Node arrays have N = n[0]*n[1]*n[2]*n[3] entries in C order
 *    [m][v_t][v_r][r]: axis 0 (r) fastest, axis 3 (m) slowest.
 *  - Value functions are float32; residuals and read-outs are float64.
 *  - One context must not be used from two threads at once.
 */
#ifndef DPO_H
#define DPO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DPO_OK = 0,
  DPO_ENOCONV = 1,   /* max sweeps / iterations reached; outputs hold the last iterate */
  DPO_EINVAL = -1,   /* invalid argument (null pointer, bad size, bad grid or search) */
  DPO_ENOMEM = -2,   /* device allocation failed */
  DPO_EHIP = -3,     /* a HIP runtime call failed */
  DPO_ENUMERIC = -4  /* a sweep produced a non-finite value */
};

enum { DPO_MODEL_ORBIT = 0, DPO_MODEL_EIKONAL = 1, DPO_MODEL_CROWN = 2 };

/* One-step approximation of the trajectory from a node (the foot point). */
enum { DPO_STEP_EULER = 0, DPO_STEP_HEUN = 1 };

enum {
  DPO_SEARCH_TABLE = 0,       /* coast + n_angles tabulated thrust angles (exhaustive) */
  DPO_SEARCH_SCAN_GOLDEN = 1, /* scan of n_scan angles, n_golden golden-section steps */
  DPO_SEARCH_SEEDED = 2,      /* local golden search around a per-node seed angle */
  DPO_SEARCH_TABLE_WALK = 3   /* the TABLE controls, searched by a walk from the previous optimum */
};

/* Node kinds reported by dpo_get_kind(). */
enum { DPO_KIND_FREE = 0, DPO_KIND_TARGET = 1, DPO_KIND_INACTIVE = 2 };

/* Closed uniform grid (paper Section 3, "Grid and polar coordinates"):
 * node i_k of axis k sits at lo[k] + i_k*(hi[k]-lo[k])/(n[k]-1).  Axis order
 * (r, v_r, v_t, m).  Requires 2 <= n[k] <= 256, lo[k] < hi[k] and at most
 * 2^30 nodes in total.  For DPO_MODEL_CROWN axis 3 is the polar angle theta
 * and is periodic ("closed with periodic conditions", Section 3): node i at
 * lo[3] + i*(hi[3]-lo[3])/n[3], hi[3] being lo[3]'s periodic image (2 pi
 * above it for an angle); feet wrap around along it and never leave the
 * domain there. */
typedef struct {
  int32_t n[4];
  double lo[4], hi[4];
} dpo_grid;

/* Problem (paper Section 2 and the polar system of Section 3):
 *  model ORBIT:   r' = v_r, v_r' = v_t^2/r - mu/r^2 + thr*(accel/m)*sin u,
 *                 v_t' = -v_r*v_t/r + thr*(accel/m)*cos u, m' = -mdot*thr;
 *  model EIKONAL: v_r' = thr*speed*sin u, v_t' = thr*speed*cos u (r, m fixed).
 *  model CROWN (the paper's Example 1, Section 4): state (r, v_r, v_t, theta)
 *                 with the orbit dynamics above for a constant thrust
 *                 acceleration accel (no mass), theta' = v_t/r, and the
 *                 running cost of eq:runcost_polar added to l below:
 *                 el_beta*(a - el_a)^2 + el_gamma*|e_vec - el_e*(cos el_omega,
 *                 sin el_omega)|^2, with a the vis-viva semi-major axis and
 *                 e_vec the eccentricity vector of the state (computed in FP64
 *                 per node at dpo_create).  The state constraint (I = M)
 *                 holds on the two circular faces r = lo[0], hi[0] only; a
 *                 foot beyond a v_r or v_t face is put on that face.  No
 *                 target set is implied: give an empty target box (negative
 *                 tgt_w).  Needs lo[0] > 0.
 *  The factorised sweep, the foot descriptors, the reduced-grid mask helper
 *  and the batched solver take the ORBIT and EIKONAL models only.
 *  Foot point x + dt*Phi(x, f) (eq:schema), the control held over the step:
 *  integrator DPO_STEP_EULER: Phi = b(x), one explicit Euler step;
 *  DPO_STEP_HEUN: Phi = (b(x) + b(x + dt*b(x)))/2, Heun's second-order
 *  Runge-Kutta step (the paper's choice, Section 3).  Under Heun the r and m
 *  cells of a thrust foot depend on the angle, so the factorised sweep and
 *  the foot descriptors do not apply: sweeps take the direct path, policy
 *  evaluation recomputes the foot from the stored angle, and the batched
 *  solver rejects the problem.
 *  Running cost l = w_time + w_fuel*thr; discount exp(-lambda*dt) (eq:cost).
 *  M: value of I[V] outside the domain and at inactive nodes.
 *  Target: nodes with |x_k - tgt_c[k]| <= tgt_w[k] + h_k/2 on every axis get
 *  V = 0 (use a huge tgt_w[k] for an unconstrained axis). */
typedef struct {
  int32_t model;
  double mu, accel, mdot, dt, lambda, w_time, w_fuel, M, speed;
  double tgt_c[4], tgt_w[4];
  int32_t integrator; /* DPO_STEP_EULER or DPO_STEP_HEUN */
  double el_beta, el_gamma, el_a, el_e, el_omega; /* DPO_MODEL_CROWN running cost (else unused) */
} dpo_problem;

/* Minimisation over the control set (paper Section 3, "Efficient computation
 * of the minimum"): tabulation, then golden-section refinement.
 *  TABLE:       controls = coast, u_k = -pi + 2*pi*k/n_angles (k < n_angles);
 *               first minimum in that order wins, coast wins exact ties.
 *  SCAN_GOLDEN: scan u_s = -pi + 2*pi*s/n_scan, then golden section with ratio
 *               (sqrt5-1)/2 on [u_s* - 2*pi/n_scan, u_s* + 2*pi/n_scan]: two
 *               interior evaluations then one per step (n_golden steps); the
 *               best evaluated angle is the thrust candidate; thrust is chosen
 *               iff its Q is strictly below the coast Q.
 *  SEEDED:      golden section on [seed - local_half_width, seed + local_half_width]
 *               with n_local evaluations in total, then coast; a node whose best
 *               Q differs from its current value by more than
 *               fallback_tol*max(1,|V|) repeats the SCAN_GOLDEN search.
 *  TABLE_WALK:  the TABLE controls, searched as in Section 3 ("Efficient
 *               computation of the minimum") after the first iteration: start
 *               at the table angle nearest to the node's previous optimum,
 *               look at both cyclic neighbours, move to the lower one if it is
 *               strictly below (the lower-index side on a tie between them),
 *               then keep moving the same way while the next angle is strictly
 *               lower; thrust iff the walk's Q is strictly below coast.  The
 *               walk stops on any local minimiser of the table, including a
 *               plateau of equal values.  Where no previous optimum exists
 *               (the first sweep of a solve) the full table is searched.
 *  Limits: 1 <= n_angles <= 1024; 8 <= n_scan <= 1024; 0 <= n_golden <= 64. */
typedef struct {
  int32_t mode, n_angles, n_scan, n_golden, n_local;
  double local_half_width, fallback_tol;
} dpo_search;

/* Solver statistics (all counts since the call started). */
typedef struct {
  int64_t sweeps;         /* Bellman sweeps with full search (VI sweeps or PI greedy steps) */
  int64_t eval_sweeps;    /* frozen-policy sweeps */
  int64_t evals;          /* node-control Q evaluations (TABLE_WALK: counted by the sweeps) */
  int64_t fallback_nodes; /* SEEDED: nodes that repeated the full search */
  int64_t verify_steps;   /* seeded policy iteration: full-search greedy steps after the first */
  double resid_max_rel;   /* last max |dV|/max(1,|V|) over free nodes (FP64) */
  double resid_sum_abs;   /* last sum |dV| (FP64) */
  double resid_max_abs;   /* last max |dV| (FP64) */
  double seconds;         /* wall time from the first launch to the stop decision */
  int32_t stalled;        /* 1 if stopped because the residual stopped decreasing */
  int32_t converged;      /* 1 if the stop rule was met */
  /* modified policy iteration (dpo_solve_pi with eval_sweeps >= 0; 0 elsewhere):
   * device time of the greedy sweeps and of the counted evaluation sweeps,
   * from HIP events recorded on the solver's stream around each step's greedy
   * sweep and around its run of evaluation sweeps */
  double greedy_seconds;
  double eval_seconds;
} dpo_stats;

typedef struct dpo_ctx dpo_ctx;

/* ---------------------------------------------------------------- set-up */

/* Create a context: copies *grid, *prob and *search; classifies every node
 * (target / inactive / free) on the device in FP64 and compacts the free
 * nodes into an index list (the reduced grid of Section 3).  active_mask is a
 * DEVICE u8[N] (nonzero = active) or NULL for "all nodes active".  Runs on
 * the null stream and synchronises.  *out is NULL on error. */
int dpo_create(const dpo_grid* grid, const dpo_problem* prob, const dpo_search* search,
               const uint8_t* active_mask, dpo_ctx** out);

/* Destroy a context and free its device scratch.  NULL is ignored. */
void dpo_destroy(dpo_ctx* ctx);

/* Message of the last error on ctx, or of the calling thread when ctx is NULL. */
const char* dpo_last_error(const dpo_ctx* ctx);

/* Sizes: total nodes N and free (swept) nodes. */
int dpo_sizes(const dpo_ctx* ctx, int64_t* n_nodes, int64_t* n_free);

/* Copy the node kinds (DPO_KIND_*) into a device u8[N]. */
int dpo_get_kind(dpo_ctx* ctx, uint8_t* kind, void* stream);

/* Kernel path of the Bellman sweeps: 0 = automatic, 1 = direct (every
 * evaluation gathers its 16 corners), 2 = factorised (thrust feet share their
 * r and m cells, so each node collapses its neighbourhood over r and m once;
 * applies when every thrust foot stays within two cells along v_r and v_t and
 * one cell along m).  Both give the same Q1 values up to rounding order.
 * Returns DPO_EINVAL for 2 where it does not apply. */
int dpo_set_kernel_path(dpo_ctx* ctx, int32_t path);

/* Workgroup size of the factorised sweeps (64, 128, ..., 512; default 256). */
int dpo_set_block(dpo_ctx* ctx, int32_t block);

/* The path the sweeps take now: 1 direct, 2 factorised (negative on error). */
int dpo_kernel_path(const dpo_ctx* ctx);

/* Algorithmic bytes of one dpo_policy_eval_sweep_last on ctx (*bytes, host):
 * per free node the value written and its share of the value array read
 * (4 + 4), plus the per-node stream of the foot descriptors: 16 bytes per free
 * node (packed coordinates, 32-bit cell code, two cell coordinates); 14 with
 * the compact 16-bit code, used when every foot stays within 31 cells of its
 * node along v_r and v_t; or, when at least half of the nodes are free, 8
 * per node, free or fixed (one packed descriptor per node: the compact code
 * and the two cell coordinates rounded to multiples of 2^-24 of a cell, no
 * coordinate list). */
int dpo_eval_sweep_bytes(const dpo_ctx* ctx, int64_t* bytes);

/* Replace the search settings (same rules as in dpo_create). */
int dpo_set_search(dpo_ctx* ctx, const dpo_search* search);

/* V := 0 at target nodes, M elsewhere (the initial guess of value iteration
 * and the fixed values every sweep relies on).  V is a device float[N]. */
int dpo_init_value(dpo_ctx* ctx, float* V, void* stream);

/* ---------------------------------------------------------------- sweeps */

/* One Jacobi Bellman sweep with full search (eq:schema / eq:p_impr):
 * for every free node writes V_out, the best thrust angle pol_angle (radians
 * in [-pi, pi)) and pol_thr (1 = thrust).  Target and inactive nodes are not
 * written: V_out must already hold their fixed values (dpo_init_value or a
 * copy of V_in).  V_in and V_out must not overlap.  If resid is not NULL it
 * receives (device double[5]) max|dV|/max(1,|V_out|), sum|dV|, max|dV|, the
 * count of non-finite outputs and the count of seeded-search fallbacks (for
 * TABLE_WALK: the walks' thrust evaluations),
 * accumulated over the free nodes in FP64 in a fixed order.  pol_angle /
 * pol_thr may be NULL.  SEEDED mode needs dpo_bellman_sweep_seeded instead.
 * TABLE_WALK: pol_angle is required and read on entry: each node's walk
 * starts at the table angle nearest to its entry (a non-finite entry starts
 * at index 0), and the entry is then overwritten with the walk's result. */
int dpo_bellman_sweep(dpo_ctx* ctx, const float* V_in, float* V_out, float* pol_angle,
                      uint8_t* pol_thr, double* resid, void* stream);

/* SEEDED sweep: seed_angle is a device float[N] of proposed thrust angles.
 * Nodes failing the fallback test repeat the SCAN_GOLDEN search; their count
 * is resid[4].  On the factorised path the full searches of sparse fallback
 * nodes run in a second launch over a list built with atomics, so resid[1]
 * (the FP64 sum) may differ between runs in its last bits; values, policy
 * and the other residual entries are deterministic. */
int dpo_bellman_sweep_seeded(dpo_ctx* ctx, const float* V_in, float* V_out, float* pol_angle,
                             uint8_t* pol_thr, const float* seed_angle, double* resid,
                             void* stream);

/* One frozen-policy sweep (eq:p_eval applied once): Q of the stored control
 * at every free node.  Same fixed-node and resid rules as dpo_bellman_sweep. */
int dpo_policy_eval_sweep(dpo_ctx* ctx, const float* V_in, float* V_out, const float* pol_angle,
                          const uint8_t* pol_thr, double* resid, void* stream);

/* Kernels of the frozen-policy sweeps: 0 automatic, 1 corner gathers from
 * global memory (one node per thread over the free list, or per node from
 * the greedy step's foot descriptors), 2 every node of the grid, workgroups
 * walking columns of nodes through the mass planes with the value bricks
 * their feet reach staged in LDS (orbit model, Euler foot, a thrust step
 * below one mass cell; DPO_EINVAL otherwise).  Automatic takes 2 for the
 * descriptor sweeps of policy iteration (and dpo_policy_eval_sweep_last)
 * where the descriptors are stored per node, and 1 for the sweeps that take
 * the policy arrays (dpo_policy_eval_sweep and its static form), where
 * recomputing the foot makes the brick kernel arithmetic-bound; 2 forces
 * the bricks for both.  Each pair of kernels gives the same values bit for
 * bit.  dpo_eval_path returns the kernel policy iteration's evaluation
 * sweeps use (1 or 2). */
int dpo_set_eval_path(dpo_ctx* ctx, int32_t path);
int dpo_eval_path(const dpo_ctx* ctx);

/* Frozen-policy sweep for the policy chosen by the most recent
 * dpo_bellman_sweep / dpo_bellman_sweep_seeded on this context: the sweep
 * stores, per free node, the cell and cell coordinates of its chosen
 * control's foot, so this sweep is one descriptor load, 16 gathers and 15
 * lerps per node (the evaluation sweep of policy iteration, eq:p_eval).
 * Where the descriptors are stored per node (dpo_eval_sweep_bytes) the two
 * cell coordinates along v_r and v_t are kept to the nearest multiple of
 * 2^-24 of a cell, so the sweep reproduces the Bellman sweep's Q of the
 * chosen control up to 2^-25 of the differences between neighbouring
 * values (below the rounding of the float32 interpolation itself).
 * Same fixed-node rule as dpo_bellman_sweep; no residual.  DPO_EINVAL if no
 * Bellman sweep has run on ctx, or for the Heun foot (descriptors need the
 * Euler step). */
int dpo_policy_eval_sweep_last(dpo_ctx* ctx, const float* V_in, float* V_out, void* stream);

/* dpo_policy_eval_sweep for callers that cannot allocate device memory (code
 * under stream or graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, bit for bit, but the
 * residual's per-workgroup partials and its two-stage reduction use a
 * static device array of 10,496,000 bytes that each GPU holds from the first
 * call on it until the process ends; the call itself allocates nothing (the
 * context was allocated by dpo_create beforehand).  At most 67,108,864 free
 * nodes (DPO_EINVAL beyond).  All calls on one GPU share that array: calls
 * that overlap in time on one GPU (different streams, or host threads) race
 * on it and must be serialised by the caller; consecutive calls on one
 * stream are safe.  With no free node, resid (if given) is written by a
 * kernel, not a memset. */
int dpo_policy_eval_sweep_static(dpo_ctx* ctx, const float* V_in, float* V_out, const float* pol_angle,
                                 const uint8_t* pol_thr, double* resid, void* stream);

/* --------------------------------------------------------------- solvers */

/* Value iteration (paper Section 3, "Policy Iteration", first display):
 * V <- T V from the given V (initialise with dpo_init_value) until the
 * relative residual max|dV|/max(1,|V|) < tol_rel, checked every check_every
 * sweeps, or until it has not decreased for 64 checks (stalled).  Returns
 * DPO_ENOCONV after max_sweeps.  V, pol_angle, pol_thr: device, N entries.
 * TABLE_WALK: the first sweep searches the full table, every later sweep
 * walks from the previous sweep's angles.
 * Accuracy: tol_rel bounds the one-step change, not the distance to the
 * fixed point, which is larger by the number of sweeps over which the
 * slowest mode of the iteration carries a change (on the undiscounted orbit
 * workloads a 1e-6 stop lies 1e-4 to 3e-3 from the fixed point).  Carry a
 * solve on with dpo_solve_pi to 3e-7, which float32 meets or stalls at, for
 * a value within ~2e-5 of the fixed point. */
int dpo_solve_vi(dpo_ctx* ctx, float* V, float* pol_angle, uint8_t* pol_thr, double tol_rel,
                 int64_t max_sweeps, int32_t check_every, dpo_stats* stats, void* stream);

/* Modified policy iteration (eq:p_impr then eq:p_eval by eval_sweeps
 * frozen-policy sweeps): stops when the residual of the greedy step is below
 * tol_rel; V then holds T V and the policy its argmin.  From the second
 * greedy step on, a node keeps its current control unless the search finds a
 * strictly smaller Q (the search is only approximately the argmin; this keeps
 * the iterates from alternating between nearly tied controls).  A step's
 * evaluation sweeps are queued before its residual is read back, and are
 * discarded if the step meets the stop rule.  seed_angle (device,
 * nullable) enables the SEEDED greedy step for every outer iteration after the
 * first, until a seeded step meets tol_rel or 8 seeded steps in a row bring
 * no new lowest residual; from then on the greedy steps
 * use the full search again (SCAN_GOLDEN parameters of the context's search)
 * and the solve stops at the first full step that meets tol_rel, so the
 * result is certified by the same rule as an unseeded solve.  seed_angle may
 * be pol_angle itself (each node reads its seed before its angle is
 * overwritten), which warm-starts every node from its previous optimum as in
 * paper Section 3, "Efficient computation of the minimum".
 * TABLE_WALK: the first greedy step searches the full table, later ones walk
 * from the current policy's angles (the incumbent rule applies as above).
 * eval_sweeps < 0: the policy iteration of Section 3 with eq:p_eval solved
 * exactly: after every greedy step that does not stop the solve, the new
 * policy is evaluated by dpo_policy_evaluate to a node-wise relative
 * residual of 5e-7 (at most 300 operator applications), starting from the
 * greedy values;
 * stats->eval_sweeps counts the operator applications.  Needs lambda > 0
 * and the TABLE or SCAN_GOLDEN search; no seed_angle.
 * Returns DPO_ENOCONV after max_outer greedy steps, or when 32 full-search
 * greedy steps in a row bring no new lowest residual (stats->stalled).
 * Accuracy as for dpo_solve_vi.  A seeded solve carried on to a tighter
 * tolerance starts with seeded steps again, which drift towards the local
 * search's own fixed point: carry it on without seed_angle. */
/* Exact policy evaluation (eq:p_eval solved as the sparse linear system
 * (I - exp(-lambda dt) P) v = b of Section 3, by restarted GMRES(8), the
 * solver the paper names): V (device, N) holds the fixed nodes' values and,
 * at free nodes, the initial guess on entry and the solution on exit; the
 * frozen policy is pol_angle / pol_thr.  The operator is applied matrix-free
 * by the frozen-policy sweep without its affine part; vectors are float32,
 * dot products FP64 in a fixed order.  Stops when the node-wise relative
 * residual max_j |b - A v|_j / max(1, |v_j|) <= tol_rel (checked between
 * restart cycles; a cycle ends after 8 steps or once its 2-norm residual
 * has fallen 100-fold) or after max_iter operator applications
 * (DPO_ENOCONV, V holds the last iterate).  *matvecs and
 * *resid_rel (host, nullable): operator applications and the final
 * relative residual.  Needs lambda > 0 (undiscounted, a policy whose chains
 * never leave the free set makes the system singular).  Synchronises. */
int dpo_policy_evaluate(dpo_ctx* ctx, float* V, const float* pol_angle, const uint8_t* pol_thr, double tol_rel,
                        int32_t max_iter, int64_t* matvecs, double* resid_rel, void* stream);

int dpo_solve_pi(dpo_ctx* ctx, float* V, float* pol_angle, uint8_t* pol_thr, double tol_rel,
                 int32_t eval_sweeps, int64_t max_outer, const float* seed_angle,
                 dpo_stats* stats, void* stream);

/* ----------------------------------------------------- read-out, feedback */

/* FP64 Q1 read-out of the float V at one physical state x (host double[4]);
 * *out (host) = M outside the domain.  Synchronises stream. */
int dpo_value_at(dpo_ctx* ctx, const float* V, const double* x, double* out, void* stream);

/* Approximate optimal feedback eq:feed at n arbitrary states (device
 * double[n*4]) with time step tau, using the context's search (TABLE or
 * SCAN_GOLDEN; TABLE_WALK searches its full table) and integrator: best
 * thrust angle, throttle, and the minimal Q (q_out nullable). */
int dpo_extract_feedback(dpo_ctx* ctx, const float* V, const double* states, int64_t n,
                         double tau, float* angle_out, uint8_t* thr_out, float* q_out,
                         void* stream);

/* Closed loop (paper Section 3, eq:feed, and the simulations of Section 4):
 * from each of n states (device double[n*4], updated in place), `steps`
 * times: the feedback of dpo_extract_feedback at the current state with time
 * step tau, then `substeps` classical fourth-order Runge-Kutta steps of
 * length tau/substeps of the simulated system in FP64 with that control
 * held.  The simulated system is the model's own dynamics plus, when drag >
 * 0, the aerodynamic drag of Section 4's Example 2: an acceleration of
 * magnitude drag * |v|^2 opposite to the velocity (v_r, v_t), drag in 1 /
 * (the grid's length unit); V and the feedback stay those of the model
 * without it.  drag must be 0 for DPO_MODEL_EIKONAL.  One device thread
 * follows each trajectory for all its steps.
 * Histories (device, nullable), step-major so that a step's writes are
 * contiguous: traj double[(steps+1)*n*4] (the states before every step and
 * after the last), thr_hist u8[steps*n], ang_hist float[steps*n].
 * Asynchronous on stream.  Limits: 0 <= n < 2^31 - 256, steps >= 0,
 * 1 <= substeps <= 4096, tau > 0, drag >= 0 and finite; SEEDED search is
 * refused. */
int dpo_simulate(dpo_ctx* ctx, const float* V, double* states, int64_t n, double tau, int32_t steps,
                 int32_t substeps, double drag, double* traj, uint8_t* thr_hist, float* ang_hist,
                 void* stream);

/* Reachability mask for a reduced grid: for every node of `fine` (same
 * domain box as ctx), keep = (FP64 Q1 value of the coarse V at the node <
 * thresh), then box-dilated by dilate[k] cells along axis k.  mask: device
 * u8[N_fine].  Synchronises stream. */
int dpo_mask_from_coarse(dpo_ctx* coarse, const float* V_coarse, const dpo_grid* fine,
                         double thresh, const int32_t* dilate, uint8_t* mask, void* stream);

/* ---------------------------------------------------------------- probes */

/* Q1 interpolation (the sweep's device function) at n points given in grid
 * coordinates (device float[n*4]); out: device float[n]; M outside. */
int dpo_probe_interp(dpo_ctx* ctx, const float* V, const float* s, int64_t n, float* out,
                     void* stream);

/* Q(x_j, f) of eq:schema for n (node, control) pairs: nodes (device int32[n],
 * flat indices), thr (device u8[n]), angle (device float[n]); q_out device
 * float[n].  The node indices are copied to the host and range-checked first
 * (blocking), so out-of-range indices give DPO_EINVAL. */
int dpo_probe_q(dpo_ctx* ctx, const float* V, const int32_t* nodes, const uint8_t* thr,
                const float* angle, int64_t n, float* q_out, void* stream);

/* Foot displacement of n (node, control) pairs in cells per axis (device
 * float[n*4]): s_k - i_k as used by the sweep. */
int dpo_probe_foot(dpo_ctx* ctx, const int32_t* nodes, const uint8_t* thr, const float* angle,
                   int64_t n, float* off_out, void* stream);

/* Machine ceilings, the measured denominators of the sweeps' rooflines (the
 * published peaks are reported beside them).  Asynchronous on stream; the
 * caller times them with events.
 * dpo_probe_copy: dst[0..n) = src[0..n) with 16-byte loads and stores (both
 *   device, 16-byte aligned, n a positive multiple of 4): 8n bytes of HBM
 *   traffic when n is far above the last-level cache.
 * dpo_probe_read: reads src[0..n) (the same constraints); sink (device
 *   float[1]) is written only for data that holds -1e38.
 * dpo_probe_fma: blocks x 256 threads, each issuing iters x 8 dependent-free
 *   FP32 fused multiply-adds (plain v_fma_f32, no packed form): 16 * 256 *
 *   blocks * iters flops; sink as above. */
int dpo_probe_copy(const float* src, float* dst, int64_t n, void* stream);
int dpo_probe_read(const float* src, int64_t n, float* sink, void* stream);
int dpo_probe_fma(int32_t blocks, int32_t iters, float* sink, void* stream);

/* ------------------------------------------------------------ batched solve */

/* Many transfer problems solved together by value iteration (paper Section 3):
 * each sweep is ONE kernel launch over the tiles of every problem still
 * running.  S sweeps and a per-problem FP64 stop decision on the last sweep's
 * relative residual max|dV|/max(1,|V|) < tol_rel are captured into one
 * hipGraph and replayed, with one host synchronisation per replay; when a
 * problem stops, the graph is re-captured over the remaining ones.  Sweep
 * counts are therefore multiples of S.  Each problem gets its own grid and physics; the search
 * (TABLE or SCAN_GOLDEN) is shared, and the factorised sweep must apply to
 * every problem (so the Euler foot only). */
typedef struct dpo_batch dpo_batch;

typedef struct {
  int64_t sweeps;        /* sweeps until this problem stopped */
  double resid_max_rel;  /* its last residual (FP64) */
  double resid_sum_abs;
  double resid_max_abs;
  int32_t converged;     /* 1 if stopped by the tolerance */
  int32_t status;        /* 0 running at the end, 1 converged, 2 non-finite values */
} dpo_batch_stats;

/* Create: grids, probs are host arrays of n_prob entries (copied). */
int dpo_batch_create(int32_t n_prob, const dpo_grid* grids, const dpo_problem* probs, const dpo_search* search,
                     dpo_batch** out);
void dpo_batch_destroy(dpo_batch* b);
const char* dpo_batch_last_error(const dpo_batch* b);

/* Node and free-node counts per problem (host int64[n_prob], nullable). */
int dpo_batch_sizes(const dpo_batch* b, int64_t* n_nodes, int64_t* n_free);

/* V: host array of n_prob device pointers, each float[N_p]; V[p] := 0 on its
 * target nodes, M elsewhere. */
int dpo_batch_init_value(dpo_batch* b, float* const* V, void* stream);

/* Value iteration of all problems from the given V (in/out, host array of
 * device pointers).  pol_angle / pol_thr: host arrays of device pointers, or
 * NULL.  sweeps_per_graph: even, 2..256; block: 64..512 (multiple of 64).
 * stats: host array of n_prob (nullable); *seconds: wall time (nullable).
 * Synchronises `stream` first and runs on the batch's own stream.  Returns
 * DPO_ENOCONV if some problem did not converge within max_sweeps. */
int dpo_batch_solve_vi(dpo_batch* b, float* const* V, float* const* pol_angle, uint8_t* const* pol_thr, double tol_rel,
                       int64_t max_sweeps, int32_t sweeps_per_graph, int32_t block, dpo_batch_stats* stats,
                       double* seconds, void* stream);

/* The same problems solved one after another by dpo_solve_vi (reference for
 * the batched form); same arguments as dpo_batch_solve_vi plus check_every. */
int dpo_batch_solve_sequential(dpo_batch* b, float* const* V, float* const* pol_angle, uint8_t* const* pol_thr,
                               double tol_rel, int64_t max_sweeps, int32_t check_every, dpo_batch_stats* stats,
                               double* seconds, void* stream);

/* Autotuning probe: seconds per batched sweep for (block, sweeps_per_graph),
 * timed over `replays` graph replays on scratch buffers (the solve's data is
 * not touched). */
int dpo_batch_time_config(dpo_batch* b, int32_t block, int32_t sweeps_per_graph, int32_t replays,
                          double* seconds_per_sweep);

/* ------------------------------------------------- learned control proposal */

/* A 4 -> 128 -> 128 -> 3 perceptron (exact erf GELU after each hidden layer)
 * from a node's grid position, scaled to [-1, 1] per axis as
 * 2*i_k/(n_k-1) - 1, to (cos u, sin u, throttle logit).  Its angle seeds the
 * SEEDED search (the learned form of the warm-started minimisation of paper
 * Section 3, "Efficient computation of the minimum"); the paper itself has no
 * network, so every choice below is this library's.
 *  Parameters: float32[DPO_MLP_PARAMS] in the order W1[128][4], b1[128],
 *  W2[128][128], b2[128], W3[3][128], b3[3] (row = output unit).  The middle
 *  layer runs on the matrix cores with bfloat16 operands (h1 and W2 forward;
 *  delta2, h1 and W2 backward, rounded to nearest even) and float32
 *  accumulation; everything else is float32.
 *  Loss of a sample with target (c*, s*, t*), t* in {0, 1}:
 *      t* ((c - c*)^2 + (s - s*)^2) + BCE(logit, t*),   mean over the batch.
 *  Training: Adam (default lr 1e-3, betas 0.9 / 0.999, eps 1e-8), FP32
 *  moments, bias-corrected with the network's own step count.
 *  Samples x are float32[n][4] (16-byte aligned), targets float32[n][4]
 *  (c*, s*, t*, unused). */
#define DPO_MLP_PARAMS 17539
typedef struct dpo_mlp dpo_mlp;

/* Create with the given parameters (host, nullable = zeros); Adam state zero. */
int dpo_mlp_create(const float* params, dpo_mlp** out);
void dpo_mlp_destroy(dpo_mlp* m);
const char* dpo_mlp_last_error(const dpo_mlp* m);
/* Host copies in/out; set_params also clears the Adam state and step count.
 * Both synchronise the device. */
int dpo_mlp_set_params(dpo_mlp* m, const float* params);
int dpo_mlp_get_params(dpo_mlp* m, float* params);
/* Gradient of the last dpo_mlp_grad / dpo_mlp_train batch (host float[P]). */
int dpo_mlp_get_grad(dpo_mlp* m, float* grad);
int dpo_mlp_set_adam(dpo_mlp* m, double lr, double beta1, double beta2, double eps);
/* Adam steps taken since the last set_params. */
int64_t dpo_mlp_steps(const dpo_mlp* m);

/* y (device float[n][3]) = network(x). */
int dpo_mlp_forward(dpo_mlp* m, const float* x, int64_t n, float* y, void* stream);

/* Gradient of the mean loss over the n samples (1 <= n <= 65536) into grad
 * (device float[P], nullable) and the mean loss into *loss (device, nullable);
 * parameters are not changed. */
int dpo_mlp_grad(dpo_mlp* m, const float* x, const float* tgt, int64_t n, float* grad, float* loss,
                 void* stream);

/* One epoch: ceil(n/batch) Adam steps over the samples in the order perm
 * (host int32[n] of indices in [0, n), checked; NULL = 0..n-1), batch b taking
 * positions [b*batch, min(n, (b+1)*batch)).  loss_hist (device
 * float[ceil(n/batch)], nullable) receives each batch's mean loss before its
 * step.  1 <= batch <= 65536.  Asynchronous on stream: perm is copied into
 * the context before the call returns (the caller may reuse it at once), and
 * the call waits only for the previous call's copy of its order. */
/* Ordering: the asynchronous network calls (forward, grad, train, propose)
 * may be issued on different streams; each makes its stream wait, on the
 * device, for the work the previous such call queued on the same network. */
int dpo_mlp_train(dpo_mlp* m, const float* x, const float* tgt, int64_t n, const int32_t* perm, int32_t batch,
                  float* loss_hist, void* stream);

/* Seed angles atan2(s, c) of the network at every free node of ctx, written
 * to seed_angle[j] (device float[N]; other entries untouched), for
 * dpo_bellman_sweep_seeded and dpo_solve_pi. */
int dpo_mlp_propose(dpo_mlp* m, const dpo_ctx* ctx, float* seed_angle, void* stream);

/* Ordered list (node order) of the free nodes with V < thresh, as packed grid
 * coordinates i0 | i1<<8 | i2<<16 | i3<<24 into nodes (device u32, capacity
 * n_free); *n_out (host) = their count.  Synchronises stream. */
int dpo_feasible_nodes(dpo_ctx* ctx, const float* V, double thresh, uint32_t* nodes, int64_t* n_out,
                       void* stream);

/* Training pairs from a policy: for t < n, node = nodes[sel[t]] (sel: host
 * int32[n], checked against [0, n_nodes)); x[t] = the node's scaled position,
 * tgt[t] = (cos, sin) of pol_angle at the node and its throttle (0/1).
 * Synchronises stream. */
int dpo_gather_pairs(dpo_ctx* ctx, const uint32_t* nodes, int64_t n_nodes, const int32_t* sel, int64_t n,
                     const float* pol_angle, const uint8_t* pol_thr, float* x, float* tgt, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DPO_H */
