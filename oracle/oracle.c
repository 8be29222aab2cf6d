/*
 * Plain, slow, single-threaded CPU oracle for the semi-Lagrangian dynamic
 * programming scheme of "Dynamic Programming Techniques for Planar Orbital
 * Transfer of LEO Satellites" (arXiv 2407.14675).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path calls, links or
 * loads this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the device library.
 *
 * Arithmetic is in `real`, which is double unless ORACLE_FLOAT is defined
 * (the float build exists only to measure what single precision alone costs).
 * Residuals and sums are always accumulated in double.
 *
 * What it computes (Section 3 of the paper):
 *   - the fixed-point scheme eq:schema: for every grid node x_j
 *       v_j = min_f { dt*l(x_j,f) + exp(-lambda*dt) * I[V](x_j + dt*Phi(x_j,f)) }
 *     with I[V] the tensor-product (Q1) interpolation of the nodal values and
 *     I[V](z) = M for z outside the domain (state-constraint penalty,
 *     paragraph "Grid and polar coordinates");
 *   - value iteration (paragraph "Policy Iteration", first display);
 *   - policy iteration, eq:p_eval then eq:p_impr, with the evaluation done by
 *     a fixed number of frozen-policy sweeps (modified policy iteration);
 *   - the minimisation by tabulation and golden-section refinement
 *     (paragraph "Efficient computation of the minimum"), and a seeded local
 *     golden search with the full search as fallback (the warm-started
 *     minimisation of the same paragraph, with the seed given per node);
 *   - the approximate feedback eq:feed, and the closed loop that applies it
 *     to the model integrated by the classical fourth-order Runge-Kutta
 *     method (Section 4's simulations).
 *
 * Pins (tests): exact multilinear reproduction, Euler defects in closed
 * form, the Heun step's third-order local error against an accurate ODE
 * integration, the eikonal closed form, monotonicity and contraction,
 * VI = PI, brute-force enumeration of the control, and the walk's result a
 * local minimiser of the full table that equals its global minimiser where
 * the table is unimodal.  Parity unpinned: the converged
 * value function of the orbit problems has no closed form and is pinned only
 * through those parts.
 *
 * Problem instance (nondimensional, mu = 1): state x = (r, v_r, v_t, m),
 *   r'   = v_r
 *   v_r' = v_t^2/r - mu/r^2 + thr*(a/m)*sin u
 *   v_t' = -v_r*v_t/r       + thr*(a/m)*cos u
 *   m'   = -c*thr
 * (the polar system of Section 3 with the angle measured from the tangential
 * direction, the cyclic angle theta dropped and mass added; the centrifugal
 * term carries a plus sign, which is the physically correct one).  The foot
 * point is one explicit Euler step, or one Heun (second-order Runge-Kutta)
 * step, the scheme the paper itself uses.  A second model, a 2-D minimum-time
 * eikonal x' = s*(sin u, cos u) in axes (v_r, v_t), exists to pin the scheme
 * against a closed form.
 *
 * Grid: closed uniform tensor grid, node i_k at lo_k + i_k*h_k with
 * h_k = (hi_k - lo_k)/(n_k - 1); storage is C order [m][v_t][v_r][r].
 * The crown problem (model 2, the paper's Example 1: polar grid "closed with
 * periodic conditions", Section 3) has theta as axis 3 instead of the mass:
 * node i at lo + i*h with h = (hi - lo)/n (hi is lo's periodic image), and
 * interpolation wraps around along that axis, which never leaves the domain.
 * The foot is expressed in grid coordinates, s_k = i_k + dt*b_k/h_k, which
 * is the same point as (z_k - lo_k)/h_k but exact for a zero displacement.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_FLOAT
typedef float real;
#else
typedef double real;
#endif

#define OR_PI 3.14159265358979323846

typedef struct {
  int32_t n[4];
  double lo[4], hi[4];
  int32_t model; /* 0 = planar orbit, 1 = 2-D eikonal in axes (v_r, v_t),
                    2 = the crown problem: planar orbit in axes (r, v_r, v_t, theta)
                        with theta periodic, constant thrust, orbital-element cost */
  double mu, accel, mdot, dt, lambda, w_time, w_fuel, M, speed;
  double tgt_c[4], tgt_w[4];
  int32_t integrator; /* foot point: 0 = one explicit Euler step, 1 = Heun (RK2) */
  /* model 2 running cost: beta*(a - a_bar)^2 + gamma*|e_vec - e_bar_vec|^2 */
  double el_beta, el_gamma, el_a, el_e, el_omega;
} or_problem;

typedef struct {
  int32_t mode; /* 0 = discrete table of n_angles thrust angles plus coast,
                   1 = scan of n_scan angles, golden-section refinement,
                   2 = seeded: golden section around a given angle, with the
                       mode-1 search as fallback,
                   3 = the mode-0 table searched by a walk from the previous
                       optimum (mode 0 where no previous optimum exists) */
  int32_t n_angles, n_scan, n_golden;
  int32_t n_local;         /* mode 2: thrust evaluations of the local search */
  double local_half_width; /* mode 2: half-width of its bracket (rad) */
  double fallback_tol;     /* mode 2: relative change that triggers the fallback */
} or_search;

enum { KIND_FREE = 0, KIND_TARGET = 1, KIND_INACTIVE = 2 };

/* ------------------------------------------------------------------ grid */
static int periodic(const or_problem *p, int k) { return k == 3 && p->model == 2; }

static double step(const or_problem *p, int k) {
  if (periodic(p, k)) return (p->hi[k] - p->lo[k]) / (double)p->n[k];
  return (p->hi[k] - p->lo[k]) / (double)(p->n[k] - 1);
}

static int64_t n_total(const or_problem *p) {
  return (int64_t)p->n[0] * p->n[1] * p->n[2] * p->n[3];
}

static void node_index(const or_problem *p, int64_t j, int i[4]) {
  for (int k = 0; k < 4; k++) {
    i[k] = (int)(j % p->n[k]);
    j /= p->n[k];
  }
}

static int64_t flat_index(const or_problem *p, const int i[4]) {
  return (((int64_t)i[3] * p->n[2] + i[2]) * p->n[1] + i[1]) * p->n[0] + i[0];
}

static void node_coords(const or_problem *p, const int i[4], real x[4]) {
  for (int k = 0; k < 4; k++) x[k] = (real)(p->lo[k] + i[k] * step(p, k));
}

/* Fixed sets.  Target nodes: every node within the target box enlarged by
 * half a cell on each constrained axis (nearest-node snapping of the box);
 * V = 0 there.  Inactive nodes: mask[j] == 0; V = M there (nodes dropped
 * from the reduced grid behave as outside the domain).  Target wins. */
void or_classify(const or_problem *p, const uint8_t *mask, uint8_t *kind) {
  int64_t N = n_total(p);
  for (int64_t j = 0; j < N; j++) {
    int i[4];
    node_index(p, j, i);
    int target = 1;
    for (int k = 0; k < 4; k++) {
      double x = p->lo[k] + i[k] * step(p, k);
      if (!(fabs(x - p->tgt_c[k]) <= p->tgt_w[k] + 0.5 * step(p, k))) target = 0;
    }
    if (target) kind[j] = KIND_TARGET;
    else if (mask && !mask[j]) kind[j] = KIND_INACTIVE;
    else kind[j] = KIND_FREE;
  }
}

void or_init_value(const or_problem *p, const uint8_t *kind, real *V) {
  int64_t N = n_total(p);
  for (int64_t j = 0; j < N; j++) V[j] = (kind[j] == KIND_TARGET) ? (real)0 : (real)p->M;
}

/* ------------------------------------------------------------- dynamics */
/* Right-hand side b(x, f) for throttle thr in {0,1} and thrust angle u. */
static void rhs(const or_problem *p, const real x[4], int thr, real u, real b[4]) {
  if (p->model == 2) {
    /* the paper's polar system (Section 3) with the centrifugal term's sign
     * corrected, thrust of constant acceleration `accel` split radial sin u,
     * tangential cos u, and theta' = v_t / r */
    real r = x[0], vr = x[1], vt = x[2];
    real acc = thr ? (real)p->accel : (real)0;
    b[0] = vr;
    b[1] = vt * vt / r - (real)p->mu / (r * r) + acc * (real)sin(u);
    b[2] = -vr * vt / r + acc * (real)cos(u);
    b[3] = vt / r;
    return;
  }
  if (p->model == 1) {
    real s = thr ? (real)p->speed : (real)0;
    b[0] = 0;
    b[1] = s * (real)sin(u);
    b[2] = s * (real)cos(u);
    b[3] = 0;
    return;
  }
  real r = x[0], vr = x[1], vt = x[2], m = x[3];
  real acc = thr ? (real)p->accel / m : (real)0;
  b[0] = vr;
  b[1] = vt * vt / r - (real)p->mu / (r * r) + acc * (real)sin(u);
  b[2] = -vr * vt / r + acc * (real)cos(u);
  b[3] = -(real)p->mdot * (real)thr;
}

/* Mean slope of the one-step approximation of the trajectory from x over a
 * step tau with the control held fixed (Section 3: the foot point
 * x + tau*Phi(x, f) of eq:schema).  Euler: Phi = b(x).  Heun, the
 * second-order Runge-Kutta method the paper names: Phi = (b(x) + b(x~))/2
 * with the Euler predictor x~ = x + tau*b(x). */
static void step_slope(const or_problem *p, const real x[4], int thr, real u, real tau, real phi[4]) {
  real b[4];
  rhs(p, x, thr, u, b);
  if (p->integrator != 1) {
    for (int k = 0; k < 4; k++) phi[k] = b[k];
    return;
  }
  real xt[4], b2[4];
  for (int k = 0; k < 4; k++) xt[k] = x[k] + tau * b[k];
  rhs(p, xt, thr, u, b2);
  for (int k = 0; k < 4; k++) phi[k] = (real)0.5 * (b[k] + b2[k]);
}

/* One step of length tau from an arbitrary state x: z = x + tau*Phi. */
void or_step(const or_problem *p, const real x[4], int thr, real u, real tau, real z[4]) {
  real phi[4];
  step_slope(p, x, thr, u, tau, phi);
  for (int k = 0; k < 4; k++) z[k] = x[k] + tau * phi[k];
}

/* Foot of node i in grid coordinates: s_k = i_k + tau*Phi_k/h_k. */
static void foot_grid(const or_problem *p, const int i[4], int thr, real u, real tau, real s[4]) {
  real x[4], phi[4];
  node_coords(p, i, x);
  step_slope(p, x, thr, u, tau, phi);
  for (int k = 0; k < 4; k++) s[k] = (real)i[k] + tau * phi[k] / (real)step(p, k);
}

/* --------------------------------------------------------- interpolation */
/* Q1 interpolation at grid coordinates s (paper: multilinear I[V]).
 * Outside the closed box [0, n_k - 1] in any axis the value is M.
 * Inside, the cell is base_k = min(floor(s_k), n_k - 2), the local
 * coordinate t_k = s_k - base_k, and I = sum over the 16 corners e of
 * prod_k (e_k ? t_k : 1 - t_k) * V[base + e].
 * If idx/w are given, the 16 corner indices and weights are returned. */
static int cell(const or_problem *p, const real s[4], int base[4], real t[4]) {
  for (int k = 0; k < 4; k++) {
    if (periodic(p, k)) {
      /* wrap into [0, n): the cell between node n-1 and node 0 is a cell too */
      if (!isfinite((double)s[k])) return 0;
      const real n = (real)p->n[k];
      real w = s[k] - n * (real)floor((double)(s[k] / n));
      int b = (int)floor((double)w);
      if (b >= p->n[k]) b = p->n[k] - 1;
      if (b < 0) b = 0;
      base[k] = b;
      t[k] = w - (real)b;
      continue;
    }
    real sk = s[k];
    /* crown problem: the state constraint (I = M) holds on the two circular
     * faces r = r_min, r_max only; a foot beyond a velocity face is put on it */
    if (p->model == 2 && (k == 1 || k == 2) && isfinite((double)sk)) {
      if (sk < 0) sk = 0;
      if (sk > (real)(p->n[k] - 1)) sk = (real)(p->n[k] - 1);
    }
    if (!(sk >= 0 && sk <= (real)(p->n[k] - 1))) return 0;
    int b = (int)floor(sk);
    if (b > p->n[k] - 2) b = p->n[k] - 2;
    base[k] = b;
    t[k] = sk - (real)b;
  }
  return 1;
}

static real interp(const or_problem *p, const real *V, const real s[4]) {
  int base[4];
  real t[4];
  if (!cell(p, s, base, t)) return (real)p->M;
  real acc = 0;
  for (int c = 0; c < 16; c++) {
    real w = 1;
    int corner[4];
    for (int k = 0; k < 4; k++) {
      int e = (c >> k) & 1;
      w *= e ? t[k] : (real)1 - t[k];
      corner[k] = base[k] + e;
      if (periodic(p, k) && corner[k] == p->n[k]) corner[k] = 0;
    }
    acc += w * V[flat_index(p, corner)];
  }
  return acc;
}

/* Exported: value of I[V] at grid coordinates s. */
real or_interp(const or_problem *p, const real *V, const real s[4]) { return interp(p, V, s); }

/* Exported: corner indices and weights; returns 0 when s is outside. */
int or_interp_weights(const or_problem *p, const real s[4], int64_t idx[16], real w[16]) {
  int base[4];
  real t[4];
  if (!cell(p, s, base, t)) return 0;
  for (int c = 0; c < 16; c++) {
    real ww = 1;
    int corner[4];
    for (int k = 0; k < 4; k++) {
      int e = (c >> k) & 1;
      ww *= e ? t[k] : (real)1 - t[k];
      corner[k] = base[k] + e;
      if (periodic(p, k) && corner[k] == p->n[k]) corner[k] = 0;
    }
    idx[c] = flat_index(p, corner);
    w[c] = ww;
  }
  return 1;
}

/* FP64 read-out of I[V] at a physical state x (float or double V). */
/* Grid coordinate of a physical coordinate.  A state given in physical
 * units that lies on a face of the box can round to just outside it; points
 * within FACE_EPS cells of a face are put on the face. */
#define FACE_EPS 1e-6
static real to_grid(const or_problem *p, int k, double xk) {
  double s = (xk - p->lo[k]) / step(p, k);
  if (periodic(p, k)) return (real)s;
  double top = (double)(p->n[k] - 1);
  if (s < 0 && s > -FACE_EPS) s = 0;
  if (s > top && s < top + FACE_EPS) s = top;
  return (real)s;
}

double or_value_at(const or_problem *p, const real *V, const double x[4]) {
  real s[4];
  for (int k = 0; k < 4; k++) s[k] = to_grid(p, k, x[k]);
  return (double)interp(p, V, s);
}

/* --------------------------------------------------- Bellman Q of a control */
static real discount(const or_problem *p, real tau) { return (real)exp(-p->lambda * tau); }

/* Orbital elements of the crown problem's state x = (r, v_r, v_t, theta),
 * as the paper writes them (Section 3, polar running cost), except that the
 * printed semi-major axis -mu/(v^2 r - 2 mu) lacks a factor r (it is
 * dimensionless as printed): a = -mu r/(v^2 r - 2 mu), the vis-viva form;
 * eccentricity e = sqrt(1 + 2 E h^2/mu^2) with the
 * energy E = v^2/2 - mu/r and the angular momentum h = r v_t; argument of
 * perigee omega = theta - theta*, the true anomaly theta* = 2 arctan(r v_r
 * sqrt(p/mu) / (r (e - 1) + p)) with the semi-latus rectum p = a (1 - e^2).
 * That half-angle tangent is (e sin theta*)/(e + e cos theta*) with
 * e sin theta* = v_r sqrt(p/mu) and e cos theta* = p/r - 1; it is 0/0 at the
 * apoapsis, so the angle is taken from those two components directly,
 * theta* = atan2(v_r sqrt(p/mu), p/r - 1): the same angle wherever the
 * half-angle form is defined. */
void or_elements(const or_problem *p, const real x[4], real out[3]) {
  const double mu = p->mu;
  const double r = x[0], vr = x[1], vt = x[2], th = x[3];
  const double v2 = vr * vr + vt * vt;
  const double a = -mu * r / (v2 * r - 2.0 * mu);
  const double E = 0.5 * v2 - mu / r;
  const double h = r * vt;
  double e2 = 1.0 + 2.0 * E * h * h / (mu * mu);
  if (e2 < 0) e2 = 0;
  const double e = sqrt(e2);
  double ecw = 0, esw = 0;
  if (e > 0) {
    const double pp = a * (1.0 - e * e);
    const double ts = atan2(vr * sqrt(pp / mu), pp / r - 1.0);
    const double om = th - ts;
    ecw = e * cos(om);
    esw = e * sin(om);
  }
  out[0] = (real)a;
  out[1] = (real)ecw;
  out[2] = (real)esw;
}

/* Running cost l(x, f): w_time + w_fuel*thr, plus for the crown problem the
 * paper's orbital-element terms (eq:runcost_polar) beta*(a - a_bar)^2 +
 * gamma*((e cos w - e_bar cos w_bar)^2 + (e sin w - e_bar sin w_bar)^2); the
 * fuel term alpha*u_bar*thr is w_fuel*thr. */
real or_running_cost(const or_problem *p, const real x[4], int thr) {
  double l = p->w_time + p->w_fuel * (double)thr;
  if (p->model == 2) {
    real el[3];
    or_elements(p, x, el);
    const double da = (double)el[0] - p->el_a;
    const double dx = (double)el[1] - p->el_e * cos(p->el_omega);
    const double dy = (double)el[2] - p->el_e * sin(p->el_omega);
    l += p->el_beta * da * da + p->el_gamma * (dx * dx + dy * dy);
  }
  return (real)l;
}

/* Q(x_j, f) = dt*l + exp(-lambda*dt) * I[V](foot) at node i with step tau. */
static real q_node(const or_problem *p, const real *V, const int i[4], int thr, real u, real tau) {
  real s[4], x[4];
  foot_grid(p, i, thr, u, tau, s);
  node_coords(p, i, x);
  return tau * or_running_cost(p, x, thr) + discount(p, tau) * interp(p, V, s);
}

real or_q(const or_problem *p, const real *V, int64_t j, int thr, real u) {
  int i[4];
  node_index(p, j, i);
  return q_node(p, V, i, thr, u, (real)p->dt);
}

/* Q for many (node, throttle, angle) triples. */
void or_q_many(const or_problem *p, const real *V, const int64_t *nodes, const uint8_t *thr,
               const real *ang, int64_t count, real *out) {
  for (int64_t c = 0; c < count; c++) out[c] = or_q(p, V, nodes[c], thr[c], ang[c]);
}

/* Q at an arbitrary state y (feedback, eq:feed): interpolation at y + tau*b. */
static real q_state(const or_problem *p, const real *V, const real y[4], int thr, real u, real tau) {
  real z[4], s[4];
  or_step(p, y, thr, u, tau, z);
  for (int k = 0; k < 4; k++) s[k] = to_grid(p, k, (double)z[k]);
  return tau * or_running_cost(p, y, thr) + discount(p, tau) * interp(p, V, s);
}

/* Exported: Q at an arbitrary state y with step tau (tests of the closed loop). */
real or_q_state(const or_problem *p, const real *V, const real y[4], int thr, real u, real tau) {
  return q_state(p, V, y, thr, u, tau);
}

/* ------------------------------------------------------------- search */
typedef struct {
  real q;      /* best Q over all controls */
  real angle;  /* best thrust angle, wrapped into [-pi, pi) */
  int thr;     /* 1 if thrust beats coast */
  real margin; /* gap to the runner-up (tie indicator) */
} choice;

static real wrap_angle(real u) {
  const real two_pi = (real)(2.0 * OR_PI);
  while (u < (real)(-OR_PI)) u += two_pi;
  while (u >= (real)OR_PI) u -= two_pi;
  return u;
}

/* Q as a function of the control alone, at either a node or a free state. */
typedef struct {
  const or_problem *p;
  const real *V;
  const int *i;     /* node, or NULL */
  const real *y;    /* state, when i == NULL */
  real tau;
} qfun;

static real qeval(const qfun *f, int thr, real u) {
  if (f->i) return q_node(f->p, f->V, f->i, thr, u, f->tau);
  return q_state(f->p, f->V, f->y, thr, u, f->tau);
}

/* Discrete table: coast (index 0) and angles u_k = -pi + 2*pi*k/K (index k+1).
 * The first minimum in index order wins (strict <), so coast wins exact ties. */
static choice search_table(const qfun *f, int K) {
  real q_coast = qeval(f, 0, 0);
  real best = q_coast, second = INFINITY;
  real best_thr_q = INFINITY, best_thr_u = 0;
  int thr = 0;
  for (int k = 0; k < K; k++) {
    real u = (real)(-OR_PI + 2.0 * OR_PI * (double)k / (double)K);
    real q = qeval(f, 1, u);
    if (q < best_thr_q) { best_thr_q = q; best_thr_u = u; }
    if (q < best) { second = best; best = q; thr = 1; }
    else if (q < second) second = q;
  }
  choice c;
  c.q = best;
  c.angle = wrap_angle(best_thr_u);
  c.thr = thr;
  c.margin = second - best;
  return c;
}

/* Golden-section search (ratio (sqrt 5 - 1)/2) on [center - half, center +
 * half]: two interior evaluations, then one per iteration.  best_q and best_u
 * hold the best point evaluated so far (strict <, in evaluation order). */
static void golden_refine(const qfun *f, real center, real half, int iters, real *best_q, real *best_u) {
  const real rho = (real)((sqrt(5.0) - 1.0) / 2.0);
  real a = center - half, b = center + half;
  real x1 = b - rho * (b - a), x2 = a + rho * (b - a);
  real f1 = qeval(f, 1, x1);
  if (f1 < *best_q) { *best_q = f1; *best_u = x1; }
  real f2 = qeval(f, 1, x2);
  if (f2 < *best_q) { *best_q = f2; *best_u = x2; }
  for (int it = 0; it < iters; it++) {
    if (f1 < f2) {
      b = x2; x2 = x1; f2 = f1;
      x1 = b - rho * (b - a);
      f1 = qeval(f, 1, x1);
      if (f1 < *best_q) { *best_q = f1; *best_u = x1; }
    } else {
      a = x1; x1 = x2; f1 = f2;
      x2 = a + rho * (b - a);
      f2 = qeval(f, 1, x2);
      if (f2 < *best_q) { *best_q = f2; *best_u = x2; }
    }
  }
}

/* Scan of n_scan angles u_s = -pi + 2*pi*s/n_scan, then golden-section search
 * (ratio (sqrt 5 - 1)/2) on [u_s* - 2*pi/n_scan, u_s* + 2*pi/n_scan]: two
 * interior evaluations, then one per iteration.  The best evaluated point
 * (scan sample included, strict < in evaluation order) is the thrust
 * candidate; thrust is chosen iff its Q is strictly below the coast Q. */
static choice search_scan_golden(const qfun *f, int n_scan, int n_golden) {
  real *qs = (real *)calloc((size_t)(n_scan > 0 ? n_scan : 1), sizeof(real));
  int s_best = 0;
  for (int s = 0; s < n_scan; s++) {
    real u = (real)(-OR_PI + 2.0 * OR_PI * (double)s / (double)n_scan);
    qs[s] = qeval(f, 1, u);
    if (qs[s] < qs[s_best]) s_best = s;
  }
  real best_q = qs[s_best];
  real best_u = (real)(-OR_PI + 2.0 * OR_PI * (double)s_best / (double)n_scan);

  /* runner-up basin: best other local minimum of the cyclic scan at distance >= 2 */
  real basin_gap = INFINITY;
  for (int s = 0; s < n_scan; s++) {
    int d = abs(s - s_best);
    if (n_scan - d < d) d = n_scan - d;
    if (d < 2) continue;
    real ql = qs[(s + n_scan - 1) % n_scan], qr = qs[(s + 1) % n_scan];
    if (qs[s] <= ql && qs[s] <= qr && qs[s] - best_q < basin_gap) basin_gap = qs[s] - best_q;
  }
  free(qs);

  if (n_golden > 0)
    golden_refine(f, best_u, (real)(2.0 * OR_PI / (double)n_scan), n_golden, &best_q, &best_u);

  real q_coast = qeval(f, 0, 0);
  choice c;
  c.angle = wrap_angle(best_u);
  c.thr = best_q < q_coast;
  c.q = c.thr ? best_q : q_coast;
  c.margin = fabs(best_q - q_coast);
  if (basin_gap < c.margin) c.margin = basin_gap;
  return c;
}

/* Mode 3 without a previous optimum is the mode-0 table. */
static choice search(const qfun *f, const or_search *sr) {
  if (sr->mode == 0 || sr->mode == 3) return search_table(f, sr->n_angles);
  return search_scan_golden(f, sr->n_scan, sr->n_golden);
}

static real table_angle(int k, int K) { return (real)(-OR_PI + 2.0 * OR_PI * (double)k / (double)K); }

/* Index of the table angle nearest to u on the circle (halves round up);
 * 0 for a non-finite u. */
static int table_index(real u, int K) {
  if (!isfinite((double)u)) return 0;
  double k = floor(((double)u + OR_PI) * (double)K / (2.0 * OR_PI) + 0.5);
  k -= (double)K * floor(k / (double)K);
  int ki = (int)k;
  return (ki >= 0 && ki < K) ? ki : 0;
}

static void keep_smaller(real *m, real gap) {
  gap = (real)fabs((double)gap);
  if (gap < *m) *m = gap;
}

/* Walk over the mode-0 table from the previous optimum (Section 3,
 * "Efficient computation of the minimum": after the first iteration the
 * search starts at the previous optimal control and moves one step at a time
 * towards lower Q until it stands on a local minimiser).  Start at the table
 * angle nearest to u_prev; look at both cyclic neighbours; move to the lower
 * one if it is strictly below the current Q (the k-1 side when the two are
 * equal); from then on keep moving the same way while the next angle is
 * strictly lower (the angle just left is higher, so it never needs a second
 * look).  Thrust iff the walk's Q is strictly below the coast Q.  The margin
 * is the smallest gap of any comparison the walk decided (tie indicator).
 * *evals (nullable) accumulates the thrust evaluations. */
static choice search_walk(const qfun *f, int K, real u_prev, int64_t *evals) {
  int k = table_index(u_prev, K);
  const int km = (k + K - 1) % K, kp = (k + 1) % K;
  real qk = qeval(f, 1, table_angle(k, K));
  const real qm = qeval(f, 1, table_angle(km, K));
  const real qp = qeval(f, 1, table_angle(kp, K));
  int64_t n = 3;
  real margin = INFINITY;
  keep_smaller(&margin, qm - qk);
  keep_smaller(&margin, qp - qk);
  int d = 0;
  if (qm < qk && qm <= qp) d = -1;
  else if (qp < qk) d = 1;
  if (qm < qk && qp < qk) keep_smaller(&margin, qm - qp);
  if (d != 0) {
    k = d < 0 ? km : kp;
    qk = d < 0 ? qm : qp;
    for (int step_no = 0; step_no < K; step_no++) {
      const int kn = (k + d + K) % K;
      const real qn = qeval(f, 1, table_angle(kn, K));
      n++;
      keep_smaller(&margin, qn - qk);
      if (!(qn < qk)) break;
      k = kn;
      qk = qn;
    }
  }
  const real q_coast = qeval(f, 0, 0);
  keep_smaller(&margin, qk - q_coast);
  choice c;
  c.angle = wrap_angle(table_angle(k, K));
  c.thr = qk < q_coast;
  c.q = c.thr ? qk : q_coast;
  c.margin = margin;
  if (evals) *evals += n;
  return c;
}

/* Seeded search (the warm-started minimisation of Section 3, "Efficient
 * computation of the minimum", with the seed given per node): Q at the seed,
 * then golden_refine on [seed - w, seed + w] with n_local - 3 iterations, so
 * n_local thrust evaluations in all; thrust iff its best Q is strictly below
 * the coast Q.  Where the result differs from the node's current value vin
 * by more than fallback_tol * max(1, |vin|), the node repeats the full
 * mode-1 search and *fell_back is set. */
static choice search_seeded(const qfun *f, const or_search *sr, real seed, real vin, int *fell_back) {
  real best_q = qeval(f, 1, seed), best_u = seed;
  golden_refine(f, seed, (real)sr->local_half_width, sr->n_local - 3, &best_q, &best_u);
  real q_coast = qeval(f, 0, 0);
  choice c;
  c.angle = wrap_angle(best_u);
  c.thr = best_q < q_coast;
  c.q = c.thr ? best_q : q_coast;
  c.margin = fabs(best_q - q_coast);
  real den = fabs(vin) > 1 ? fabs(vin) : 1;
  *fell_back = fabs(c.q - vin) > (real)sr->fallback_tol * den;
  if (*fell_back) return search_scan_golden(f, sr->n_scan, sr->n_golden);
  return c;
}

/* ------------------------------------------------------------- sweeps */
/* Relative residual used by the device stop rule:
 * max_j |Vn_j - Vo_j| / max(1, |Vn_j|) and sum_j |Vn_j - Vo_j|, over free nodes. */
void or_residual(int64_t N, const uint8_t *kind, const real *Vo, const real *Vn, double out[3]) {
  double mx_rel = 0, sum = 0, mx_abs = 0;
  for (int64_t j = 0; j < N; j++) {
    if (kind[j] != KIND_FREE) continue;
    double d = fabs((double)Vn[j] - (double)Vo[j]);
    double den = fabs((double)Vn[j]);
    if (den < 1.0) den = 1.0;
    if (d / den > mx_rel) mx_rel = d / den;
    if (d > mx_abs) mx_abs = d;
    sum += d;
  }
  out[0] = mx_rel;
  out[1] = sum;
  out[2] = mx_abs;
}

/* One Jacobi Bellman sweep with full search.  Fixed nodes are copied.
 * pol_ang / pol_thr / margin may be NULL. */
void or_bellman_sweep(const or_problem *p, const uint8_t *kind, const or_search *sr,
                      const real *Vin, real *Vout, real *pol_ang, uint8_t *pol_thr, real *margin) {
  int64_t N = n_total(p);
  for (int64_t j = 0; j < N; j++) {
    if (kind[j] != KIND_FREE) {
      Vout[j] = Vin[j];
      if (pol_ang) pol_ang[j] = 0;
      if (pol_thr) pol_thr[j] = 0;
      if (margin) margin[j] = INFINITY;
      continue;
    }
    int i[4];
    node_index(p, j, i);
    qfun f = {p, Vin, i, NULL, (real)p->dt};
    choice c = search(&f, sr);
    Vout[j] = c.q;
    if (pol_ang) pol_ang[j] = c.angle;
    if (pol_thr) pol_thr[j] = (uint8_t)c.thr;
    if (margin) margin[j] = c.margin;
  }
}

/* One Jacobi Bellman sweep with the table walk (mode 3) started at each
 * node's previous angle ang_prev[j] (may alias pol_ang); with ang_prev NULL,
 * the full mode-0 table.  *evals (nullable) accumulates the thrust
 * evaluations.  Fixed nodes are copied. */
void or_bellman_sweep_walk(const or_problem *p, const uint8_t *kind, const or_search *sr, const real *Vin,
                           const real *ang_prev, real *Vout, real *pol_ang, uint8_t *pol_thr, real *margin,
                           int64_t *evals) {
  int64_t N = n_total(p);
  for (int64_t j = 0; j < N; j++) {
    if (kind[j] != KIND_FREE) {
      Vout[j] = Vin[j];
      if (pol_ang) pol_ang[j] = 0;
      if (pol_thr) pol_thr[j] = 0;
      if (margin) margin[j] = INFINITY;
      continue;
    }
    int i[4];
    node_index(p, j, i);
    qfun f = {p, Vin, i, NULL, (real)p->dt};
    choice c;
    if (ang_prev) {
      c = search_walk(&f, sr->n_angles, ang_prev[j], evals);
    } else {
      c = search_table(&f, sr->n_angles);
      if (evals) *evals += sr->n_angles;
    }
    Vout[j] = c.q;
    if (pol_ang) pol_ang[j] = c.angle;
    if (pol_thr) pol_thr[j] = (uint8_t)c.thr;
    if (margin) margin[j] = c.margin;
  }
}

/* Bellman operator at a list of nodes only (sampled checks on large grids). */
void or_bellman_nodes(const or_problem *p, const uint8_t *kind_at_nodes, const or_search *sr,
                      const real *Vin, const int64_t *nodes, int64_t count,
                      real *Vout, real *pol_ang, uint8_t *pol_thr, real *margin) {
  for (int64_t c = 0; c < count; c++) {
    int64_t j = nodes[c];
    if (kind_at_nodes[c] != KIND_FREE) {
      Vout[c] = Vin[j];
      pol_ang[c] = 0;
      pol_thr[c] = 0;
      margin[c] = INFINITY;
      continue;
    }
    int i[4];
    node_index(p, j, i);
    qfun f = {p, Vin, i, NULL, (real)p->dt};
    choice ch = search(&f, sr);
    Vout[c] = ch.q;
    pol_ang[c] = ch.angle;
    pol_thr[c] = (uint8_t)ch.thr;
    margin[c] = ch.margin;
  }
}

/* One Jacobi Bellman sweep with the seeded search (sr->mode is ignored):
 * seed[j] is the proposed thrust angle of node j; fell_back (nullable) marks
 * the nodes that repeated the full search. */
void or_bellman_sweep_seeded(const or_problem *p, const uint8_t *kind, const or_search *sr, const real *Vin,
                             const real *seed, real *Vout, real *pol_ang, uint8_t *pol_thr, real *margin,
                             uint8_t *fell_back) {
  int64_t N = n_total(p);
  for (int64_t j = 0; j < N; j++) {
    if (kind[j] != KIND_FREE) {
      Vout[j] = Vin[j];
      if (pol_ang) pol_ang[j] = 0;
      if (pol_thr) pol_thr[j] = 0;
      if (margin) margin[j] = INFINITY;
      if (fell_back) fell_back[j] = 0;
      continue;
    }
    int i[4];
    node_index(p, j, i);
    qfun f = {p, Vin, i, NULL, (real)p->dt};
    int fb = 0;
    choice c = search_seeded(&f, sr, seed[j], Vin[j], &fb);
    Vout[j] = c.q;
    if (pol_ang) pol_ang[j] = c.angle;
    if (pol_thr) pol_thr[j] = (uint8_t)c.thr;
    if (margin) margin[j] = c.margin;
    if (fell_back) fell_back[j] = (uint8_t)fb;
  }
}

/* One frozen-policy sweep (eq:p_eval applied once). */
void or_policy_eval_sweep(const or_problem *p, const uint8_t *kind, const real *Vin, real *Vout,
                          const real *pol_ang, const uint8_t *pol_thr) {
  int64_t N = n_total(p);
  for (int64_t j = 0; j < N; j++) {
    if (kind[j] != KIND_FREE) { Vout[j] = Vin[j]; continue; }
    int i[4];
    node_index(p, j, i);
    Vout[j] = q_node(p, Vin, i, pol_thr[j], pol_ang[j], (real)p->dt);
  }
}

/* The linear system of eq:p_eval for the frozen policy (pol_ang, pol_thr),
 * written out as the paper describes (Section 3): at every free node j,
 *   v_j - exp(-lambda dt) sum_i w_ji v_i = dt l(x_j, f_j)
 *            + exp(-lambda dt) (sum over fixed corners of w_ji V_i, or M
 *              when the foot leaves the domain),
 * with w_ji the Q1 weights of the foot's 16 corners.  Free unknowns are
 * numbered by node order (unknown[j], -1 at fixed nodes, caller-provided).
 * Triplets (row, col, val) of the matrix I - exp(-lambda dt) P_ff are
 * written to rows/cols/vals (at most 17 per free node; *nnz receives the
 * count) and the right-hand side to rhs (one per free node). */
void or_policy_system(const or_problem *p, const uint8_t *kind, const real *Vfixed, const real *pol_ang,
                      const uint8_t *pol_thr, const int64_t *unknown, int64_t *rows, int64_t *cols, double *vals,
                      double *rhs, int64_t *nnz) {
  const int64_t N = n_total(p);
  const double g = (double)discount(p, (real)p->dt);
  int64_t k = 0;
  for (int64_t j = 0; j < N; j++) {
    if (kind[j] != KIND_FREE) continue;
    const int64_t row = unknown[j];
    int i[4];
    node_index(p, j, i);
    real s[4], x[4];
    foot_grid(p, i, pol_thr[j], pol_ang[j], (real)p->dt, s);
    node_coords(p, i, x);
    double b = (double)p->dt * (double)or_running_cost(p, x, pol_thr[j]);
    rows[k] = row;
    cols[k] = row;
    vals[k] = 1.0;
    k++;
    int64_t idx[16];
    real w[16];
    if (!or_interp_weights(p, s, idx, w)) {
      b += g * p->M;
    } else {
      for (int c = 0; c < 16; c++) {
        if (kind[idx[c]] == KIND_FREE) {
          rows[k] = row;
          cols[k] = unknown[idx[c]];
          vals[k] = -g * (double)w[c];
          k++;
        } else {
          b += g * (double)w[c] * (double)Vfixed[idx[c]];
        }
      }
    }
    rhs[row] = b;
  }
  *nnz = k;
}

/* ------------------------------------------------------------- solvers */
/* Value iteration: V <- T V until max_j |dV_j| < tol_abs (FP64 rule) or, if
 * tol_abs <= 0, until the relative residual is below tol_rel.
 * Returns sweeps done (negative if max_sweeps was hit). */
int64_t or_solve_vi(const or_problem *p, const uint8_t *kind, const or_search *sr, real *V,
                    real *pol_ang, uint8_t *pol_thr, double tol_abs, double tol_rel,
                    int64_t max_sweeps, double *last_resid) {
  int64_t N = n_total(p);
  real *W = (real *)malloc(sizeof(real) * (size_t)N);
  int64_t k;
  double res[3] = {0, 0, 0};
  int done = 0;
  for (k = 1; k <= max_sweeps; k++) {
    /* the walk (mode 3) starts from the previous sweep's angles */
    if (sr->mode == 3) or_bellman_sweep_walk(p, kind, sr, V, k > 1 ? pol_ang : NULL, W, pol_ang, pol_thr, NULL, NULL);
    else or_bellman_sweep(p, kind, sr, V, W, pol_ang, pol_thr, NULL);
    or_residual(N, kind, V, W, res);
    memcpy(V, W, sizeof(real) * (size_t)N);
    if (tol_abs > 0 ? res[2] < tol_abs : res[0] < tol_rel) { done = 1; break; }
  }
  free(W);
  if (last_resid) { last_resid[0] = res[0]; last_resid[1] = res[1]; last_resid[2] = res[2]; }
  return done ? k : -max_sweeps;
}

/* Modified policy iteration: greedy step (eq:p_impr together with T V);
 * stop if its residual is below tolerance; otherwise eval_sweeps frozen-policy
 * sweeps (eq:p_eval solved approximately); repeat.  eval_sweeps < 0 means
 * "evaluate until the frozen-policy sweep changes V by less than tol/10".
 * From the second greedy step on, a node keeps its current control unless
 * the search finds a strictly smaller Q (eq:p_impr with the search standing
 * in for the exact argmin: the improvement step never returns a control worse
 * than the current one). */
int64_t or_solve_pi(const or_problem *p, const uint8_t *kind, const or_search *sr, real *V,
                    real *pol_ang, uint8_t *pol_thr, double tol_abs, double tol_rel,
                    int32_t eval_sweeps, int64_t max_outer, double *last_resid,
                    int64_t *total_eval_sweeps) {
  int64_t N = n_total(p);
  real *W = (real *)malloc(sizeof(real) * (size_t)N);
  double res[3] = {0, 0, 0};
  int64_t it, evals = 0;
  int done = 0;
  for (it = 1; it <= max_outer; it++) {
    if (it == 1) {
      or_bellman_sweep(p, kind, sr, V, W, pol_ang, pol_thr, NULL);
    } else {
      /* policy improvement: the search result, unless the node's current
       * control has a Q no larger (the incumbent is kept on ties) */
      for (int64_t j = 0; j < N; j++) {
        if (kind[j] != KIND_FREE) { W[j] = V[j]; continue; }
        int i[4];
        node_index(p, j, i);
        qfun f = {p, V, i, NULL, (real)p->dt};
        /* mode 3: the walk starts at the current policy's angle */
        choice c = sr->mode == 3 ? search_walk(&f, sr->n_angles, pol_ang[j], NULL) : search(&f, sr);
        real q_inc = q_node(p, V, i, pol_thr[j], pol_ang[j], (real)p->dt);
        if (q_inc <= c.q) {
          W[j] = q_inc;
        } else {
          W[j] = c.q;
          pol_ang[j] = c.angle;
          pol_thr[j] = (uint8_t)c.thr;
        }
      }
    }
    or_residual(N, kind, V, W, res);
    memcpy(V, W, sizeof(real) * (size_t)N);
    if (tol_abs > 0 ? res[2] < tol_abs : res[0] < tol_rel) { done = 1; break; }
    if (eval_sweeps >= 0) {
      for (int e = 0; e < eval_sweeps; e++) {
        or_policy_eval_sweep(p, kind, V, W, pol_ang, pol_thr);
        memcpy(V, W, sizeof(real) * (size_t)N);
        evals++;
      }
    } else {
      double inner_tol = (tol_abs > 0 ? tol_abs : tol_rel) * 0.1;
      for (int64_t e = 0; e < 1000000; e++) {
        double r2[3];
        or_policy_eval_sweep(p, kind, V, W, pol_ang, pol_thr);
        or_residual(N, kind, V, W, r2);
        memcpy(V, W, sizeof(real) * (size_t)N);
        evals++;
        if ((tol_abs > 0 ? r2[2] : r2[0]) < inner_tol) break;
      }
    }
  }
  free(W);
  if (last_resid) { last_resid[0] = res[0]; last_resid[1] = res[1]; last_resid[2] = res[2]; }
  if (total_eval_sweeps) *total_eval_sweeps = evals;
  return done ? it : -max_outer;
}

/* ------------------------------------------------------------- feedback */
/* Approximate optimal feedback eq:feed at arbitrary states y (count x 4),
 * with time step tau and the same search as the solver.  margin_out (may be
 * NULL) receives the search's tie margin, as the sweeps report it per node. */
void or_feedback(const or_problem *p, const or_search *sr, const real *V, const double *states,
                 int64_t count, double tau, real *angle_out, uint8_t *thr_out, real *q_out,
                 real *margin_out) {
  for (int64_t c = 0; c < count; c++) {
    real y[4];
    for (int k = 0; k < 4; k++) y[k] = (real)states[4 * c + k];
    qfun f = {p, V, NULL, y, (real)tau};
    choice ch = search(&f, sr);
    angle_out[c] = ch.angle;
    thr_out[c] = (uint8_t)ch.thr;
    if (q_out) q_out[c] = ch.q;
    if (margin_out) margin_out[c] = ch.margin;
  }
}

/* ------------------------------------------------- closed-loop simulation */
/* The "real system" of the simulations: the model's dynamics plus, for the
 * orbit models, the aerodynamic drag of Section 4's Example 2, an
 * acceleration of magnitude drag * |v|^2 against the velocity (v_r, v_t)
 * (the air at rest); drag = 0 leaves the model's own dynamics. */
static void plant_rhs(const or_problem *p, const real x[4], int thr, real u, real drag, real b[4]) {
  rhs(p, x, thr, u, b);
  if (drag != 0 && p->model != 1) {
    real speed = (real)sqrt((double)(x[1] * x[1] + x[2] * x[2]));
    b[1] -= drag * speed * x[1];
    b[2] -= drag * speed * x[2];
  }
}

/* One classical fourth-order Runge-Kutta step of length h of the real
 * system with the control (thr, u) held over the step. */
void or_rk4_step(const or_problem *p, real x[4], int thr, real u, real h, real drag) {
  real k1[4], k2[4], k3[4], k4[4], y[4];
  plant_rhs(p, x, thr, u, drag, k1);
  for (int k = 0; k < 4; k++) y[k] = x[k] + (real)0.5 * h * k1[k];
  plant_rhs(p, y, thr, u, drag, k2);
  for (int k = 0; k < 4; k++) y[k] = x[k] + (real)0.5 * h * k2[k];
  plant_rhs(p, y, thr, u, drag, k3);
  for (int k = 0; k < 4; k++) y[k] = x[k] + h * k3[k];
  plant_rhs(p, y, thr, u, drag, k4);
  for (int k = 0; k < 4; k++) x[k] += h / (real)6 * (k1[k] + (real)2 * k2[k] + (real)2 * k3[k] + k4[k]);
}

/* Closed loop (Section 3, feedback eq:feed, and the simulations of
 * Section 4): from each of count states, `steps` times: the feedback control
 * at the current state with time step tau (the context's search), then
 * `substeps` fourth-order Runge-Kutta steps of length tau/substeps with that
 * control held.  states (count x 4) is updated in place; traj (nullable)
 * receives the states before every step and after the last, step-major
 * ((steps+1) x count x 4); thr_hist / ang_hist (nullable) the controls,
 * step-major (steps x count).  drag: the Example 2 drag coefficient of the
 * real system (0: none); the feedback still uses V of the model without it. */
void or_simulate(const or_problem *p, const or_search *sr, const real *V, double *states, int64_t count,
                 double tau, int32_t steps, int32_t substeps, double drag, double *traj, uint8_t *thr_hist,
                 real *ang_hist) {
  for (int64_t c = 0; c < count; c++) {
    real y[4];
    for (int k = 0; k < 4; k++) y[k] = (real)states[4 * c + k];
    if (traj)
      for (int k = 0; k < 4; k++) traj[4 * c + k] = (double)y[k];
    for (int32_t s = 0; s < steps; s++) {
      qfun f = {p, V, NULL, y, (real)tau};
      choice ch = search(&f, sr);
      const real h = (real)(tau / (double)substeps);
      for (int32_t q = 0; q < substeps; q++) or_rk4_step(p, y, ch.thr, ch.angle, h, (real)drag);
      if (thr_hist) thr_hist[(int64_t)s * count + c] = (uint8_t)ch.thr;
      if (ang_hist) ang_hist[(int64_t)s * count + c] = ch.angle;
      if (traj)
        for (int k = 0; k < 4; k++) traj[((int64_t)(s + 1) * count + c) * 4 + k] = (double)y[k];
    }
    for (int k = 0; k < 4; k++) states[4 * c + k] = (double)y[k];
  }
}

/* Brute force for tests: min over n angles u = -pi + 2*pi*k/n of the thrust Q. */
real or_brute_thrust_min(const or_problem *p, const real *V, int64_t j, int64_t n, real *u_best) {
  int i[4];
  node_index(p, j, i);
  real best = INFINITY, bu = 0;
  for (int64_t k = 0; k < n; k++) {
    real u = (real)(-OR_PI + 2.0 * OR_PI * (double)k / (double)n);
    real q = q_node(p, V, i, 1, u, (real)p->dt);
    if (q < best) { best = q; bu = u; }
  }
  if (u_best) *u_best = bu;
  return best;
}

/* --------------------------------------------------------- reduced grid */
/* Reachability mask of a fine grid from a coarse solution: a fine node is
 * kept where the coarse value, interpolated at the node, is below `thresh`;
 * the kept set is then dilated by dil[k] cells along each axis (box
 * dilation).  Coarse and fine problems must share the domain box. */
void or_mask_from_coarse(const or_problem *pc, const real *Vc, const or_problem *pf,
                         double thresh, const int32_t dil[4], uint8_t *mask) {
  int64_t N = n_total(pf);
  uint8_t *seed = (uint8_t *)malloc((size_t)N);
  for (int64_t j = 0; j < N; j++) {
    int i[4];
    node_index(pf, j, i);
    double x[4];
    for (int k = 0; k < 4; k++) x[k] = pf->lo[k] + i[k] * step(pf, k);
    seed[j] = or_value_at(pc, Vc, x) < thresh;
  }
  for (int64_t j = 0; j < N; j++) {
    int i[4];
    node_index(pf, j, i);
    int keep = 0;
    int lo[4], hi[4];
    for (int k = 0; k < 4; k++) {
      lo[k] = i[k] - dil[k] < 0 ? 0 : i[k] - dil[k];
      hi[k] = i[k] + dil[k] > pf->n[k] - 1 ? pf->n[k] - 1 : i[k] + dil[k];
    }
    int q[4];
    for (q[3] = lo[3]; q[3] <= hi[3] && !keep; q[3]++)
      for (q[2] = lo[2]; q[2] <= hi[2] && !keep; q[2]++)
        for (q[1] = lo[1]; q[1] <= hi[1] && !keep; q[1]++)
          for (q[0] = lo[0]; q[0] <= hi[0] && !keep; q[0]++)
            if (seed[flat_index(pf, q)]) keep = 1;
    mask[j] = (uint8_t)keep;
  }
  free(seed);
}

int32_t or_real_size(void) { return (int32_t)sizeof(real); }
