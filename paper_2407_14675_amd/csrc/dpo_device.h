// Device-side building blocks shared by the sweep kernels of libdpo.
//
// Grid coordinates: node i_k of axis k, foot displacement off_k in cells, so
// the foot sits at s_k = i_k + off_k (paper Section 3: the foot point
// x_j + dt*Phi(x_j, f) of eq:schema, expressed on the grid).  Keeping the
// integer and the fractional parts apart keeps the local cell coordinate
// accurate to about 1e-7 of a cell in float32, where an absolute float32
// coordinate would only resolve ulp(1)/h ~ 5e-5 of a cell.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpo {

constexpr int kBlock = 256;     // threads per workgroup of the node kernels (4 waves)
constexpr int kMaxBlock = 512;  // largest workgroup of the factorised sweeps

struct Grid {
  int n[4];
  int st[4];  // element strides: 1, n0, n0*n1, n0*n1*n2
  double lo[4];
  double h[4];
  double inv_h[4];
  int periodic3;  // axis 3 is periodic (the crown problem's theta): h3 = (hi - lo)/n, feet wrap
  int clamp12;    // feet beyond the v_r / v_t faces are put on them (the crown problem's state
                  // constraint holds on the two circular faces r = r_min, r_max only)
};

struct Phys {
  int model;  // 0 orbit, 1 eikonal, 2 crown (polar state with theta, orbital-element cost)
  int heun;   // 1: Heun (second-order Runge-Kutta) foot point, 0: Euler
  double mu, accel, mdot, dt, speed;
  // crown running cost: el_beta*(a - el_a)^2 + el_gamma*|e_vec - (el_ex, el_ey)|^2
  double el_beta, el_gamma, el_a, el_ex, el_ey;
  float q_coast;  // dt * w_time
  float q_thr;    // dt * (w_time + w_fuel)
  float gamma;    // exp(-lambda * dt)
  float M;
};

// Control-independent part of the displacement of one node and the thrust
// coefficients, all in cells.  Computed once per node in FP64 and rounded:
// the gravity/centrifugal difference cancels to ~2% of its terms, so float32
// here would cost ~1e-6 of a cell per step.
struct NodeTerms {
  int i[4];
  float drift[4];
  float g1, g2;  // displacement along v_r per unit sin u, along v_t per unit cos u
  float gm;      // displacement along m under thrust (<= 0)
};

__device__ inline void decode_node(const Grid& G, int j, int i[4]) {
  int q = j;
  i[0] = q % G.n[0];
  q /= G.n[0];
  i[1] = q % G.n[1];
  q /= G.n[1];
  i[2] = q % G.n[2];
  i[3] = q / G.n[2];
}

// Right-hand side of the planar dynamics at a physical state x, scaled by
// tau and divided by the grid steps.  Orbit: (v_r, v_t^2/r - mu/r^2,
// -v_r v_t / r, 0) + thr*(0, (a/m) sin u, (a/m) cos u, -c).  Crown: the same
// with a constant thrust acceleration and theta' = v_t / r on axis 3.
__device__ inline void state_terms(const Grid& G, const Phys& P, const double x[4], double tau,
                                   float drift[4], float& g1, float& g2, float& gm) {
#pragma clang fp contract(off)
  if (P.model == 2) {
    const double r = x[0], vr = x[1], vt = x[2];
    const double inv_r = 1.0 / r;
    drift[0] = (float)(tau * vr * G.inv_h[0]);
    drift[1] = (float)(tau * (vt * vt * inv_r - P.mu * inv_r * inv_r) * G.inv_h[1]);
    drift[2] = (float)(tau * (-vr * vt * inv_r) * G.inv_h[2]);
    drift[3] = (float)(tau * vt * inv_r * G.inv_h[3]);
    g1 = (float)(tau * P.accel * G.inv_h[1]);
    g2 = (float)(tau * P.accel * G.inv_h[2]);
    gm = 0.0f;
  } else if (P.model == 0) {
    const double r = x[0], vr = x[1], vt = x[2], m = x[3];
    const double inv_r = 1.0 / r;
    drift[0] = (float)(tau * vr * G.inv_h[0]);
    drift[1] = (float)(tau * (vt * vt * inv_r - P.mu * inv_r * inv_r) * G.inv_h[1]);
    drift[2] = (float)(tau * (-vr * vt * inv_r) * G.inv_h[2]);
    drift[3] = 0.0f;
    const double acc = P.accel / m;
    g1 = (float)(tau * acc * G.inv_h[1]);
    g2 = (float)(tau * acc * G.inv_h[2]);
    gm = (float)(-tau * P.mdot * G.inv_h[3]);
  } else {
    drift[0] = drift[1] = drift[2] = drift[3] = 0.0f;
    g1 = (float)(tau * P.speed * G.inv_h[1]);
    g2 = (float)(tau * P.speed * G.inv_h[2]);
    gm = 0.0f;
  }
}

__device__ inline uint32_t pack_node(const int i[4]) {
  return (uint32_t)i[0] | ((uint32_t)i[1] << 8) | ((uint32_t)i[2] << 16) | ((uint32_t)i[3] << 24);
}

__device__ inline int unpack_node(const Grid& G, uint32_t p, int i[4]) {
  i[0] = (int)(p & 0xffu);
  i[1] = (int)((p >> 8) & 0xffu);
  i[2] = (int)((p >> 16) & 0xffu);
  i[3] = (int)(p >> 24);
  return i[0] + i[1] * G.st[1] + i[2] * G.st[2] + i[3] * G.st[3];
}

__device__ inline void node_terms(const Grid& G, const Phys& P, int j, double tau, NodeTerms& T) {
#pragma clang fp contract(off)
  decode_node(G, j, T.i);
  double x[4];
#pragma unroll
  for (int k = 0; k < 4; k++) x[k] = G.lo[k] + (double)T.i[k] * G.h[k];
  state_terms(G, P, x, tau, T.drift, T.g1, T.g2, T.gm);
}

// (1 - t) a + t b, exact at t = 0 and t = 1 (feet on nodes and faces).
__device__ inline float lerp(float a, float b, float t) { return fmaf(t, b, fmaf(-t, a, a)); }

// Cell of the foot s = i + off (paper Section 3: Q1 on the closed box):
// false if s_k lies outside [0, n_k - 1] on some axis; else the cell base
// base_k = min(floor(s_k), n_k - 2) and the local coordinate t_k = s_k - base_k.
// kSnap: feet of states given in physical units (feedback) that lie within
// 1e-6 cells outside a face are put on the face.
// One axis of the foot's cell: inside iff 0 <= i + o <= n - 1; then
// b = min(floor(i + o), n - 2) and t = i + o - b.
__device__ inline bool axis_cell(int i, int n, float o, int& b, float& t) {
  if (!(o >= (float)(-i) && o <= (float)(n - 1 - i))) return false;
  const float fl = floorf(o);
  b = i + (int)fl;
  t = o - fl;
  if (b > n - 2) {
    b = n - 2;
    t = 1.0f;
  }
  return true;
}

// Periodic axis: the foot wraps into [0, n); the cell between node n-1 and
// node 0 is a cell like any other.  False only for a non-finite offset.
__device__ inline bool periodic_cell(int i, int n, float o, int& b, float& t) {
  if (!(fabsf(o) <= 1.0e30f)) return false;
  const float nf = (float)n;
  const float s = (float)i + o;
  const float w = s - nf * floorf(s / nf);
  const float fl = floorf(w);
  b = (int)fl;
  t = w - fl;
  if (b >= n) {  // w rounded up to n: node 0
    b = 0;
    t = 0.0f;
  }
  if (b < 0) {
    b = 0;
    t = 0.0f;
  }
  return true;
}

template <bool kSnap = false>
__device__ inline bool foot_cell(const Grid& G, const int i[4], const float off[4], int base[4], float t[4]) {
#pragma unroll
  for (int k = 0; k < 4; k++) {
    float o = off[k];
    if (k == 3 && G.periodic3) {
      if (!periodic_cell(i[3], G.n[3], o, base[3], t[3])) return false;
      continue;
    }
    if ((k == 1 || k == 2) && G.clamp12 && fabsf(o) <= 1.0e30f)
      o = fminf(fmaxf(o, (float)(-i[k])), (float)(G.n[k] - 1 - i[k]));
    if (kSnap) {
      const float lo = (float)(-i[k]), hi = (float)(G.n[k] - 1 - i[k]);
      if (o < lo && o > lo - 1e-6f) o = lo;
      if (o > hi && o < hi + 1e-6f) o = hi;
    }
    if (!axis_cell(i[k], G.n[k], o, base[k], t[k])) return false;
  }
  return true;
}

// Two r-adjacent corners fetched by one dword-aligned 8-byte load.
struct __attribute__((aligned(4))) CornerPair {
  float lo, hi;
};

// 16-corner Q1 value of the cell whose lowest corner is p: 15 lerps, r first
// (the 8 r-adjacent corner pairs are 8 loads).  s3: element step from the
// cell's lower to its upper corner along axis 3 (G.st[3], or back to node 0
// on a periodic axis).
__device__ inline float cell_value(const float* __restrict__ p, const Grid& G, const float t[4], int s3) {
  const int s1 = G.st[1], s2 = G.st[2];
  float c[8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int o = ((e & 1) ? s1 : 0) + ((e & 2) ? s2 : 0) + ((e & 4) ? s3 : 0);
    const CornerPair v = *reinterpret_cast<const CornerPair*>(p + o);
    c[e] = lerp(v.lo, v.hi, t[0]);
  }
  const float d0 = lerp(c[0], c[1], t[1]);
  const float d1 = lerp(c[2], c[3], t[1]);
  const float d2 = lerp(c[4], c[5], t[1]);
  const float d3 = lerp(c[6], c[7], t[1]);
  const float e0 = lerp(d0, d1, t[2]);
  const float e1 = lerp(d2, d3, t[2]);
  return lerp(e0, e1, t[3]);
}

// The 16 corners of the cell a node's last evaluation read, kept in
// registers: the feet of one node's controls mostly share a cell (on the
// crown problem a step moves a foot by less than a tenth of a cell), so a
// search reloads the corners only when the cell changes.  key: offset of the
// cell's lowest corner in V (-1 = empty); the lerps are cell_value's, in the
// same order, so the value is the same bit for bit.
struct CornerCache {
  int key;
  CornerPair v[8];
};

__device__ inline float cell_value_cached(const float* __restrict__ V, const Grid& G, int key, const float t[4], int s3,
                                          CornerCache& cc) {
  if (key != cc.key) {
    const int s1 = G.st[1], s2 = G.st[2];
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int o = ((e & 1) ? s1 : 0) + ((e & 2) ? s2 : 0) + ((e & 4) ? s3 : 0);
      cc.v[e] = *reinterpret_cast<const CornerPair*>(V + key + o);
    }
    cc.key = key;
  }
  float c[8];
#pragma unroll
  for (int e = 0; e < 8; e++) c[e] = lerp(cc.v[e].lo, cc.v[e].hi, t[0]);
  const float d0 = lerp(c[0], c[1], t[1]);
  const float d1 = lerp(c[2], c[3], t[1]);
  const float d2 = lerp(c[4], c[5], t[1]);
  const float d3 = lerp(c[6], c[7], t[1]);
  const float e0 = lerp(d0, d1, t[2]);
  const float e1 = lerp(d2, d3, t[2]);
  return lerp(e0, e1, t[3]);
}

// Q1 interpolation of V at s = i + off (paper Section 3: multilinear I[V],
// M outside the closed box).
template <bool kSnap = false>
__device__ inline float interp_off(const float* __restrict__ V, const Grid& G, const int i[4],
                                   const float off[4], float M) {
  int base[4];
  float t[4];
  if (!foot_cell<kSnap>(G, i, off, base, t)) return M;
  const int s3 = (G.periodic3 && base[3] == G.n[3] - 1) ? -base[3] * G.st[3] : G.st[3];
  return cell_value(V + (base[0] + base[1] * G.st[1] + base[2] * G.st[2] + base[3] * G.st[3]), G, t, s3);
}

// ---- Heun foot point (paper Section 3 names a second-order Runge-Kutta
// step): foot = x + tau*(b(x) + b(x~))/2 with x~ = x + tau*b(x), i.e. the
// Euler displacement tau*b(x) plus (tau/2)*(b(x~) - b(x)).  The Euler part
// comes from NodeTerms as on the Euler path; the correction is formed in
// float from the predictor's increments, with every difference of nearly
// equal terms (1/r~ - 1/r, v_t~^2/r~ - v_t^2/r, ...) written as a product of
// increments, so it carries float's relative error on its own size
// (~1e-2 cell) instead of on the slopes.  The eikonal field does not depend
// on the state: there the correction is zero.
struct HeunTerms {
  float r, vr, vt, m;  // the state the step starts from (m = 1 for the crown problem)
  float d1, d2;        // control-free slopes along v_r and v_t (rounded from FP64)
  float acc;           // accel / m
  float tau, mdot, mu, accel;
  float sc[4];         // (tau/2) / h_k
  int orbit;           // orbit or crown dynamics (the eikonal field is constant)
  int crown;           // axis 3 is theta, theta' = v_t / r
};

__device__ inline void heun_terms(const Grid& G, const Phys& P, const double x[4], double tau, HeunTerms& H) {
#pragma clang fp contract(off)
  H.orbit = P.model == 0 || P.model == 2;
  H.crown = P.model == 2;
  const double r = x[0], vr = x[1], vt = x[2], m = H.crown ? 1.0 : x[3];
  H.r = (float)r;
  H.vr = (float)vr;
  H.vt = (float)vt;
  H.m = (float)m;
  if (H.orbit) {
    const double inv_r = 1.0 / r;
    H.d1 = (float)(vt * vt * inv_r - P.mu * inv_r * inv_r);
    H.d2 = (float)(-vr * vt * inv_r);
    H.acc = (float)(P.accel / m);
  } else {
    H.d1 = H.d2 = H.acc = 0.0f;
  }
  H.tau = (float)tau;
  H.mdot = H.crown ? 0.0f : (float)P.mdot;
  H.mu = (float)P.mu;
  H.accel = (float)P.accel;
  for (int k = 0; k < 4; k++) H.sc[k] = (float)(0.5 * tau * G.inv_h[k]);
}

// (tau/2)*(b(x~) - b(x)) in cells along r, v_r, v_t and axis 3 (the mass:
// zero, its rate is constant; the crown's theta: v_t~/r~ - v_t/r).
__device__ inline void heun_corr(const HeunTerms& H, int thr, float sn, float cs, float c[4]) {
  if (!H.orbit) {
    c[0] = c[1] = c[2] = c[3] = 0.0f;
    return;
  }
  const float k1v = thr ? fmaf(H.acc, sn, H.d1) : H.d1;
  const float k1t = thr ? fmaf(H.acc, cs, H.d2) : H.d2;
  const float dr = H.tau * H.vr, dv = H.tau * k1v, dw = H.tau * k1t;
  const float rt = H.r + dr;
  const float inv = 1.0f / (H.r * rt);
  // v_t~^2/r~ - v_t^2/r and -mu (1/r~^2 - 1/r^2)
  const float cent = (dw * (2.0f * H.vt + dw) * H.r - H.vt * H.vt * dr) * inv;
  const float grav = H.mu * dr * (2.0f * H.r + dr) * inv * inv;
  // -(v_r~ v_t~/r~ - v_r v_t/r)
  const float cor = -((dv * H.vt + H.vr * dw + dv * dw) * H.r - H.vr * H.vt * dr) * inv;
  float tv = 0.0f, tt = 0.0f;
  if (thr) {
    const float dm = -H.tau * H.mdot;
    const float dinv_m = -dm / (H.m * (H.m + dm));  // 1/m~ - 1/m
    tv = H.accel * sn * dinv_m;
    tt = H.accel * cs * dinv_m;
  }
  c[0] = H.sc[0] * dv;
  c[1] = H.sc[1] * (cent + grav + tv);
  c[2] = H.sc[2] * (cor + tt);
  c[3] = H.crown ? H.sc[3] * ((dw * H.r - H.vt * dr) * inv) : 0.0f;
}

// Foot displacement (cells) of a control under the node's integrator.
template <bool kHeun>
__device__ inline void foot_off(const NodeTerms& T, const HeunTerms& H, int thr, float sn, float cs, float off[4]) {
  off[0] = T.drift[0];
  off[1] = thr ? fmaf(T.g1, sn, T.drift[1]) : T.drift[1];
  off[2] = thr ? fmaf(T.g2, cs, T.drift[2]) : T.drift[2];
  off[3] = T.drift[3] + (thr ? T.gm : 0.0f);
  if (kHeun) {
    float c[4];
    heun_corr(H, thr, sn, cs, c);
    off[0] += c[0];
    off[1] += c[1];
    off[2] += c[2];
    off[3] += c[3];
  }
}

// Q of one control at a node, dt*l + gamma * I[V](foot), for thr (angle given
// by its sin/cos) under either integrator.  qx: the state-dependent part of
// dt*l at the node (the crown problem's orbital-element cost; 0 otherwise).
template <bool kHeun, bool kSnap = false>
__device__ inline float q_step(const float* __restrict__ V, const Grid& G, const Phys& P, const NodeTerms& T,
                               const HeunTerms& H, int thr, float sn, float cs, float qx = 0.0f) {
  float off[4];
  foot_off<kHeun>(T, H, thr, sn, cs, off);
  return fmaf(P.gamma, interp_off<kSnap>(V, G, T.i, off, P.M), (thr ? P.q_thr : P.q_coast) + qx);
}

// q_step through a node's corner cache (the cell's corners are loaded only
// when the foot leaves the cell of the previous evaluation).
template <bool kHeun>
__device__ inline float q_step_cached(const float* __restrict__ V, const Grid& G, const Phys& P, const NodeTerms& T,
                                      const HeunTerms& H, int thr, float sn, float cs, float qx, CornerCache& cc) {
  float off[4];
  foot_off<kHeun>(T, H, thr, sn, cs, off);
  int base[4];
  float t[4];
  float I = P.M;
  if (foot_cell(G, T.i, off, base, t)) {
    const int s3 = (G.periodic3 && base[3] == G.n[3] - 1) ? -base[3] * G.st[3] : G.st[3];
    I = cell_value_cached(V, G, base[0] + base[1] * G.st[1] + base[2] * G.st[2] + base[3] * G.st[3], t, s3, cc);
  }
  return fmaf(P.gamma, I, (thr ? P.q_thr : P.q_coast) + qx);
}

// The crown problem's orbital-element running cost at a physical state x =
// (r, v_r, v_t, theta), in FP64: beta*(a - a_bar)^2 + gamma*|e - e_bar|^2,
// a from vis-viva and the eccentricity vector in polar form,
// e = ((h^2/(mu r) - 1) (cos th, sin th) + (v_r h/mu) (sin th, -cos th)), h = r v_t.
__device__ inline double crown_cost(const Phys& P, const double x[4]) {
#pragma clang fp contract(off)
  const double r = x[0], vr = x[1], vt = x[2], th = x[3];
  const double v2 = vr * vr + vt * vt;
  const double a = -P.mu * r / (v2 * r - 2.0 * P.mu);
  const double h = r * vt;
  const double ec = h * h / (P.mu * r) - 1.0, es = vr * h / P.mu;
  double sth, cth;
  sincos(th, &sth, &cth);
  const double ex = ec * cth + es * sth, ey = ec * sth - es * cth;
  const double da = a - P.el_a, dx = ex - P.el_ex, dy = ey - P.el_ey;
  return P.el_beta * da * da + P.el_gamma * (dx * dx + dy * dy);
}

__device__ inline float wrap_pi(float u) {
  const float two_pi = 6.283185307179586f;
  const float pi = 3.14159265358979f;
  if (u < -pi) u += two_pi;
  if (u >= pi) u -= two_pi;
  return u;
}

// Workgroup -> tile remap: the hardware deals consecutive workgroups round
// robin over the 8 XCDs; giving each XCD a contiguous run of tiles keeps the
// gather footprint of neighbouring tiles in that XCD's L2.
__device__ inline int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, local = b >> 3;
  return x * q + (x < r ? x : r) + local;
}

// Per-workgroup partials: max rel, sum |dV|, max |dV|, non-finite count,
// fallback count.
constexpr int kPartial = 5;

// Wave64 + workgroup reduction of one node kernel's residual partials,
// written to partial[block*kPartial + 0..4] in a fixed order (any workgroup
// size that is a multiple of 64, up to kMaxBlock).
__device__ inline void block_residual(double rel, double sum, double mabs, double bad,
                                      double fb, double* __restrict__ partial, int block) {
  __shared__ double red[kPartial][kMaxBlock / 64];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    rel = fmax(rel, __shfl_xor(rel, o, 64));
    sum += __shfl_xor(sum, o, 64);
    mabs = fmax(mabs, __shfl_xor(mabs, o, 64));
    bad += __shfl_xor(bad, o, 64);
    fb += __shfl_xor(fb, o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = rel;
    red[1][wave] = sum;
    red[2][wave] = mabs;
    red[3][wave] = bad;
    red[4][wave] = fb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = red[0][0], b = red[1][0], c = red[2][0], d = red[3][0], e = red[4][0];
    const int nw = (int)(blockDim.x >> 6);
    for (int w = 1; w < nw; w++) {
      a = fmax(a, red[0][w]);
      b += red[1][w];
      c = fmax(c, red[2][w]);
      d += red[3][w];
      e += red[4][w];
    }
    partial[kPartial * block + 0] = a;
    partial[kPartial * block + 1] = b;
    partial[kPartial * block + 2] = c;
    partial[kPartial * block + 3] = d;
    partial[kPartial * block + 4] = e;
  }
}

// Per-node residual contribution: |dV| is exact in FP64 for float inputs.
__device__ inline void node_residual(float v_old, float v_new, double& rel, double& sum,
                                     double& mabs, double& bad) {
  if (!isfinite(v_new)) {
    bad += 1.0;
    return;
  }
  const double d = fabs((double)v_new - (double)v_old);
  const double den = fmax(1.0, fabs((double)v_new));
  rel = fmax(rel, d / den);
  sum += d;
  mabs = fmax(mabs, d);
}

}  // namespace dpo
