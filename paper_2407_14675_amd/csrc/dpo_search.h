// Device-side search machinery shared by the single-problem and the batched
// sweep kernels: node terms from the per-axis tables, the tabulated scan,
// the golden section, the seeded local search, the foot descriptors of the
// chosen control, and the factorised thrust evaluation.
//
// Paper: arXiv 2407.14675, Section 3 (eq:schema; minimisation by tabulation
// and golden-section refinement).
#pragma once

#include "dpo_kernels.h"

namespace dpo {

// Node terms from the packed coordinates of a free node and the per-axis
// tables: FP64 for the control-independent drift, float for the rest.
// Node coordinates are formed as lo + i*h with the product rounded before the
// sum (no fused multiply-add), the plain definition of the grid: a node whose
// coordinate is exactly zero (the middle v_r node of an odd grid) then gets
// exactly zero, and its feet on a face stay on the face.
//
// The r displacement dt*v_r/h_r (cells) of nodes in v_r row i1.
__device__ inline float drift_r(const SweepArgs& a, int i1) {
#pragma clang fp contract(off)
  if (a.P.model == 1) return 0.0f;
  const double vr = a.G.lo[1] + (double)i1 * a.G.h[1];
  return (float)(a.c0 * vr);
}

// Node terms of the node whose grid coordinates are already in T.i.
__device__ inline void node_terms_at(const SweepArgs& a, NodeTerms& T) {
#pragma clang fp contract(off)
  T.drift[3] = 0.0f;
  if (a.P.model != 1) {
    const double ri = a.rinv[T.i[0]];
    const double vr = a.G.lo[1] + (double)T.i[1] * a.G.h[1];
    const double vt = a.G.lo[2] + (double)T.i[2] * a.G.h[2];
    T.drift[0] = drift_r(a, T.i[1]);
    T.drift[1] = (float)(a.c1 * (vt * vt * ri - a.P.mu * ri * ri));
    T.drift[2] = (float)(-a.c2 * vr * vt * ri);
    // crown: theta' = v_t / r along axis 3
    if (a.P.model == 2) T.drift[3] = (float)(a.c3 * vt * ri);
  } else {
    T.drift[0] = T.drift[1] = T.drift[2] = 0.0f;
  }
  T.g1 = a.g1tab[T.i[3]];
  T.g2 = a.g2tab[T.i[3]];
  T.gm = a.gm;
}

__device__ inline int node_terms_tab(const SweepArgs& a, uint32_t packed, NodeTerms& T) {
  const int j = unpack_node(a.G, packed, T.i);
  node_terms_at(a, T);
  return j;
}

// Golden-section refinement around the centre angle u0 (sin/cos s0, c0) on
// [u0 - half, u0 + half]: two interior points u0 -+ half*rho^3, then one new
// point per step; the best evaluated point is kept (strict <, evaluation
// order).  The new point of step k is the previous point on the kept side
// moved by L0*rho^(k+4) (L0 = 2*half), because 2*rho - 1 = rho^3 and
// rho^2 - rho^3 = rho^4; its sin/cos are formed by rotating the previous
// point's sin/cos with the per-step constants rot = (sin, cos) of
// half*rho^3, then of L0*rho^(k+4) for k = 0, 1, ...  qf(sin, cos) returns
// the thrust Q at that angle.  Offsets from u0 are tracked in float for the
// stored angle.
struct GoldenState {
  float best_q, best_d;  // best Q and its offset from u0
  float best_s, best_c;  // its sin/cos as evaluated
};

template <class QF>
__device__ inline void golden(const QF& qf, float s0, float c0, float half, int steps, const float* __restrict__ rot,
                              GoldenState& g) {
  const float rho = 0.6180339887498949f;
  const float sp = rot[0], cp = rot[1];
  // the two interior points u0 -+ half*rho^3 (rho^3 = 2 rho - 1)
  const float x0 = half * 0.2360679774997897f;
  float xN = -x0, sN = fmaf(s0, cp, -c0 * sp), cN = fmaf(c0, cp, s0 * sp);  // left point
  float xK = x0, sK = fmaf(s0, cp, c0 * sp), cK = fmaf(c0, cp, -s0 * sp);   // right point
  float fN = qf(sN, cN);
  if (fN < g.best_q) {
    g.best_q = fN;
    g.best_d = xN;
    g.best_s = sN;
    g.best_c = cN;
  }
  float fK = qf(sK, cK);
  if (fK < g.best_q) {
    g.best_q = fK;
    g.best_d = xK;
    g.best_s = sK;
    g.best_c = cK;
  }
  // K: the interior point kept from the previous step; N: the point just
  // evaluated, on the left of K when nl.  Each step keeps the lower interior
  // point and places the new one symmetrically, at distance 2*half*rho^(k+4)
  // from it, by rotating (sin, cos) of the kept point.
  bool nl = true;
  float delta = 2.0f * half * 0.1458980337503155f;  // 2*half*rho^4
  for (int it = 0; it < steps; it++) {
    const float sd = rot[2 + 2 * it], cd = rot[3 + 2 * it];
    const float f_left = nl ? fN : fK, f_right = nl ? fK : fN;
    const bool left = f_left < f_right;  // the left point is the lower one
    const bool keepN = left == nl;
    const float xk = keepN ? xN : xK, sk = keepN ? sN : sK, ck = keepN ? cN : cK, fk = keepN ? fN : fK;
    const float sdd = left ? -sd : sd;
    sN = fmaf(sk, cd, ck * sdd);
    cN = fmaf(ck, cd, -sk * sdd);
    xN = left ? xk - delta : xk + delta;
    delta *= rho;
    xK = xk;
    sK = sk;
    cK = ck;
    fK = fk;
    nl = left;
    fN = qf(sN, cN);
    if (fN < g.best_q) {
      g.best_q = fN;
      g.best_d = xN;
      g.best_s = sN;
      g.best_c = cN;
    }
  }
}

// Exhaustive pass over the n_ang tabulated angles: first strict minimum.
// kWave: the 64 lanes of a wave search for one state together, lane l taking
// the entries l, l + 64, ...; the wave then keeps the smallest value with
// the lowest index among equal values, which is the same first strict
// minimum (entries whose Q is not below +inf are never taken, and with none
// taken the index is 0, as in the one-lane pass).  Every lane ends with the
// result; the caller's lanes must all be active.
template <bool kWave = false, class QF>
__device__ inline void scan_table(const QF& qf, const SweepArgs& a, float& bq, int& bk) {
  bq = INFINITY;
  bk = 0;
  if (!kWave) {
#pragma unroll 8
    for (int k = 0; k < a.n_ang; k++) {
      const float q = qf(a.tab_sin[k], a.tab_cos[k]);
      if (q < bq) {
        bq = q;
        bk = k;
      }
    }
    return;
  }
  int k_best = 0x7fffffff;
  for (int k = (int)(threadIdx.x & 63); k < a.n_ang; k += 64) {
    const float q = qf(a.tab_sin[k], a.tab_cos[k]);
    if (q < bq) {
      bq = q;
      k_best = k;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const float q2 = __shfl_xor(bq, o, 64);
    const int k2 = __shfl_xor(k_best, o, 64);
    if (q2 < bq || (q2 == bq && k2 < k_best)) {
      bq = q2;
      k_best = k2;
    }
  }
  bk = k_best == 0x7fffffff ? 0 : k_best;
}

// The outcome of the search at one node.
struct Choice {
  float v;       // min Q
  float ang;     // best thrust angle in [-pi, pi)
  float sn, cs;  // sin/cos of the best thrust angle as evaluated
  int thr;       // 1 = thrust
};

// Full search: scan, golden section around the best sample (if n_golden > 0),
// then thrust iff strictly below the coast value qc.
template <bool kWave = false, class QF>
__device__ inline void full_search(const QF& qf, const SweepArgs& a, float qc, Choice& ch) {
  float bq;
  int bk;
  scan_table<kWave>(qf, a, bq, bk);
  GoldenState g{bq, 0.0f, a.tab_sin[bk], a.tab_cos[bk]};
  if (a.n_golden > 0) golden(qf, a.tab_sin[bk], a.tab_cos[bk], a.half_width, a.n_golden, a.rot_scan, g);
  ch.thr = g.best_q < qc ? 1 : 0;
  ch.v = ch.thr ? g.best_q : qc;
  ch.ang = wrap_pi(a.tab_ang[bk] + g.best_d);
  ch.sn = g.best_s;
  ch.cs = g.best_c;
}

// Tabulated search: first strict minimum over the table, coast on ties.
template <bool kWave = false, class QF>
__device__ inline void table_search(const QF& qf, const SweepArgs& a, float qc, Choice& ch) {
  float bq;
  int bk;
  scan_table<kWave>(qf, a, bq, bk);
  ch.thr = bq < qc ? 1 : 0;
  ch.v = ch.thr ? bq : qc;
  ch.ang = a.tab_ang[bk];
  ch.sn = a.tab_sin[bk];
  ch.cs = a.tab_cos[bk];
}

// Seeded local search: the seed angle, then a golden section with n_local - 3
// steps on [seed - w, seed + w] (n_local thrust evaluations), then coast.
// Returns true when the result differs from the node's current value by more
// than fallback_tol * max(1, |V|): the node must repeat the full search.
template <class QF>
__device__ inline bool seeded_local(const QF& qf, const SweepArgs& a, float seed, float qc, float vin, Choice& ch) {
  float s0, c0;
  sincosf(seed, &s0, &c0);
  GoldenState g{qf(s0, c0), 0.0f, s0, c0};
  golden(qf, s0, c0, a.local_half_width, a.n_local - 3, a.rot_local, g);
  ch.thr = g.best_q < qc ? 1 : 0;
  ch.v = ch.thr ? g.best_q : qc;
  ch.ang = wrap_pi(seed + g.best_d);
  ch.sn = g.best_s;
  ch.cs = g.best_c;
  return fabsf(ch.v - vin) > a.fallback_tol * fmaxf(1.0f, fabsf(vin));
}

// Table index nearest to the angle u on the circle (halves round up); 0 for
// a non-finite u.  Exact for the table's own angles, whose distance to an
// index is ~1e-6 of a step.
__device__ inline int table_index(float u, int K) {
  if (!(fabsf(u) <= 1.0e30f)) return 0;
  const float t = floorf((u + 3.14159265358979f) * ((float)K * 0.159154943091895f) + 0.5f);
  const int k = (int)(t - (float)K * floorf(t / (float)K));
  return (k >= 0 && k < K) ? k : 0;
}

// sin/cos of a stored policy angle, as the greedy step formed them: an angle
// that is one of the tabulated controls (or scan samples) takes the table's
// values, which the search evaluated it with; any other angle (golden-section
// and seeded points, formed there by rotation recurrences) takes sincosf.
__device__ inline void policy_sincos(const SweepArgs& a, float u, float& sn, float& cs) {
  if (a.n_ang > 0) {
    const int k = table_index(u, a.n_ang);
    if (a.tab_ang[k] == u) {
      sn = a.tab_sin[k];
      cs = a.tab_cos[k];
      return;
    }
  }
  sincosf(u, &sn, &cs);
}

// Walk over the tabulated angles from the previous optimum (paper Section 3,
// "Efficient computation of the minimum"): start at the table angle nearest
// to u_prev, look at both cyclic neighbours, move to the lower one if it is
// strictly below (the k-1 side when the two are equal), then keep moving the
// same way while the next angle is strictly lower (the angle just left is
// higher, so it never needs another look).  Thrust iff the walk's Q is
// strictly below the coast value.  At most K + 2 evaluations; returns their
// number.
template <class QF>
__device__ inline int walk_search(const QF& qf, const SweepArgs& a, float u_prev, float qc, Choice& ch) {
  const int K = a.n_ang;
  int k = table_index(u_prev, K);
  const int km = k == 0 ? K - 1 : k - 1, kp = k == K - 1 ? 0 : k + 1;
  float qk = qf(a.tab_sin[k], a.tab_cos[k]);
  const float qm = qf(a.tab_sin[km], a.tab_cos[km]);
  const float qp = qf(a.tab_sin[kp], a.tab_cos[kp]);
  int n = 3;
  int d = 0;
  if (qm < qk && qm <= qp) d = -1;
  else if (qp < qk) d = 1;
  if (d != 0) {
    k = d < 0 ? km : kp;
    qk = d < 0 ? qm : qp;
    for (int it = 0; it < K; it++) {
      int kn = k + d;
      kn = kn < 0 ? K - 1 : (kn >= K ? 0 : kn);
      const float qn = qf(a.tab_sin[kn], a.tab_cos[kn]);
      n++;
      if (!(qn < qk)) break;
      k = kn;
      qk = qn;
    }
  }
  ch.thr = qk < qc ? 1 : 0;
  ch.v = ch.thr ? qk : qc;
  ch.ang = a.tab_ang[k];
  ch.sn = a.tab_sin[k];
  ch.cs = a.tab_cos[k];
  return n;
}

// Adds the workgroup's sum of v to acc[blockIdx.x] (each workgroup owns its
// entry, so successive sweeps on one stream accumulate without atomics).
// Every thread of the workgroup must call it.
__device__ inline void block_add_count(int v, unsigned long long* acc) {
  __shared__ int wsum[kMaxBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) wsum[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) s += wsum[i];
    acc[blockIdx.x] += (unsigned long long)s;
  }
}

// At most this many fallback lanes of a wave are deferred to the second pass.
constexpr int kDeferLanes = 16;

// Seeded search with the fallback done in place.
template <class QF>
__device__ inline int seeded_search(const QF& qf, const SweepArgs& a, float seed, float qc, float vin, Choice& ch) {
  if (seeded_local(qf, a, seed, qc, vin, ch)) {
    full_search(qf, a, qc, ch);
    return 1;
  }
  return 0;
}

// Policy iteration's greedy step also evaluates the node's current control
// (pol_thr_in / pol_ang_in, read before the node's outputs are written) and
// keeps it unless the search found a strictly smaller Q.  The scan + golden
// search is only approximately the argmin; with the incumbent as a candidate
// the greedy value never exceeds the current policy's, so policy iteration
// from above decreases monotonically instead of alternating between two
// nearly tied basins.
template <class QF>
__device__ inline void keep_incumbent(const QF& qf, const SweepArgs& a, int j, float qc, Choice& ch) {
  if (!a.pol_thr_in) return;
  const int thr0 = a.pol_thr_in[j] ? 1 : 0;
  const float u0 = a.pol_ang_in[j];
  float s0 = 0.0f, c0 = 1.0f, q0 = qc;
  if (thr0) {
    policy_sincos(a, u0, s0, c0);
    q0 = qf(s0, c0);
  }
  if (q0 <= ch.v) {
    ch.v = q0;
    ch.ang = u0;
    ch.sn = s0;
    ch.cs = c0;
    ch.thr = thr0;
  }
}

// Foot descriptor of the chosen control (see SweepArgs::desc_code).
__device__ inline void write_desc(const SweepArgs& a, int t, int j, const NodeTerms& T, const Choice& ch) {
  float off[4];
  off[0] = T.drift[0];
  off[1] = ch.thr ? fmaf(T.g1, ch.sn, T.drift[1]) : T.drift[1];
  off[2] = ch.thr ? fmaf(T.g2, ch.cs, T.drift[2]) : T.drift[2];
  off[3] = T.drift[3] + (ch.thr ? T.gm : 0.0f);
  int base[4];
  float w[4];
  const bool inside = foot_cell(a.G, T.i, off, base, w);
  const float2 wv = inside ? make_float2(w[1], w[2]) : make_float2(0.0f, 0.0f);
  if (a.desc_pk) {
    uint32_t code = ch.thr ? kDescThr : 0;
    if (inside) code |= (uint32_t)((base[1] - T.i[1] + 32) | ((base[2] - T.i[2] + 32) << 6));
    else code |= kDescOut;
    a.desc_pk[j] = desc_pack(code, wv.x, wv.y);
    return;
  }
  if (a.desc16) {
    const int k = a.desc_dense ? j : t;
    uint16_t code = ch.thr ? kDescThr : 0;
    if (inside) code |= (uint16_t)((base[1] - T.i[1] + 32) | ((base[2] - T.i[2] + 32) << 6));
    else code |= kDescOut;
    a.desc16[k] = code;
    a.desc_w[k] = wv;
    return;
  }
  const unsigned flat = inside ? (unsigned)(base[0] + base[1] * a.G.st[1] + base[2] * a.G.st[2] + base[3] * a.G.st[3])
                               : (1u << 30);
  a.desc_code[t] = (int)(flat | ((unsigned)ch.thr << 31));
  a.desc_w[t] = wv;
}

// ---- fast path for thrust controls.
// Under thrust the r displacement (v_r * dt) and the m displacement (-c*dt)
// do not depend on the angle, so every thrust foot of a node shares its r and
// m cell and weights; only the v_r and v_t displacements move, by at most
// |g| < 0.5 cell around the coast foot.  The node therefore collapses its
// neighbourhood over r and m once (36 corner values, 27 lerps) into a 3 x 3
// patch over (v_r, v_t), and every thrust evaluation is the bilinear
// interpolant of the patch cell its foot falls in: the same Q1 value as the
// 16-corner sum, with the lerps reordered.  Along each of v_r, v_t the feet
// span at most two regions split at one threshold (a node or a domain face);
// a region outside the domain has the constant value M.  The four region
// pairs are stored per thread in LDS as Q = A + B dv + C dt + D dv dt in the
// displacements dv = g1 sin u, dt = g2 cos u from the coast foot.
struct Regions {
  int b0;     // first cell (node index) of region 0; region 1 is cell b0 + 1
  float bnd;  // region 1 <=> displacement offset >= bnd (node offsets)
  bool ok0, ok1;
};

// Smallest float above x (x finite; 0 maps to the smallest normal float).
__device__ inline float next_up(float x) {
  if (x == 0.0f) return 1.17549435e-38f;
  return __int_as_float(__float_as_int(x) + (x > 0.0f ? 1 : -1));
}

__device__ inline Regions axis_regions(int i, int n, float d, float g) {
  Regions R;
  const float ag = fabsf(g) + 1e-6f;  // margin over the rounding of d + g*s
  const float lo = d - ag, hi = d + ag;
  const float top = (float)(n - 1 - i), bot = (float)(-i);
  if (hi < bot || lo > top) {  // every foot outside
    R.b0 = 0;
    R.bnd = INFINITY;
    R.ok0 = R.ok1 = false;
    return R;
  }
  const float k = floorf(hi);
  const int kk = i + (int)k;
  if (kk >= n - 1) {  // reaches the top face: last cell, then outside (the face itself is inside)
    R.b0 = n - 2;
    R.bnd = next_up(top);
    R.ok0 = true;
    R.ok1 = false;
  } else if (k > lo) {  // crosses node kk (kk == 0: the bottom face)
    R.b0 = kk - 1;
    R.bnd = k;
    R.ok0 = kk - 1 >= 0;
    R.ok1 = true;
  } else {  // one cell
    R.b0 = kk;
    R.bnd = INFINITY;
    R.ok0 = true;
    R.ok1 = false;
  }
  return R;
}

struct FastNode {
  float g1, g2;  // thrust displacement per unit sin u (v_r) and cos u (v_t), cells
  float d1, d2;  // coast displacements along v_r and v_t
  float bv, bt;  // region 1 <=> offset >= threshold (the same float test as foot_cell)
  const char* coef;  // this thread's first region pair in LDS
  int offv, offt;    // byte offsets of the region pairs with v_r region 1 / v_t region 1
};

__device__ inline float fast_q(const FastNode& F, float sn, float cs) {
  const float ov = fmaf(F.g1, sn, F.d1), ot = fmaf(F.g2, cs, F.d2);
  const int off = (ov >= F.bv ? F.offv : 0) + (ot >= F.bt ? F.offt : 0);
  const float4 c = *reinterpret_cast<const float4*>(F.coef + off);
  const float dv = ov - F.d1, dt = ot - F.d2;
  return fmaf(fmaf(c.w, dt, c.y), dv, fmaf(c.z, dt, c.x));
}

// Lerp along r of the corner pair (p[0], p[1]), fetched by one 8-byte load.
__device__ inline float lerp_pair(const float* p, float t) {
  const CornerPair v = *reinterpret_cast<const CornerPair*>(p);
  return lerp(v.lo, v.hi, t);
}

// Per-node set-up of the thrust evaluations; returns the coast Q, which is
// the same Q1 value read from the patch (plane i_m, coast cell).
// lds: 4 * blockDim.x float4, laid out [region pair][thread].
__device__ inline float fast_setup(const SweepArgs& a, const NodeTerms& T, float4* lds, FastNode& F) {
  const Grid& G = a.G;
  F.g1 = T.g1;
  F.g2 = T.g2;
  F.d1 = T.drift[1];
  F.d2 = T.drift[2];
  F.offv = 2 * (int)blockDim.x * (int)sizeof(float4);
  F.offt = (int)blockDim.x * (int)sizeof(float4);
  F.coef = reinterpret_cast<const char*>(lds + threadIdx.x);
  // r cell, shared by every control
  int br = 0, bm = 0;
  float tr = 0.0f, tm = 0.0f;
  const bool ok_r = axis_cell(T.i[0], G.n[0], T.drift[0], br, tr);
  // m cell under thrust; the coast foot stays on plane i_m
  const bool ok_m = axis_cell(T.i[3], G.n[3], T.gm, bm, tm);
  const int m_lo = ok_m ? bm : T.i[3];
  const int m_hi = ok_m ? bm + 1 : T.i[3];
  const int coast_plane = T.i[3];  // either m_lo or m_hi
  const Regions Rv = axis_regions(T.i[1], G.n[1], T.drift[1], T.g1);
  const Regions Rt = axis_regions(T.i[2], G.n[2], T.drift[2], T.g2);
  F.bv = Rv.bnd;
  F.bt = Rt.bnd;
  const float qM = fmaf(a.P.gamma, a.P.M, a.P.q_thr);
  float W[3][3], Wc[3][3];
  if (ok_r) {
    const float* __restrict__ base = a.V_in + br + m_lo * G.st[3];
    const int so = (m_hi - m_lo) * G.st[3];
#pragma unroll
    for (int p = 0; p < 3; p++) {
      const int v = min(max(Rv.b0 + p, 0), G.n[1] - 1);
      // the row's six corner pairs are loaded before any of them is used,
      // so that their latencies overlap
      CornerPair lo[3], hi[3];
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const int w = min(max(Rt.b0 + q, 0), G.n[2] - 1);
        const float* pp = base + v * G.st[1] + w * G.st[2];
        lo[q] = *reinterpret_cast<const CornerPair*>(pp);
        hi[q] = *reinterpret_cast<const CornerPair*>(pp + so);
      }
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const float l = lerp(lo[q].lo, lo[q].hi, tr), h = lerp(hi[q].lo, hi[q].hi, tr);
        W[p][q] = lerp(l, h, tm);
        Wc[p][q] = coast_plane == m_lo ? l : h;
      }
    }
  }
  const float gam = a.P.gamma, q0 = a.P.q_thr;
#pragma unroll
  for (int av = 0; av < 2; av++) {
#pragma unroll
    for (int bt = 0; bt < 2; bt++) {
      float4 c = make_float4(qM, 0.0f, 0.0f, 0.0f);
      const bool valid = ok_r && ok_m && (av ? Rv.ok1 : Rv.ok0) && (bt ? Rt.ok1 : Rt.ok0);
      if (valid) {
        const float w00 = W[av][bt], w10 = W[av + 1][bt], w01 = W[av][bt + 1], w11 = W[av + 1][bt + 1];
        // local coordinates of the coast foot in this cell
        const float tv = T.drift[1] - (float)(Rv.b0 + av - T.i[1]);
        const float tt = T.drift[2] - (float)(Rt.b0 + bt - T.i[2]);
        const float cv = w10 - w00, ct = w01 - w00, dd = (w11 - w10) - (w01 - w00);
        const float A = lerp(lerp(w00, w10, tv), lerp(w01, w11, tv), tt);
        c.x = fmaf(gam, A, q0);
        c.y = gam * fmaf(dd, tt, cv);
        c.z = gam * fmaf(dd, tv, ct);
        c.w = gam * dd;
      }
      lds[(av * 2 + bt) * blockDim.x + threadIdx.x] = c;
    }
  }
  // coast: the cell of (d1, d2) on plane i_m, by the same region tests
  const int av = T.drift[1] >= Rv.bnd ? 1 : 0;
  const int bt = T.drift[2] >= Rt.bnd ? 1 : 0;
  const bool cvalid = ok_r && (av ? Rv.ok1 : Rv.ok0) && (bt ? Rt.ok1 : Rt.ok0);
  float Ic = a.P.M;
  if (cvalid) {
    const float tv = T.drift[1] - (float)(Rv.b0 + av - T.i[1]);
    const float tt = T.drift[2] - (float)(Rt.b0 + bt - T.i[2]);
    float w00, w10, w01, w11;
    // select the coast cell of the 3 x 3 patch (av, bt in {0, 1})
    w00 = av ? (bt ? Wc[1][1] : Wc[1][0]) : (bt ? Wc[0][1] : Wc[0][0]);
    w10 = av ? (bt ? Wc[2][1] : Wc[2][0]) : (bt ? Wc[1][1] : Wc[1][0]);
    w01 = av ? (bt ? Wc[1][2] : Wc[1][1]) : (bt ? Wc[0][2] : Wc[0][1]);
    w11 = av ? (bt ? Wc[2][2] : Wc[2][1]) : (bt ? Wc[1][2] : Wc[1][1]);
    Ic = lerp(lerp(w00, w10, tv), lerp(w01, w11, tv), tt);
  }
  return fmaf(a.P.gamma, Ic, a.P.q_coast);
}


// One free node of a sweep on the factorised path: search, outputs and the
// residual contributions.  kMode: 0 tabulated, 1 scan + golden, 2 seeded.
template <int kMode>
__device__ inline void fast_node(const SweepArgs& a, int t, float4* lds, double& rel, double& sum, double& mabs,
                                 double& bad, int& fell_back, int& deferred, int& evals) {
  NodeTerms T;
  const int j = node_terms_tab(a, a.free_node[t], T);
  FastNode F;
  const float qc = fast_setup(a, T, lds, F);
  auto qf = [&](float sn, float cs) { return fast_q(F, sn, cs); };
  const float vin = a.V_in[j];
  Choice ch;
  if (kMode == 0) table_search(qf, a, qc, ch);
  else if (kMode == 1) full_search(qf, a, qc, ch);
  else if (kMode == 3) evals = walk_search(qf, a, a.walk_from[j], qc, ch);
  else {
    const bool need = seeded_local(qf, a, a.seed[j], qc, vin, ch);
    // A wave where only a few lanes fall back would leave the others idle
    // through a full search: those lanes are listed for a second pass.
    // Where many lanes fall back, the wave does the full search in place.
    const bool few = __popcll(__ballot(need)) <= kDeferLanes;
    if (need) {
      fell_back = 1;
      if (a.fb_list && few) {
        deferred = 1;
        return;
      }
      full_search(qf, a, qc, ch);
    }
  }
  keep_incumbent(qf, a, j, qc, ch);
  a.V_out[j] = ch.v;
  if (a.pol_ang) a.pol_ang[j] = ch.ang;
  if (a.pol_thr) a.pol_thr[j] = (uint8_t)ch.thr;
  if (a.desc_code || a.desc16 || a.desc_pk) write_desc(a, t, j, T, ch);
  node_residual(vin, ch.v, rel, sum, mabs, bad);
}

}  // namespace dpo
