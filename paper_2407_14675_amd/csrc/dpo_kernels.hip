// HIP kernels of libdpo for gfx950: classification and compaction of the
// reduced grid, Bellman sweeps (tabulated search, scan + golden section,
// seeded local search), frozen-policy sweeps, FP64 residual reduction,
// FP64 read-out, feedback, reachability mask and probes.
//
// Paper: arXiv 2407.14675, Section 3 (eq:schema, value and policy iteration,
// minimisation by tabulation and golden section, feedback eq:feed).
#include "dpo_kernels.h"

namespace dpo {

// ------------------------------------------------------------------ a1
// Node kinds: target (V = 0) if every |x_k - c_k| <= w_k + h_k/2; else
// inactive if the mask says so; else free.  FP64 without contraction so the
// decision is the same one the plain definition gives.
__global__ __launch_bounds__(kBlock) void k_classify(Grid G, TargetBox tb, const uint8_t* __restrict__ mask,
                                                     uint8_t* __restrict__ kind, int N) {
#pragma clang fp contract(off)
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= N) return;
  int i[4];
  decode_node(G, j, i);
  bool target = true;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const double prod = (double)i[k] * G.h[k];
    const double x = G.lo[k] + prod;
    const double lim = tb.w[k] + 0.5 * G.h[k];
    if (!(fabs(x - tb.c[k]) <= lim)) target = false;
  }
  uint8_t kd = 0;
  if (target) kd = 1;
  else if (mask != nullptr && mask[j] == 0) kd = 2;
  kind[j] = kd;
}

// Compaction of free nodes, in node order: per-chunk counts, one exclusive
// scan over the chunks, then an ordered scatter using wave ballots.
constexpr int kChunk = kBlock * 16;

__global__ __launch_bounds__(kBlock) void k_count_free(const uint8_t* __restrict__ kind, int N,
                                                       int* __restrict__ counts) {
  __shared__ int red[kBlock / 64];
  const int base = blockIdx.x * kChunk;
  int c = 0;
  for (int e = threadIdx.x; e < kChunk; e += kBlock) {
    const int j = base + e;
    if (j < N && kind[j] == 0) c++;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < kBlock / 64; w++) s += red[w];
    counts[blockIdx.x] = s;
  }
}

// Single workgroup: exclusive scan of nchunks counts (sequential per thread
// slice, then across threads); total written to offsets[nchunks].
__global__ __launch_bounds__(1024) void k_scan_counts(const int* __restrict__ counts, int nchunks,
                                                      int* __restrict__ offsets) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (nchunks + 1023) / 1024;
  const int lo = t * per, hi = min(nchunks, lo + per);
  int s = 0;
  for (int c = lo; c < hi; c++) s += counts[c];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int w = 0; w < 1024; w++) {
      const int v = part[w];
      part[w] = acc;
      acc += v;
    }
    offsets[nchunks] = acc;
  }
  __syncthreads();
  int acc = part[t];
  for (int c = lo; c < hi; c++) {
    offsets[c] = acc;
    acc += counts[c];
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter_free(Grid G, const uint8_t* __restrict__ kind, int N,
                                                         const int* __restrict__ offsets,
                                                         uint32_t* __restrict__ free_node) {
  __shared__ int wave_tot[kBlock / 64];
  __shared__ int running;
  const int base = blockIdx.x * kChunk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) running = offsets[blockIdx.x];
  __syncthreads();
  for (int e0 = 0; e0 < kChunk; e0 += kBlock) {
    const int j = base + e0 + threadIdx.x;
    const bool f = (j < N) && kind[j] == 0;
    const unsigned long long bal = __ballot(f);
    const int below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wave] = __popcll(bal);
    __syncthreads();
    int wave_off = 0;
    for (int w = 0; w < wave; w++) wave_off += wave_tot[w];
    if (f) {
      int i[4];
      decode_node(G, j, i);
      free_node[running + wave_off + below] = pack_node(i);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int s = 0;
      for (int w = 0; w < kBlock / 64; w++) s += wave_tot[w];
      running += s;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_init_value(const uint8_t* __restrict__ kind, float M,
                                                       float* __restrict__ V, int N) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < N) V[j] = (kind[j] == 1) ? 0.0f : M;
}

// --------------------------------------------------------------- a2..a8
// Node terms from the packed coordinates of a free node and the per-axis
// tables: FP64 for the control-independent drift, float for the rest.
// The r displacement dt*v_r/h_r (cells) of nodes in v_r row i1.
__device__ inline float drift_r(const SweepArgs& a, int i1) {
  if (a.P.model != 0) return 0.0f;
  const double vr = a.G.lo[1] + (double)i1 * a.G.h[1];
  return (float)(a.c0 * vr);
}

__device__ inline int node_terms_tab(const SweepArgs& a, uint32_t packed, NodeTerms& T) {
  const int j = unpack_node(a.G, packed, T.i);
  if (a.P.model == 0) {
    const double ri = a.rinv[T.i[0]];
    const double vr = a.G.lo[1] + (double)T.i[1] * a.G.h[1];
    const double vt = a.G.lo[2] + (double)T.i[2] * a.G.h[2];
    T.drift[0] = drift_r(a, T.i[1]);
    T.drift[1] = (float)(a.c1 * (vt * vt * ri - a.P.mu * ri * ri));
    T.drift[2] = (float)(-a.c2 * vr * vt * ri);
  } else {
    T.drift[0] = T.drift[1] = T.drift[2] = 0.0f;
  }
  T.drift[3] = 0.0f;
  T.g1 = a.g1tab[T.i[3]];
  T.g2 = a.g2tab[T.i[3]];
  T.gm = a.gm;
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
  float lo = -half, hi = half;
  float x1 = hi - rho * (hi - lo), x2 = lo + rho * (hi - lo);
  const float sp = rot[0], cp = rot[1];
  float s1 = fmaf(s0, cp, -c0 * sp), c1 = fmaf(c0, cp, s0 * sp);  // u0 - half*rho^3
  float s2 = fmaf(s0, cp, c0 * sp), c2 = fmaf(c0, cp, -s0 * sp);  // u0 + half*rho^3
  float f1 = qf(s1, c1);
  if (f1 < g.best_q) {
    g.best_q = f1;
    g.best_d = x1;
    g.best_s = s1;
    g.best_c = c1;
  }
  float f2 = qf(s2, c2);
  if (f2 < g.best_q) {
    g.best_q = f2;
    g.best_d = x2;
    g.best_s = s2;
    g.best_c = c2;
  }
  for (int it = 0; it < steps; it++) {
    const float sd = rot[2 + 2 * it], cd = rot[3 + 2 * it];
    const bool left = f1 < f2;  // keep [lo, x2]; new point left of x1
    float xn, sn, cn;
    if (left) {
      hi = x2;
      x2 = x1;
      f2 = f1;
      xn = hi - rho * (hi - lo);
      sn = fmaf(s1, cd, -c1 * sd);
      cn = fmaf(c1, cd, s1 * sd);
      s2 = s1;
      c2 = c1;
    } else {
      lo = x1;
      x1 = x2;
      f1 = f2;
      xn = lo + rho * (hi - lo);
      sn = fmaf(s2, cd, c2 * sd);
      cn = fmaf(c2, cd, -s2 * sd);
      s1 = s2;
      c1 = c2;
    }
    const float fn = qf(sn, cn);
    if (left) {
      x1 = xn;
      s1 = sn;
      c1 = cn;
      f1 = fn;
    } else {
      x2 = xn;
      s2 = sn;
      c2 = cn;
      f2 = fn;
    }
    if (fn < g.best_q) {
      g.best_q = fn;
      g.best_d = xn;
      g.best_s = sn;
      g.best_c = cn;
    }
  }
}

// Exhaustive pass over the n_ang tabulated angles: first strict minimum.
template <class QF>
__device__ inline void scan_table(const QF& qf, const SweepArgs& a, float& bq, int& bk) {
  bq = INFINITY;
  bk = 0;
  for (int k = 0; k < a.n_ang; k++) {
    const float q = qf(a.tab_sin[k], a.tab_cos[k]);
    if (q < bq) {
      bq = q;
      bk = k;
    }
  }
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
template <class QF>
__device__ inline void full_search(const QF& qf, const SweepArgs& a, float qc, Choice& ch) {
  float bq;
  int bk;
  scan_table(qf, a, bq, bk);
  GoldenState g{bq, 0.0f, a.tab_sin[bk], a.tab_cos[bk]};
  if (a.n_golden > 0) golden(qf, a.tab_sin[bk], a.tab_cos[bk], a.half_width, a.n_golden, a.rot_scan, g);
  ch.thr = g.best_q < qc ? 1 : 0;
  ch.v = ch.thr ? g.best_q : qc;
  ch.ang = wrap_pi(a.tab_ang[bk] + g.best_d);
  ch.sn = g.best_s;
  ch.cs = g.best_c;
}

// Tabulated search: first strict minimum over the table, coast on ties.
template <class QF>
__device__ inline void table_search(const QF& qf, const SweepArgs& a, float qc, Choice& ch) {
  float bq;
  int bk;
  scan_table(qf, a, bq, bk);
  ch.thr = bq < qc ? 1 : 0;
  ch.v = ch.thr ? bq : qc;
  ch.ang = a.tab_ang[bk];
  ch.sn = a.tab_sin[bk];
  ch.cs = a.tab_cos[bk];
}

// Seeded local search: the seed angle, then a golden section with n_local - 3
// steps on [seed - w, seed + w] (n_local thrust evaluations), then coast.  A
// node whose result differs from its current value by more than
// fallback_tol * max(1, |V|) repeats the full search.
template <class QF>
__device__ inline int seeded_search(const QF& qf, const SweepArgs& a, float seed, float qc, float vin, Choice& ch) {
  float s0, c0;
  sincosf(seed, &s0, &c0);
  GoldenState g{qf(s0, c0), 0.0f, s0, c0};
  golden(qf, s0, c0, a.local_half_width, a.n_local - 3, a.rot_local, g);
  ch.thr = g.best_q < qc ? 1 : 0;
  ch.v = ch.thr ? g.best_q : qc;
  ch.ang = wrap_pi(seed + g.best_d);
  ch.sn = g.best_s;
  ch.cs = g.best_c;
  if (fabsf(ch.v - vin) > a.fallback_tol * fmaxf(1.0f, fabsf(vin))) {
    full_search(qf, a, qc, ch);
    return 1;
  }
  return 0;
}

// Foot descriptor of the chosen control (see SweepArgs::desc_code).
__device__ inline void write_desc(const SweepArgs& a, int t, const NodeTerms& T, const Choice& ch) {
  float off[4];
  off[0] = T.drift[0];
  off[1] = ch.thr ? fmaf(T.g1, ch.sn, T.drift[1]) : T.drift[1];
  off[2] = ch.thr ? fmaf(T.g2, ch.cs, T.drift[2]) : T.drift[2];
  off[3] = T.drift[3] + (ch.thr ? T.gm : 0.0f);
  int base[4];
  float w[4];
  const bool inside = foot_cell(a.G, T.i, off, base, w);
  const unsigned flat = inside ? (unsigned)(base[0] + base[1] * a.G.st[1] + base[2] * a.G.st[2] + base[3] * a.G.st[3])
                               : (1u << 30);
  a.desc_code[t] = (int)(flat | ((unsigned)ch.thr << 31));
  a.desc_w[t] = inside ? make_float2(w[1], w[2]) : make_float2(0.0f, 0.0f);
}

// ---- direct path: every evaluation gathers its 16 corners from V.
// Used for any problem; the fast path below covers the orbit workloads.
template <int kMode>
__global__ __launch_bounds__(kBlock) void k_sweep_direct(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  int fell_back = 0;
  if (t < a.n_free) {
    NodeTerms T;
    const int j = node_terms_tab(a, a.free_node[t], T);
    const float* __restrict__ V = a.V_in;
    auto qf = [&](float sn, float cs) { return q_thrust(V, a.G, a.P, T, sn, cs); };
    const float qc = q_coast(V, a.G, a.P, T);
    const float vin = V[j];
    Choice ch;
    if (kMode == 0) table_search(qf, a, qc, ch);
    else if (kMode == 1) full_search(qf, a, qc, ch);
    else fell_back = seeded_search(qf, a, a.seed[j], qc, vin, ch);
    a.V_out[j] = ch.v;
    if (a.pol_ang) a.pol_ang[j] = ch.ang;
    if (a.pol_thr) a.pol_thr[j] = (uint8_t)ch.thr;
    if (a.desc_code) write_desc(a, t, T, ch);
    node_residual(vin, ch.v, rel, sum, mabs, bad);
  }
  block_residual(rel, sum, mabs, bad, (double)fell_back, a.partial, blockIdx.x);
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
  const float4* coef;
};

__device__ inline float fast_q(const FastNode& F, float sn, float cs) {
  const float ov = fmaf(F.g1, sn, F.d1), ot = fmaf(F.g2, cs, F.d2);
  const int idx = (ov >= F.bv ? 2 * kBlock : 0) + (ot >= F.bt ? kBlock : 0);
  const float4 c = F.coef[idx];
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
__device__ inline float fast_setup(const SweepArgs& a, const NodeTerms& T, float4 (*coef)[kBlock], FastNode& F) {
  const Grid& G = a.G;
  F.g1 = T.g1;
  F.g2 = T.g2;
  F.d1 = T.drift[1];
  F.d2 = T.drift[2];
  F.coef = &coef[0][threadIdx.x];
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
    const float* __restrict__ base = a.V_in + br;
    const int so = (m_hi - m_lo) * G.st[3];
#pragma unroll
    for (int p = 0; p < 3; p++) {
      const int v = min(max(Rv.b0 + p, 0), G.n[1] - 1);
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const int w = min(max(Rt.b0 + q, 0), G.n[2] - 1);
        const float* pp = base + v * G.st[1] + w * G.st[2] + m_lo * G.st[3];
        const float lo = lerp_pair(pp, tr);
        const float hi = lerp_pair(pp + so, tr);
        W[p][q] = lerp(lo, hi, tm);
        Wc[p][q] = coast_plane == m_lo ? lo : hi;
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
      coef[av * 2 + bt][threadIdx.x] = c;
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

template <int kMode>
__global__ __launch_bounds__(kBlock) void k_sweep_fast(SweepArgs a) {
  __shared__ float4 s_coef[4][kBlock];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  int fell_back = 0;
  if (t < a.n_free) {
    NodeTerms T;
    const int j = node_terms_tab(a, a.free_node[t], T);
    FastNode F;
    const float qc = fast_setup(a, T, s_coef, F);
    auto qf = [&](float sn, float cs) { return fast_q(F, sn, cs); };
    const float vin = a.V_in[j];
    Choice ch;
    if (kMode == 0) table_search(qf, a, qc, ch);
    else if (kMode == 1) full_search(qf, a, qc, ch);
    else fell_back = seeded_search(qf, a, a.seed[j], qc, vin, ch);
    a.V_out[j] = ch.v;
    if (a.pol_ang) a.pol_ang[j] = ch.ang;
    if (a.pol_thr) a.pol_thr[j] = (uint8_t)ch.thr;
    if (a.desc_code) write_desc(a, t, T, ch);
    node_residual(vin, ch.v, rel, sum, mabs, bad);
  }
  block_residual(rel, sum, mabs, bad, (double)fell_back, a.partial, blockIdx.x);
}

// Frozen-policy sweep (eq:p_eval applied once).  The residual reduction is
// only compiled in when a caller asks for it; the policy-iteration loop does
// not, since it stops on the residual of the greedy step.
template <bool kResid>
__global__ __launch_bounds__(kBlock) void k_policy_eval(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  if (t < a.n_free) {
    NodeTerms T;
    const int j = node_terms_tab(a, a.free_node[t], T);
    float v;
    if (a.pol_thr_in[j]) {
      float sn, cs;
      __sincosf(a.pol_ang_in[j], &sn, &cs);
      v = q_thrust(a.V_in, a.G, a.P, T, sn, cs);
    } else {
      v = q_coast(a.V_in, a.G, a.P, T);
    }
    a.V_out[j] = v;
    if (kResid) node_residual(a.V_in[j], v, rel, sum, mabs, bad);
  }
  if (kResid) block_residual(rel, sum, mabs, bad, 0.0, a.partial, blockIdx.x);
}

// Frozen-policy sweep from the foot descriptors written by the last greedy
// sweep: per node the packed coordinates and the 12-byte descriptor in one
// coalesced trip, the r and m cell coordinates recomputed, 16 gathers and 15
// lerps.  Each workgroup owns kDescNpt * kBlock consecutive free nodes; every
// thread handles kDescNpt of them so their loads are in flight together.
constexpr int kDescNpt = 2;

__global__ __launch_bounds__(kBlock) void k_policy_eval_desc(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t0 = tile * (kDescNpt * kBlock) + threadIdx.x;
  uint32_t packed[kDescNpt];
  int code[kDescNpt];
  float2 w[kDescNpt];
#pragma unroll
  for (int k = 0; k < kDescNpt; k++) {
    const int t = t0 + k * kBlock;
    if (t < a.n_free) {
      packed[k] = a.free_node[t];
      code[k] = a.desc_code_in[t];
      w[k] = a.desc_w_in[t];
    }
  }
#pragma unroll
  for (int k = 0; k < kDescNpt; k++) {
    const int t = t0 + k * kBlock;
    if (t >= a.n_free) continue;
    int i[4];
    const int j = unpack_node(a.G, packed[k], i);
    const bool thr = code[k] < 0;
    float I = a.P.M;
    if (!(code[k] & (1 << 30))) {
      // r and m cell coordinates, exactly as the greedy sweep formed them
      const float o0 = drift_r(a, i[1]);
      int b0, b3;
      float tt[4];
      axis_cell(i[0], a.G.n[0], o0, b0, tt[0]);
      axis_cell(i[3], a.G.n[3], thr ? a.gm : 0.0f, b3, tt[3]);
      tt[1] = w[k].x;
      tt[2] = w[k].y;
      I = cell_value(a.V_in + (code[k] & 0x3fffffff), a.G, tt);
    }
    a.V_out[j] = fmaf(a.P.gamma, I, thr ? a.P.q_thr : a.P.q_coast);
  }
}

// Final FP64 reduction of the workgroup partials in a fixed order.
__global__ __launch_bounds__(kBlock) void k_resid_final(const double* __restrict__ partial, int nblocks,
                                                        double* __restrict__ out) {
  __shared__ double red[kPartial][kBlock];
  double acc[kPartial] = {0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < nblocks; i += kBlock) {
    acc[0] = fmax(acc[0], partial[kPartial * i + 0]);
    acc[1] += partial[kPartial * i + 1];
    acc[2] = fmax(acc[2], partial[kPartial * i + 2]);
    acc[3] += partial[kPartial * i + 3];
    acc[4] += partial[kPartial * i + 4];
  }
  for (int q = 0; q < kPartial; q++) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int s = kBlock / 2; s >= 1; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + s]);
      red[3][threadIdx.x] += red[3][threadIdx.x + s];
      red[4][threadIdx.x] += red[4][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < kPartial; q++) out[q] = red[q][0];
}

// ------------------------------------------------------------------ a9
// FP64 grid coordinate of a physical coordinate, with points within 1e-6
// cells of a face put on the face.
__device__ inline double to_grid(const Grid& G, int k, double x) {
  double s = (x - G.lo[k]) * G.inv_h[k];
  const double top = (double)(G.n[k] - 1);
  if (s < 0.0 && s > -1e-6) s = 0.0;
  if (s > top && s < top + 1e-6) s = top;
  return s;
}

// FP64 Q1 read-out at one physical state.
__global__ void k_value_at(const float* __restrict__ V, Grid G, double M, double x0, double x1,
                           double x2, double x3, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double x[4] = {x0, x1, x2, x3};
  int base[4];
  double t[4];
  for (int k = 0; k < 4; k++) {
    const double s = to_grid(G, k, x[k]);
    if (!(s >= 0.0 && s <= (double)(G.n[k] - 1))) {
      *out = M;
      return;
    }
    int b = (int)floor(s);
    if (b > G.n[k] - 2) b = G.n[k] - 2;
    base[k] = b;
    t[k] = s - (double)b;
  }
  const float* p = V + (base[0] + base[1] * G.st[1] + base[2] * G.st[2] + base[3] * G.st[3]);
  double acc3[2];
  for (int e3 = 0; e3 < 2; e3++) {
    double acc2[2];
    for (int e2 = 0; e2 < 2; e2++) {
      double acc1[2];
      for (int e1 = 0; e1 < 2; e1++) {
        const float* q = p + e1 * G.st[1] + e2 * G.st[2] + e3 * G.st[3];
        acc1[e1] = (double)q[0] + t[0] * ((double)q[1] - (double)q[0]);
      }
      acc2[e2] = acc1[0] + t[1] * (acc1[1] - acc1[0]);
    }
    acc3[e3] = acc2[0] + t[2] * (acc2[1] - acc2[0]);
  }
  *out = acc3[0] + t[3] * (acc3[1] - acc3[0]);
}

// Feedback eq:feed at arbitrary states: the state is split into a grid node
// and an in-cell offset, so the sweep's search runs unchanged on it.
__global__ __launch_bounds__(kBlock) void k_feedback(SweepArgs a, const double* __restrict__ states,
                                                     int n, double tau, float* __restrict__ ang_out,
                                                     uint8_t* __restrict__ thr_out,
                                                     float* __restrict__ q_out) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  double y[4];
  NodeTerms T;
  float frac[4];
  for (int k = 0; k < 4; k++) {
    y[k] = states[4 * c + k];
    const double s = (y[k] - a.G.lo[k]) * a.G.inv_h[k];
    double fl = floor(s);
    if (!(fl >= 0.0)) fl = 0.0;  // outside (or NaN) states keep a valid node; the bounds test decides
    if (fl > (double)(a.G.n[k] - 1)) fl = (double)(a.G.n[k] - 1);
    T.i[k] = (int)fl;
    frac[k] = (float)(s - fl);
  }
  state_terms(a.G, a.P, y, tau, T.drift, T.g1, T.g2, T.gm);
  for (int k = 0; k < 4; k++) T.drift[k] += frac[k];
  SweepArgs b = a;
  b.P.q_coast = (float)(tau * (double)a.w_time);
  b.P.q_thr = (float)(tau * ((double)a.w_time + (double)a.w_fuel));
  b.P.gamma = (float)exp(-a.lambda * tau);
  auto qf = [&](float sn, float cs) { return q_thrust<true>(b.V_in, b.G, b.P, T, sn, cs); };
  const float qc = q_coast<true>(b.V_in, b.G, b.P, T);
  Choice ch;
  if (a.mode == 0) table_search(qf, b, qc, ch);
  else full_search(qf, b, qc, ch);
  ang_out[c] = ch.ang;
  thr_out[c] = (uint8_t)ch.thr;
  if (q_out) q_out[c] = ch.v;
}

// Reachability seed: FP64 Q1 value of the coarse V at every fine node.
__global__ __launch_bounds__(kBlock) void k_mask_seed(const float* __restrict__ Vc, Grid Gc, double M,
                                                      Grid Gf, double thresh, uint8_t* __restrict__ seed,
                                                      int Nf) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= Nf) return;
  int i[4];
  decode_node(Gf, j, i);
  int base[4];
  double t[4];
  bool inside = true;
  for (int k = 0; k < 4; k++) {
    const double x = Gf.lo[k] + (double)i[k] * Gf.h[k];
    const double s = to_grid(Gc, k, x);
    if (!(s >= 0.0 && s <= (double)(Gc.n[k] - 1))) inside = false;
    int b = (int)floor(s);
    if (b > Gc.n[k] - 2) b = Gc.n[k] - 2;
    if (b < 0) b = 0;
    base[k] = b;
    t[k] = s - (double)b;
  }
  double val = M;
  if (inside) {
    const float* p = Vc + (base[0] + base[1] * Gc.st[1] + base[2] * Gc.st[2] + base[3] * Gc.st[3]);
    double acc3[2];
    for (int e3 = 0; e3 < 2; e3++) {
      double acc2[2];
      for (int e2 = 0; e2 < 2; e2++) {
        double acc1[2];
        for (int e1 = 0; e1 < 2; e1++) {
          const float* q = p + e1 * Gc.st[1] + e2 * Gc.st[2] + e3 * Gc.st[3];
          acc1[e1] = (double)q[0] + t[0] * ((double)q[1] - (double)q[0]);
        }
        acc2[e2] = acc1[0] + t[1] * (acc1[1] - acc1[0]);
      }
      acc3[e3] = acc2[0] + t[2] * (acc2[1] - acc2[0]);
    }
    val = acc3[0] + t[3] * (acc3[1] - acc3[0]);
  }
  seed[j] = val < thresh ? 1 : 0;
}

// Box dilation is separable: one pass per axis of a 1-D max over +-d cells.
__global__ __launch_bounds__(kBlock) void k_dilate_axis(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                        Grid G, int axis, int d, int N) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= N) return;
  int i[4];
  decode_node(G, j, i);
  const int lo = max(0, i[axis] - d), hi = min(G.n[axis] - 1, i[axis] + d);
  uint8_t v = 0;
  for (int q = lo; q <= hi; q++) v |= in[j + (q - i[axis]) * G.st[axis]];
  out[j] = v;
}

// ---------------------------------------------------------------- probes
__global__ __launch_bounds__(kBlock) void k_probe_interp(const float* __restrict__ V, Grid G, float M,
                                                         const float* __restrict__ s, int n,
                                                         float* __restrict__ out) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  int i[4];
  float off[4];
  for (int k = 0; k < 4; k++) {
    const float sk = s[4 * c + k];
    float fl = floorf(sk);
    fl = fminf(fmaxf(fl, 0.0f), (float)(G.n[k] - 1));
    i[k] = (int)fl;
    off[k] = sk - fl;
  }
  out[c] = interp_off(V, G, i, off, M);
}

__global__ __launch_bounds__(kBlock) void k_probe_q(SweepArgs a, const int* __restrict__ nodes,
                                                    const uint8_t* __restrict__ thr,
                                                    const float* __restrict__ ang, int n,
                                                    float* __restrict__ q_out, float* __restrict__ off_out) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  NodeTerms T;
  node_terms(a.G, a.P, nodes[c], a.P.dt, T);
  float sn = 0.0f, cs = 0.0f;
  if (thr[c]) sincosf(ang[c], &sn, &cs);
  if (q_out) q_out[c] = thr[c] ? q_thrust(a.V_in, a.G, a.P, T, sn, cs) : q_coast(a.V_in, a.G, a.P, T);
  if (off_out) {
    off_out[4 * c + 0] = T.drift[0];
    off_out[4 * c + 1] = thr[c] ? fmaf(T.g1, sn, T.drift[1]) : T.drift[1];
    off_out[4 * c + 2] = thr[c] ? fmaf(T.g2, cs, T.drift[2]) : T.drift[2];
    off_out[4 * c + 3] = T.drift[3] + (thr[c] ? T.gm : 0.0f);
  }
}

}  // namespace dpo

// ------------------------------------------------------------ launchers
namespace dpo {

#define DPO_LAUNCH(kernel, grid, block, stream, ...)                        \
  do {                                                                      \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, stream, __VA_ARGS__); \
    return hipGetLastError();                                               \
  } while (0)

hipError_t launch_classify(const Grid& G, const TargetBox& tb, const uint8_t* mask, uint8_t* kind, int N,
                           hipStream_t s) {
  DPO_LAUNCH(k_classify, blocks_for(N), kBlock, s, G, tb, mask, kind, N);
}

int compact_chunks(int N) { return blocks_for(N, kChunk); }

hipError_t launch_compact(const Grid& G, const uint8_t* kind, int N, int* counts, int* offsets,
                          uint32_t* free_node, hipStream_t s) {
  const int nch = compact_chunks(N);
  hipLaunchKernelGGL(k_count_free, dim3(nch), dim3(kBlock), 0, s, kind, N, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, counts, nch, offsets);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter_free, dim3(nch), dim3(kBlock), 0, s, G, kind, N, offsets, free_node);
  return hipGetLastError();
}

hipError_t launch_init_value(const uint8_t* kind, float M, float* V, int N, hipStream_t s) {
  DPO_LAUNCH(k_init_value, blocks_for(N), kBlock, s, kind, M, V, N);
}

hipError_t launch_sweep_table(const SweepArgs& a, hipStream_t s) {
  DPO_LAUNCH(k_sweep_direct<0>, blocks_for(a.n_free), kBlock, s, a);
}

hipError_t launch_sweep_scan_golden(const SweepArgs& a, hipStream_t s) {
  DPO_LAUNCH(k_sweep_direct<1>, blocks_for(a.n_free), kBlock, s, a);
}

hipError_t launch_sweep_seeded(const SweepArgs& a, hipStream_t s) {
  DPO_LAUNCH(k_sweep_direct<2>, blocks_for(a.n_free), kBlock, s, a);
}

hipError_t launch_sweep_fast(const SweepArgs& a, int mode, hipStream_t s) {
  if (mode == 0) DPO_LAUNCH(k_sweep_fast<0>, blocks_for(a.n_free), kBlock, s, a);
  if (mode == 1) DPO_LAUNCH(k_sweep_fast<1>, blocks_for(a.n_free), kBlock, s, a);
  DPO_LAUNCH(k_sweep_fast<2>, blocks_for(a.n_free), kBlock, s, a);
}

hipError_t launch_policy_eval(const SweepArgs& a, bool want_resid, hipStream_t s) {
  if (want_resid) DPO_LAUNCH(k_policy_eval<true>, blocks_for(a.n_free), kBlock, s, a);
  DPO_LAUNCH(k_policy_eval<false>, blocks_for(a.n_free), kBlock, s, a);
}

hipError_t launch_policy_eval_desc(const SweepArgs& a, hipStream_t s) {
  DPO_LAUNCH(k_policy_eval_desc, blocks_for(a.n_free, kDescNpt * kBlock), kBlock, s, a);
}

hipError_t launch_resid_final(const double* partial, int nblocks, double* out, hipStream_t s) {
  DPO_LAUNCH(k_resid_final, 1, kBlock, s, partial, nblocks, out);
}

hipError_t launch_value_at(const float* V, const Grid& G, double M, const double x[4], double* out,
                           hipStream_t s) {
  DPO_LAUNCH(k_value_at, 1, 64, s, V, G, M, x[0], x[1], x[2], x[3], out);
}

hipError_t launch_feedback(const SweepArgs& a, const double* states, int n, double tau, float* ang,
                           uint8_t* thr, float* q, hipStream_t s) {
  DPO_LAUNCH(k_feedback, blocks_for(n), kBlock, s, a, states, n, tau, ang, thr, q);
}

hipError_t launch_mask_seed(const float* Vc, const Grid& Gc, double M, const Grid& Gf, double thresh,
                            uint8_t* seed, int Nf, hipStream_t s) {
  DPO_LAUNCH(k_mask_seed, blocks_for(Nf), kBlock, s, Vc, Gc, M, Gf, thresh, seed, Nf);
}

hipError_t launch_dilate_axis(const uint8_t* in, uint8_t* out, const Grid& G, int axis, int d, int N,
                              hipStream_t s) {
  DPO_LAUNCH(k_dilate_axis, blocks_for(N), kBlock, s, in, out, G, axis, d, N);
}

hipError_t launch_probe_interp(const float* V, const Grid& G, float M, const float* pts, int n,
                               float* out, hipStream_t s) {
  DPO_LAUNCH(k_probe_interp, blocks_for(n), kBlock, s, V, G, M, pts, n, out);
}

hipError_t launch_probe_q(const SweepArgs& a, const int* nodes, const uint8_t* thr, const float* ang,
                          int n, float* q_out, float* off_out, hipStream_t s) {
  DPO_LAUNCH(k_probe_q, blocks_for(n), kBlock, s, a, nodes, thr, ang, n, q_out, off_out);
}

}  // namespace dpo
