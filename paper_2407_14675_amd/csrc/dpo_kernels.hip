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

__global__ __launch_bounds__(kBlock) void k_scatter_free(const uint8_t* __restrict__ kind, int N,
                                                         const int* __restrict__ offsets,
                                                         int* __restrict__ free_idx) {
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
    if (f) free_idx[running + wave_off + below] = j;
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
// Tabulated search: coast, then n_ang thrust angles; first strict minimum.
__global__ __launch_bounds__(kBlock) void k_sweep_table(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  if (t < a.n_free) {
    const int j = a.free_idx[t];
    NodeTerms T;
    node_terms(a.G, a.P, j, a.P.dt, T);
    const float qc = q_coast(a.V_in, a.G, a.P, T);
    float bq = INFINITY;
    int bk = 0;
    for (int k = 0; k < a.n_ang; k++) {
      const float q = q_thrust(a.V_in, a.G, a.P, T, a.tab_sin[k], a.tab_cos[k]);
      if (q < bq) {
        bq = q;
        bk = k;
      }
    }
    const bool thr = bq < qc;
    const float v = thr ? bq : qc;
    a.V_out[j] = v;
    if (a.pol_ang) a.pol_ang[j] = a.tab_ang[bk];
    if (a.pol_thr) a.pol_thr[j] = thr ? 1 : 0;
    node_residual(a.V_in[j], v, rel, sum, mabs, bad);
  }
  block_residual(rel, sum, mabs, bad, 0.0, a.partial, blockIdx.x);
}

// Golden-section refinement in offsets d from the centre angle u0 whose
// sin/cos are (s0, c0): angles u0 + d use a rotation by d.
struct GoldenState {
  float best_q, best_d;
};

template <bool kSnap>
__device__ inline float q_at_offset(const SweepArgs& a, const NodeTerms& T, float s0, float c0,
                                    float d) {
  float sd, cd;
  small_sincos(d, sd, cd);
  const float sn = fmaf(s0, cd, c0 * sd);
  const float cs = fmaf(c0, cd, -s0 * sd);
  return q_thrust<kSnap>(a.V_in, a.G, a.P, T, sn, cs);
}

template <bool kSnap = false>
__device__ inline void golden(const SweepArgs& a, const NodeTerms& T, float s0, float c0,
                              float half, int steps, GoldenState& g) {
  const float rho = 0.6180339887498949f;
  float lo = -half, hi = half;
  float x1 = hi - rho * (hi - lo), x2 = lo + rho * (hi - lo);
  float f1 = q_at_offset<kSnap>(a, T, s0, c0, x1);
  if (f1 < g.best_q) {
    g.best_q = f1;
    g.best_d = x1;
  }
  float f2 = q_at_offset<kSnap>(a, T, s0, c0, x2);
  if (f2 < g.best_q) {
    g.best_q = f2;
    g.best_d = x2;
  }
  for (int it = 0; it < steps; it++) {
    if (f1 < f2) {
      hi = x2;
      x2 = x1;
      f2 = f1;
      x1 = hi - rho * (hi - lo);
      f1 = q_at_offset<kSnap>(a, T, s0, c0, x1);
      if (f1 < g.best_q) {
        g.best_q = f1;
        g.best_d = x1;
      }
    } else {
      lo = x1;
      x1 = x2;
      f1 = f2;
      x2 = lo + rho * (hi - lo);
      f2 = q_at_offset<kSnap>(a, T, s0, c0, x2);
      if (f2 < g.best_q) {
        g.best_q = f2;
        g.best_d = x2;
      }
    }
  }
}

// Full search of one node: scan of n_ang tabulated angles, golden section
// around the best sample, coast comparison.
template <bool kSnap = false>
__device__ inline void full_search(const SweepArgs& a, const NodeTerms& T, float& v, float& ang,
                                   int& thr) {
  const float qc = q_coast<kSnap>(a.V_in, a.G, a.P, T);
  float bq = INFINITY;
  int bk = 0;
  for (int k = 0; k < a.n_ang; k++) {
    const float q = q_thrust<kSnap>(a.V_in, a.G, a.P, T, a.tab_sin[k], a.tab_cos[k]);
    if (q < bq) {
      bq = q;
      bk = k;
    }
  }
  GoldenState g{bq, 0.0f};
  if (a.n_golden > 0) golden<kSnap>(a, T, a.tab_sin[bk], a.tab_cos[bk], a.half_width, a.n_golden, g);
  thr = g.best_q < qc ? 1 : 0;
  v = thr ? g.best_q : qc;
  ang = wrap_pi(a.tab_ang[bk] + g.best_d);
}

__global__ __launch_bounds__(kBlock) void k_sweep_scan_golden(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  if (t < a.n_free) {
    const int j = a.free_idx[t];
    NodeTerms T;
    node_terms(a.G, a.P, j, a.P.dt, T);
    float v, ang;
    int thr;
    full_search(a, T, v, ang, thr);
    a.V_out[j] = v;
    if (a.pol_ang) a.pol_ang[j] = ang;
    if (a.pol_thr) a.pol_thr[j] = (uint8_t)thr;
    node_residual(a.V_in[j], v, rel, sum, mabs, bad);
  }
  block_residual(rel, sum, mabs, bad, 0.0, a.partial, blockIdx.x);
}

// Seeded local search: the seed angle itself, then golden section with
// n_local - 1 further evaluations on [seed - w, seed + w], then coast.  A node
// whose result differs from its current value by more than
// fallback_tol*max(1, |V|) repeats the full search.
__global__ __launch_bounds__(kBlock) void k_sweep_seeded(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  int fell_back = 0;
  if (t < a.n_free) {
    const int j = a.free_idx[t];
    NodeTerms T;
    node_terms(a.G, a.P, j, a.P.dt, T);
    const float seed = a.seed[j];
    float s0, c0;
    sincosf(seed, &s0, &c0);
    GoldenState g{q_thrust(a.V_in, a.G, a.P, T, s0, c0), 0.0f};
    golden(a, T, s0, c0, a.local_half_width, a.n_local - 3, g);
    const float qc = q_coast(a.V_in, a.G, a.P, T);
    int thr = g.best_q < qc ? 1 : 0;
    float v = thr ? g.best_q : qc;
    float ang = wrap_pi(seed + g.best_d);
    const float vin = a.V_in[j];
    if (fabsf(v - vin) > a.fallback_tol * fmaxf(1.0f, fabsf(vin))) {
      full_search(a, T, v, ang, thr);
      fell_back = 1;
    }
    a.V_out[j] = v;
    if (a.pol_ang) a.pol_ang[j] = ang;
    if (a.pol_thr) a.pol_thr[j] = (uint8_t)thr;
    node_residual(vin, v, rel, sum, mabs, bad);
  }
  block_residual(rel, sum, mabs, bad, (double)fell_back, a.partial, blockIdx.x);
}

// Frozen-policy sweep (eq:p_eval applied once).
__global__ __launch_bounds__(kBlock) void k_policy_eval(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  if (t < a.n_free) {
    const int j = a.free_idx[t];
    NodeTerms T;
    node_terms(a.G, a.P, j, a.P.dt, T);
    float v;
    if (a.pol_thr_in[j]) {
      float sn, cs;
      sincosf(a.pol_ang_in[j], &sn, &cs);
      v = q_thrust(a.V_in, a.G, a.P, T, sn, cs);
    } else {
      v = q_coast(a.V_in, a.G, a.P, T);
    }
    a.V_out[j] = v;
    node_residual(a.V_in[j], v, rel, sum, mabs, bad);
  }
  block_residual(rel, sum, mabs, bad, 0.0, a.partial, blockIdx.x);
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
  float v, ang;
  int thr;
  if (a.mode == 0) {
    const float qc = q_coast<true>(b.V_in, b.G, b.P, T);
    float bq = INFINITY;
    int bk = 0;
    for (int k = 0; k < b.n_ang; k++) {
      const float q = q_thrust<true>(b.V_in, b.G, b.P, T, b.tab_sin[k], b.tab_cos[k]);
      if (q < bq) {
        bq = q;
        bk = k;
      }
    }
    thr = bq < qc ? 1 : 0;
    v = thr ? bq : qc;
    ang = b.tab_ang[bk];
  } else {
    full_search<true>(b, T, v, ang, thr);
  }
  ang_out[c] = ang;
  thr_out[c] = (uint8_t)thr;
  if (q_out) q_out[c] = v;
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

hipError_t launch_compact(const uint8_t* kind, int N, int* counts, int* offsets, int* free_idx,
                          hipStream_t s) {
  const int nch = compact_chunks(N);
  hipLaunchKernelGGL(k_count_free, dim3(nch), dim3(kBlock), 0, s, kind, N, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, counts, nch, offsets);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter_free, dim3(nch), dim3(kBlock), 0, s, kind, N, offsets, free_idx);
  return hipGetLastError();
}

hipError_t launch_init_value(const uint8_t* kind, float M, float* V, int N, hipStream_t s) {
  DPO_LAUNCH(k_init_value, blocks_for(N), kBlock, s, kind, M, V, N);
}

hipError_t launch_sweep_table(const SweepArgs& a, hipStream_t s) {
  DPO_LAUNCH(k_sweep_table, blocks_for(a.n_free), kBlock, s, a);
}

hipError_t launch_sweep_scan_golden(const SweepArgs& a, hipStream_t s) {
  DPO_LAUNCH(k_sweep_scan_golden, blocks_for(a.n_free), kBlock, s, a);
}

hipError_t launch_sweep_seeded(const SweepArgs& a, hipStream_t s) {
  DPO_LAUNCH(k_sweep_seeded, blocks_for(a.n_free), kBlock, s, a);
}

hipError_t launch_policy_eval(const SweepArgs& a, hipStream_t s) {
  DPO_LAUNCH(k_policy_eval, blocks_for(a.n_free), kBlock, s, a);
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
