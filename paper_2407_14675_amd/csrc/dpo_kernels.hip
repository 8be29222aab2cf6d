// HIP kernels of libdpo for gfx950: classification and compaction of the
// reduced grid, Bellman sweeps (tabulated search, scan + golden section,
// seeded local search), frozen-policy sweeps, FP64 residual reduction,
// FP64 read-out, feedback, reachability mask and probes.
//
// Paper: arXiv 2407.14675, Section 3 (eq:schema, value and policy iteration,
// minimisation by tabulation and golden section, feedback eq:feed).
#include <algorithm>

#include "dpo_search.h"

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
// Heun terms of a free node from its packed coordinates (grid coordinates
// formed as lo + i*h, the product rounded before the sum).
__device__ inline void node_heun(const SweepArgs& a, const int i[4], HeunTerms& H) {
#pragma clang fp contract(off)
  double x[4];
  for (int k = 0; k < 4; k++) x[k] = a.G.lo[k] + (double)i[k] * a.G.h[k];
  heun_terms(a.G, a.P, x, a.P.dt, H);
}

// ---- direct path: every evaluation forms its foot and cell; the 16 corners
// come from V when the cell differs from the previous evaluation's (a
// per-node corner cache).  Used for any problem and for the Heun foot; the
// fast path below covers the orbit workloads with the Euler foot.
template <int kMode, bool kHeun>
__global__ __launch_bounds__(kBlock) void k_sweep_direct(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  int fell_back = 0, evals = 0;
  if (t < a.n_free) {
    NodeTerms T;
    const int j = node_terms_tab(a, a.free_node[t], T);
    HeunTerms H;
    if (kHeun) node_heun(a, T.i, H);
    const float* __restrict__ V = a.V_in;
    const float qx = a.qnode ? a.qnode[j] : 0.0f;
    CornerCache cc;
    cc.key = -1;
    auto qf = [&](float sn, float cs) { return q_step_cached<kHeun>(V, a.G, a.P, T, H, 1, sn, cs, qx, cc); };
    const float qc = q_step_cached<kHeun>(V, a.G, a.P, T, H, 0, 0.0f, 1.0f, qx, cc);
    const float vin = V[j];
    Choice ch;
    if (kMode == 0) table_search(qf, a, qc, ch);
    else if (kMode == 1) full_search(qf, a, qc, ch);
    else if (kMode == 3) evals = walk_search(qf, a, a.walk_from[j], qc, ch);
    else fell_back = seeded_search(qf, a, a.seed[j], qc, vin, ch);
    keep_incumbent(qf, a, j, qc, ch);
    a.V_out[j] = ch.v;
    if (a.pol_ang) a.pol_ang[j] = ch.ang;
    if (a.pol_thr) a.pol_thr[j] = (uint8_t)ch.thr;
    if (!kHeun && (a.desc_code || a.desc16 || a.desc_pk)) write_desc(a, t, j, T, ch);
    node_residual(vin, ch.v, rel, sum, mabs, bad);
  }
  if (kMode == 3 && a.eval_acc) block_add_count(evals, a.eval_acc);
  // the fifth residual entry: seeded fallbacks, or the walk's thrust evaluations
  if (a.partial) block_residual(rel, sum, mabs, bad, (double)(kMode == 3 ? evals : fell_back), a.partial, blockIdx.x);
}

// Factorised-path sweep; the workgroup size is chosen at launch (64..512)
// and the region pairs live in dynamic LDS (4 * blockDim.x float4).
template <int kMode>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_sweep_fast(SweepArgs a) {
  extern __shared__ float4 dyn_lds[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * blockDim.x + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  int fell_back = 0, deferred = 0, evals = 0;
  if (t < a.n_free) fast_node<kMode>(a, t, dyn_lds, rel, sum, mabs, bad, fell_back, deferred, evals);
  if (kMode == 3 && a.eval_acc) block_add_count(evals, a.eval_acc);
  if (kMode == 2 && a.fb_list) {
    // append the wave's deferred nodes with one atomic per wave
    const unsigned long long bal = __ballot(deferred);
    if (bal) {
      const int lane = threadIdx.x & 63;
      int base = 0;
      if (lane == 0) base = atomicAdd(a.fb_count, __popcll(bal));
      base = __shfl(base, 0, 64);
      if (deferred) a.fb_list[base + __popcll(bal & ((1ull << lane) - 1ull))] = t;
    }
  }
  // a null partial buffer (value-iteration sweeps between checks) skips the residual;
  // the fifth entry: seeded fallbacks, or the walk's thrust evaluations
  if (a.partial) block_residual(rel, sum, mabs, bad, (double)(kMode == 3 ? evals : fell_back), a.partial, blockIdx.x);
}

// Second pass of the seeded sweep: the full search at the nodes the first
// pass listed, so that a wave's full searches run together instead of
// stalling the lanes whose local search sufficed.  Persistent grid over the
// list; the residual partials of this pass follow those of the first.
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_sweep_fallback(SweepArgs a) {
  extern __shared__ float4 dyn_lds[];
  const int count = *a.fb_count;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  int unused = 0, unused2 = 0, unused3 = 0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x)
    fast_node<1>(a, a.fb_list[k], dyn_lds, rel, sum, mabs, bad, unused, unused2, unused3);
  block_residual(rel, sum, mabs, bad, 0.0, a.partial, blockIdx.x);
}

__global__ void k_zero_count(int* count) { *count = 0; }

// Frozen-policy sweep (eq:p_eval applied once).  The residual reduction is
// only compiled in when a caller asks for it; the policy-iteration loop does
// not, since it stops on the residual of the greedy step.
template <bool kResid, bool kHeun>
__global__ __launch_bounds__(kBlock) void k_policy_eval(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  if (t < a.n_free) {
    NodeTerms T;
    const int j = node_terms_tab(a, a.free_node[t], T);
    HeunTerms H;
    if (kHeun) node_heun(a, T.i, H);
    const int thr = a.pol_thr_in[j] ? 1 : 0;
    float sn = 0.0f, cs = 1.0f;
    if (thr) policy_sincos(a, a.pol_ang_in[j], sn, cs);
    const float v = q_step<kHeun>(a.V_in, a.G, a.P, T, H, thr, sn, cs, a.qnode ? a.qnode[j] : 0.0f);
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

// kNt: bit 0 = non-temporal loads of the per-node stream (coordinates and
// descriptor), bit 1 = non-temporal store of the value.  Used when a sweep's
// data is larger than the last-level cache: the streamed bytes then no
// longer evict the value rows that neighbouring nodes' gathers reuse.  When
// everything fits, the temporal form lets the descriptors (reused by the 20
// sweeps of a policy) and the values stay cached.
template <int kNt>
__global__ __launch_bounds__(kBlock) void k_policy_eval_desc(SweepArgs a) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t0 = tile * (kDescNpt * kBlock) + threadIdx.x;
  uint32_t packed[kDescNpt];
  int code[kDescNpt];
  float2 w[kDescNpt];
  typedef float nt_f2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int k = 0; k < kDescNpt; k++) {
    const int t = t0 + k * kBlock;
    if (t < a.n_free) {
      // streamed once per sweep: non-temporal, so they do not evict the value rows the gathers reuse
      if (kNt & 1) {
        packed[k] = __builtin_nontemporal_load(a.free_node + t);
        code[k] = __builtin_nontemporal_load(a.desc_code_in + t);
        const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(a.desc_w_in) + t);
        w[k] = make_float2(v.x, v.y);
      } else {
        packed[k] = a.free_node[t];
        code[k] = a.desc_code_in[t];
        w[k] = a.desc_w_in[t];
      }
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
      I = cell_value(a.V_in + (code[k] & 0x3fffffff), a.G, tt, a.G.st[3]);
    }
    const float out = fmaf(a.P.gamma, I, thr ? a.P.q_thr : a.P.q_coast);
    if (kNt & 2) __builtin_nontemporal_store(out, a.V_out + j);
    else a.V_out[j] = out;
  }
}

// The same sweep from compact descriptors: 14 bytes per free node with the
// free list (SweepArgs::desc16: coordinates 4, code 2, weights 8), 8 bytes
// per node without it (kDense, SweepArgs::desc_pk: every node is visited in
// order, fixed ones carry kDescPkSkip and are left alone, and the node index
// is the thread's).
// kNpt nodes per thread: 2 when the data streams from HBM (more loads in
// flight per wave), 1 when it is cache-resident (twice the workgroups, a
// smaller last partial round on the CUs).
template <bool kDense, int kNt, int kNpt>
__global__ __launch_bounds__(kBlock) void k_policy_eval_d16(SweepArgs a) {
  typedef float nt_f2 __attribute__((ext_vector_type(2)));
  typedef unsigned nt_u2 __attribute__((ext_vector_type(2)));
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t0 = tile * (kNpt * kBlock) + threadIdx.x;
  const int count = kDense ? a.G.n[0] * a.G.n[1] * a.G.n[2] * a.G.n[3] : a.n_free;
  uint32_t packed[kNpt];
  uint32_t code[kNpt];
  float2 w[kNpt];
#pragma unroll
  for (int k = 0; k < kNpt; k++) {
    const int t = t0 + k * kBlock;
    if (t < count) {
      if (kDense) {
        const nt_u2 v = (kNt & 1) ? __builtin_nontemporal_load(reinterpret_cast<const nt_u2*>(a.desc_pk_in) + t)
                                  : reinterpret_cast<const nt_u2*>(a.desc_pk_in)[t];
        const uint2 d = make_uint2(v.x, v.y);
        code[k] = desc_pk_code(d);
        w[k] = make_float2(desc_pk_w1(d), desc_pk_w2(d));
      } else if (kNt & 1) {
        packed[k] = __builtin_nontemporal_load(a.free_node + t);
        code[k] = __builtin_nontemporal_load(a.desc16_in + t);
        const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(a.desc_w_in) + t);
        w[k] = make_float2(v.x, v.y);
      } else {
        packed[k] = a.free_node[t];
        code[k] = a.desc16_in[t];
        w[k] = a.desc_w_in[t];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kNpt; k++) {
    const int t = t0 + k * kBlock;
    if (t >= count) continue;
    if (kDense && code[k] == kDescPkSkip) continue;
    int i[4];
    int j;
    if (kDense) {
      j = t;
      decode_node(a.G, t, i);
    } else {
      j = unpack_node(a.G, packed[k], i);
    }
    const bool thr = (code[k] & kDescThr) != 0;
    float I = a.P.M;
    if (!(code[k] & kDescOut)) {
      // r and m cell coordinates, exactly as the greedy sweep formed them
      const float o0 = drift_r(a, i[1]);
      int b0, b3;
      float tt[4];
      axis_cell(i[0], a.G.n[0], o0, b0, tt[0]);
      axis_cell(i[3], a.G.n[3], thr ? a.gm : 0.0f, b3, tt[3]);
      tt[1] = w[k].x;
      tt[2] = w[k].y;
      const int dv = (int)(code[k] & 63u) - 32, dt = (int)((code[k] >> 6) & 63u) - 32;
      I = cell_value(a.V_in + b0 + (i[1] + dv) * a.G.st[1] + (i[2] + dt) * a.G.st[2] + b3 * a.G.st[3], a.G, tt, a.G.st[3]);
    }
    const float out = fmaf(a.P.gamma, I, thr ? a.P.q_thr : a.P.q_coast);
    if (kNt & 2) __builtin_nontemporal_store(out, a.V_out + j);
    else a.V_out[j] = out;
  }
}

// FP64 reduction of workgroup partials in a fixed order: workgroup b folds
// the partials b*kBlock + t + k*gridDim.x*kBlock and writes its result to
// out[kPartial*b ...]; one workgroup gives the final value, several give the
// first stage of a two-stage reduction.
__global__ __launch_bounds__(kBlock) void k_resid_final(const double* __restrict__ partial, int nblocks,
                                                        double* __restrict__ out) {
  __shared__ double red[kPartial][kBlock];
  double acc[kPartial] = {0, 0, 0, 0, 0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < nblocks; i += gridDim.x * kBlock) {
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
    for (int q = 0; q < kPartial; q++) out[kPartial * blockIdx.x + q] = red[q][0];
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
    if (k == 3 && G.periodic3) {
      // periodic axis: wrap into [0, n)
      const double n = (double)G.n[3];
      double w = (x[3] - G.lo[3]) * G.inv_h[3];
      if (!(fabs(w) <= 1e30)) {
        *out = M;
        return;
      }
      w -= n * floor(w / n);
      int b = (int)floor(w);
      if (b >= G.n[3]) b = 0, w = 0.0;
      base[3] = b;
      t[3] = w - (double)b;
      continue;
    }
    double s = to_grid(G, k, x[k]);
    if ((k == 1 || k == 2) && G.clamp12 && fabs(s) <= 1e30) s = fmin(fmax(s, 0.0), (double)(G.n[k] - 1));
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
  const int s3 = (G.periodic3 && base[3] == G.n[3] - 1) ? -base[3] * G.st[3] : G.st[3];
  double acc3[2];
  for (int e3 = 0; e3 < 2; e3++) {
    double acc2[2];
    for (int e2 = 0; e2 < 2; e2++) {
      double acc1[2];
      for (int e1 = 0; e1 < 2; e1++) {
        const float* q = p + e1 * G.st[1] + e2 * G.st[2] + e3 * s3;
        acc1[e1] = (double)q[0] + t[0] * ((double)q[1] - (double)q[0]);
      }
      acc2[e2] = acc1[0] + t[1] * (acc1[1] - acc1[0]);
    }
    acc3[e3] = acc2[0] + t[2] * (acc2[1] - acc2[0]);
  }
  *out = acc3[0] + t[3] * (acc3[1] - acc3[0]);
}

// Feedback eq:feed at an arbitrary state y: the state is split into a grid
// node and an in-cell offset, so the sweep's search runs unchanged on it.
// kWave: the lanes of a wave share the state and split the table (every
// lane computes the same set-up and ends with the same choice).
template <bool kWave>
__device__ inline void feedback_at(const SweepArgs& a, const double y_in[4], double tau, Choice& ch) {
  double y[4];
  NodeTerms T;
  float frac[4];
  for (int k = 0; k < 4; k++) {
    y[k] = y_in[k];
    double s = (y[k] - a.G.lo[k]) * a.G.inv_h[k];
    // periodic axis: wrap the state into [0, n) first
    if (k == 3 && a.G.periodic3 && fabs(s) <= 1e30) s -= (double)a.G.n[3] * floor(s / (double)a.G.n[3]);
    double fl = floor(s);
    if (!(fl >= 0.0)) fl = 0.0;  // outside (or NaN) states keep a valid node; the bounds test decides
    if (fl > (double)(a.G.n[k] - 1)) fl = (double)(a.G.n[k] - 1);
    T.i[k] = (int)fl;
    frac[k] = (float)(s - fl);
  }
  state_terms(a.G, a.P, y, tau, T.drift, T.g1, T.g2, T.gm);
  for (int k = 0; k < 4; k++) T.drift[k] += frac[k];
  HeunTerms H;
  heun_terms(a.G, a.P, y, tau, H);
  SweepArgs b = a;
  b.P.q_coast = (float)(tau * (double)a.w_time);
  b.P.q_thr = (float)(tau * ((double)a.w_time + (double)a.w_fuel));
  b.P.gamma = (float)exp(-a.lambda * tau);
  const bool heun = a.P.heun != 0;
  // crown: the orbital-element cost at the state itself (eq:feed evaluates l at y)
  const float qx = a.P.model == 2 ? (float)(tau * crown_cost(a.P, y)) : 0.0f;
  auto qf = [&](float sn, float cs) {
    return heun ? q_step<true, true>(b.V_in, b.G, b.P, T, H, 1, sn, cs, qx)
                : q_step<false, true>(b.V_in, b.G, b.P, T, H, 1, sn, cs, qx);
  };
  const float qc = heun ? q_step<true, true>(b.V_in, b.G, b.P, T, H, 0, 0.0f, 1.0f, qx)
                        : q_step<false, true>(b.V_in, b.G, b.P, T, H, 0, 0.0f, 1.0f, qx);
  // the walk's table (mode 3) is searched in full: a state has no previous optimum
  if (a.mode == 0 || a.mode == 3) table_search<kWave>(qf, b, qc, ch);
  else full_search<kWave>(qf, b, qc, ch);
}

// kWave: one wave per state (few states: the table is split over the lanes,
// and the chip holds 64 times as many independent waves); else one thread
// per state.
template <bool kWave>
__global__ __launch_bounds__(kBlock) void k_feedback(SweepArgs a, const double* __restrict__ states,
                                                     int n, double tau, float* __restrict__ ang_out,
                                                     uint8_t* __restrict__ thr_out,
                                                     float* __restrict__ q_out) {
  const int c = kWave ? (int)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) : (int)(blockIdx.x * kBlock + threadIdx.x);
  if (c >= n) return;  // wave-uniform in the wave mode
  double y[4];
  for (int k = 0; k < 4; k++) y[k] = states[4 * (size_t)c + k];
  Choice ch;
  feedback_at<kWave>(a, y, tau, ch);
  if (kWave && (threadIdx.x & 63) != 0) return;
  ang_out[c] = ch.ang;
  thr_out[c] = (uint8_t)ch.thr;
  if (q_out) q_out[c] = ch.v;
}

// ---- closed loop: the simulated system of Section 4 in FP64, the model's
// own dynamics plus (orbit models, drag != 0) Example 2's aerodynamic drag,
// an acceleration drag * |v|^2 against the velocity (v_r, v_t); integrated
// by the classical fourth-order Runge-Kutta method with the control held
// over each step.
__device__ inline void plant_rhs(const Phys& P, const double x[4], int thr, double sn, double cs, double drag,
                                 double b[4]) {
#pragma clang fp contract(off)
  if (P.model == 1) {
    const double s = thr ? P.speed : 0.0;
    b[0] = 0.0;
    b[1] = s * sn;
    b[2] = s * cs;
    b[3] = 0.0;
    return;
  }
  const double r = x[0], vr = x[1], vt = x[2];
  const double acc = thr ? (P.model == 2 ? P.accel : P.accel / x[3]) : 0.0;
  const double dv = drag * sqrt(vr * vr + vt * vt);
  b[0] = vr;
  b[1] = (vt * vt / r - P.mu / (r * r) + acc * sn) - dv * vr;
  b[2] = (-vr * vt / r + acc * cs) - dv * vt;
  b[3] = P.model == 2 ? vt / r : -P.mdot * (double)thr;
}

__device__ inline void rk4_step(const Phys& P, double x[4], int thr, double sn, double cs, double drag, double h) {
#pragma clang fp contract(off)
  double k1[4], k2[4], k3[4], k4[4], y[4];
  plant_rhs(P, x, thr, sn, cs, drag, k1);
  for (int k = 0; k < 4; k++) y[k] = x[k] + 0.5 * h * k1[k];
  plant_rhs(P, y, thr, sn, cs, drag, k2);
  for (int k = 0; k < 4; k++) y[k] = x[k] + 0.5 * h * k2[k];
  plant_rhs(P, y, thr, sn, cs, drag, k3);
  for (int k = 0; k < 4; k++) y[k] = x[k] + h * k3[k];
  plant_rhs(P, y, thr, sn, cs, drag, k4);
  for (int k = 0; k < 4; k++) x[k] += h / 6.0 * (k1[k] + 2.0 * k2[k] + 2.0 * k3[k] + k4[k]);
}

// One trajectory per thread (or, kWave, per wave: the lanes split the
// feedback's table and all integrate the same state): `steps` times the
// feedback at the current state (time step tau), then `substeps` RK4 steps of
// tau/substeps with that control.  Histories are step-major so that a step's
// writes are coalesced.
template <bool kWave>
__global__ __launch_bounds__(kBlock) void k_simulate(SweepArgs a, double* __restrict__ states, int n, double tau,
                                                     int steps, int substeps, double drag, double* __restrict__ traj,
                                                     uint8_t* __restrict__ thr_hist, float* __restrict__ ang_hist) {
  const int c = kWave ? (int)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) : (int)(blockIdx.x * kBlock + threadIdx.x);
  if (c >= n) return;  // wave-uniform in the wave mode
  const bool lead = !kWave || (threadIdx.x & 63) == 0;
  double y[4];
  for (int k = 0; k < 4; k++) y[k] = states[4 * (size_t)c + k];
  if (traj && lead)
    for (int k = 0; k < 4; k++) traj[4 * (size_t)c + k] = y[k];
  const double h = tau / (double)substeps;
  for (int s = 0; s < steps; s++) {
    Choice ch;
    feedback_at<kWave>(a, y, tau, ch);
    double sn, cs;
    sincos((double)ch.ang, &sn, &cs);
    for (int q = 0; q < substeps; q++) rk4_step(a.P, y, ch.thr, sn, cs, drag, h);
    if (!lead) continue;
    const size_t at = (size_t)s * (size_t)n + (size_t)c;
    if (thr_hist) thr_hist[at] = (uint8_t)ch.thr;
    if (ang_hist) ang_hist[at] = ch.ang;
    if (traj)
      for (int k = 0; k < 4; k++) traj[4 * (at + (size_t)n) + k] = y[k];
  }
  if (lead)
    for (int k = 0; k < 4; k++) states[4 * (size_t)c + k] = y[k];
}

// Reachability seed: FP64 Q1 value of the coarse V at every fine node.
__global__ __launch_bounds__(kBlock) void k_mask_seed(const float* __restrict__ Vc, Grid Gc, double M,
                                                      Grid Gf, double thresh, uint8_t* __restrict__ seed,
                                                      int Nf) {
#pragma clang fp contract(off)
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
    const float sk = s[4 * (size_t)c + k];
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
  HeunTerms H;
  node_heun(a, T.i, H);
  const int th = thr[c] ? 1 : 0;
  float sn = 0.0f, cs = 1.0f;
  if (th) sincosf(ang[c], &sn, &cs);
  const bool heun = a.P.heun != 0;
  const float qx = a.qnode ? a.qnode[nodes[c]] : 0.0f;
  if (q_out)
    q_out[c] = heun ? q_step<true>(a.V_in, a.G, a.P, T, H, th, sn, cs, qx)
                    : q_step<false>(a.V_in, a.G, a.P, T, H, th, sn, cs, qx);
  if (off_out) {
    float off[4];
    if (heun) foot_off<true>(T, H, th, sn, cs, off);
    else foot_off<false>(T, H, th, sn, cs, off);
    for (int k = 0; k < 4; k++) off_out[4 * (size_t)c + k] = off[k];
  }
}

// Crown problem: dt times the orbital-element running cost at every node, FP64
// then rounded (node coordinates lo + i*h with the product rounded first).
__global__ __launch_bounds__(kBlock) void k_node_cost(Grid G, Phys P, float* __restrict__ qnode, int N) {
#pragma clang fp contract(off)
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= N) return;
  int i[4];
  decode_node(G, j, i);
  double x[4];
  for (int k = 0; k < 4; k++) x[k] = G.lo[k] + (double)i[k] * G.h[k];
  qnode[j] = (float)(P.dt * crown_cost(P, x));
}

// Fixed-order sum of the per-workgroup evaluation counts of the table walk.
__global__ __launch_bounds__(kBlock) void k_sum_counts(const unsigned long long* __restrict__ acc, int n,
                                                       unsigned long long* __restrict__ out) {
  __shared__ unsigned long long part[kBlock];
  unsigned long long v = 0;
  for (int i = threadIdx.x; i < n; i += kBlock) v += acc[i];
  part[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
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

hipError_t launch_sweep_direct(const SweepArgs& a, int mode, hipStream_t s) {
  const int nb = blocks_for(a.n_free);
  if (a.P.heun) {
    if (mode == 0) DPO_LAUNCH((k_sweep_direct<0, true>), nb, kBlock, s, a);
    if (mode == 1) DPO_LAUNCH((k_sweep_direct<1, true>), nb, kBlock, s, a);
    if (mode == 2) DPO_LAUNCH((k_sweep_direct<2, true>), nb, kBlock, s, a);
    DPO_LAUNCH((k_sweep_direct<3, true>), nb, kBlock, s, a);
  }
  if (mode == 0) DPO_LAUNCH((k_sweep_direct<0, false>), nb, kBlock, s, a);
  if (mode == 1) DPO_LAUNCH((k_sweep_direct<1, false>), nb, kBlock, s, a);
  if (mode == 2) DPO_LAUNCH((k_sweep_direct<2, false>), nb, kBlock, s, a);
  DPO_LAUNCH((k_sweep_direct<3, false>), nb, kBlock, s, a);
}

hipError_t launch_node_cost(const Grid& G, const Phys& P, float* qnode, int N, hipStream_t s) {
  DPO_LAUNCH(k_node_cost, blocks_for(N), kBlock, s, G, P, qnode, N);
}

hipError_t launch_sum_counts(const unsigned long long* acc, int n, unsigned long long* out, hipStream_t s) {
  DPO_LAUNCH(k_sum_counts, 1, kBlock, s, acc, n, out);
}

hipError_t launch_sweep_fast(const SweepArgs& a, int mode, int block, hipStream_t s) {
  const int nb = blocks_for(a.n_free, block);
  const size_t lds = sizeof(float4) * 4 * block;
  if (mode == 0) hipLaunchKernelGGL(k_sweep_fast<0>, dim3(nb), dim3(block), lds, s, a);
  else if (mode == 1) hipLaunchKernelGGL(k_sweep_fast<1>, dim3(nb), dim3(block), lds, s, a);
  else if (mode == 2) hipLaunchKernelGGL(k_sweep_fast<2>, dim3(nb), dim3(block), lds, s, a);
  else hipLaunchKernelGGL(k_sweep_fast<3>, dim3(nb), dim3(block), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_zero_count(int* count, hipStream_t s) { DPO_LAUNCH(k_zero_count, 1, 1, s, count); }

hipError_t launch_sweep_fallback(const SweepArgs& a, int block, int blocks, hipStream_t s) {
  const size_t lds = 4 * (size_t)block * sizeof(float4);
  hipLaunchKernelGGL(k_sweep_fallback, dim3(blocks), dim3(block), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_policy_eval(const SweepArgs& a, bool want_resid, hipStream_t s) {
  const int nb = blocks_for(a.n_free);
  if (a.P.heun) {
    if (want_resid) DPO_LAUNCH((k_policy_eval<true, true>), nb, kBlock, s, a);
    DPO_LAUNCH((k_policy_eval<false, true>), nb, kBlock, s, a);
  }
  if (want_resid) DPO_LAUNCH((k_policy_eval<true, false>), nb, kBlock, s, a);
  DPO_LAUNCH((k_policy_eval<false, false>), nb, kBlock, s, a);
}

hipError_t launch_policy_eval_desc(const SweepArgs& a, bool streamed, hipStream_t s) {
  if (streamed) DPO_LAUNCH(k_policy_eval_desc<3>, blocks_for(a.n_free, kDescNpt * kBlock), kBlock, s, a);
  DPO_LAUNCH(k_policy_eval_desc<0>, blocks_for(a.n_free, kDescNpt * kBlock), kBlock, s, a);
}

hipError_t launch_policy_eval_desc16(const SweepArgs& a, int format, bool streamed, hipStream_t s) {
  if (format == 2) {
    const long long N = (long long)a.G.n[0] * a.G.n[1] * a.G.n[2] * a.G.n[3];
    if (streamed) DPO_LAUNCH((k_policy_eval_d16<true, 3, 2>), blocks_for(N, 2 * kBlock), kBlock, s, a);
    DPO_LAUNCH((k_policy_eval_d16<true, 0, 1>), blocks_for(N, kBlock), kBlock, s, a);
  }
  if (streamed) DPO_LAUNCH((k_policy_eval_d16<false, 3, 2>), blocks_for(a.n_free, 2 * kBlock), kBlock, s, a);
  DPO_LAUNCH((k_policy_eval_d16<false, 0, 1>), blocks_for(a.n_free, kBlock), kBlock, s, a);
}

hipError_t launch_resid_final(const double* partial, int nblocks, double* stage, double* out, hipStream_t s) {
  // One workgroup reads a few thousand partials quickly; beyond that (a
  // large grid leaves one partial per workgroup of its sweep) the first
  // stage spreads the read over up to kResidStage workgroups.
  const int g = std::min(kResidStage, (nblocks + 4 * kBlock - 1) / (4 * kBlock));
  if (g <= 1) DPO_LAUNCH(k_resid_final, 1, kBlock, s, partial, nblocks, out);
  hipLaunchKernelGGL(k_resid_final, dim3(g), dim3(kBlock), 0, s, partial, nblocks, stage);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  DPO_LAUNCH(k_resid_final, 1, kBlock, s, stage, g, out);
}

hipError_t launch_value_at(const float* V, const Grid& G, double M, const double x[4], double* out,
                           hipStream_t s) {
  DPO_LAUNCH(k_value_at, 1, 64, s, V, G, M, x[0], x[1], x[2], x[3], out);
}

hipError_t launch_feedback(const SweepArgs& a, const double* states, int n, double tau, float* ang,
                           uint8_t* thr, float* q, hipStream_t s) {
  if (n <= kWaveStates) DPO_LAUNCH(k_feedback<true>, (n + kBlock / 64 - 1) / (kBlock / 64), kBlock, s, a, states, n, tau, ang, thr, q);
  DPO_LAUNCH(k_feedback<false>, blocks_for(n), kBlock, s, a, states, n, tau, ang, thr, q);
}

hipError_t launch_simulate(const SweepArgs& a, double* states, int n, double tau, int steps, int substeps,
                           double drag, double* traj, uint8_t* thr_hist, float* ang_hist, hipStream_t s) {
  if (n <= kWaveStates)
    DPO_LAUNCH(k_simulate<true>, (n + kBlock / 64 - 1) / (kBlock / 64), kBlock, s, a, states, n, tau, steps, substeps,
               drag, traj, thr_hist, ang_hist);
  DPO_LAUNCH(k_simulate<false>, blocks_for(n), kBlock, s, a, states, n, tau, steps, substeps, drag, traj, thr_hist,
             ang_hist);
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
