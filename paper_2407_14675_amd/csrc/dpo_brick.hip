// Frozen-policy sweep over a dense grid with the value function staged in LDS
// (paper Section 3: eq:p_eval applied once, as modified policy iteration
// repeats it; memory is the first of the scheme's bottlenecks named there).
//
// The evaluation reads, per node, only the stored control (angle and
// throttle), writes the new value, and gathers 16 corners of V around the
// foot.  Feet stay within a few cells of their node, and mass only decreases
// (a thrust foot of mass plane p lies between planes p - 1 and p, a coast
// foot on plane p), so a workgroup owns a column of nodes -- every r, a tile
// of v_r rows and a tile of v_t rows -- and walks it through a run of mass
// planes in increasing order: the brick of V its nodes can reach on one plane
// (the tile plus the reach of the feet along v_r and v_t) is loaded into LDS
// once with 16-byte loads of contiguous v_r rows, two planes are resident (p - 1
// and p), and the next plane's brick is loaded into registers while plane p
// is computed.  The foot, the cell and the 15 lerps are those of the
// descriptor-free sweep (k_policy_eval), so the values are the same bit for
// bit; only where a corner comes from differs.
#include <type_traits>

#include "dpo_search.h"

namespace dpo {

namespace {

constexpr int kNodesPerThread = kBrickNodes;  // nodes of one plane-tile per thread, at most

// The cell value of one mass plane of the brick: 4 r-pairs, 7 lerps, in the
// order cell_value forms the same quantities (r, then v_r, then v_t).
__device__ inline float plane_value(const float* __restrict__ p, int s1, int s2, float t0, float t1, float t2) {
  const float c0 = lerp(p[0], p[1], t0);
  const float c1 = lerp(p[s1], p[s1 + 1], t0);
  const float c2 = lerp(p[s2], p[s2 + 1], t0);
  const float c3 = lerp(p[s1 + s2], p[s1 + s2 + 1], t0);
  const float d0 = lerp(c0, c1, t1);
  const float d1 = lerp(c2, c3, t1);
  return lerp(d0, d1, t2);
}

// q / d for 0 <= q < 2^20 and d >= 1 through a float reciprocal, with one
// correction step (the float quotient is within one of the true one).
__device__ inline int small_div(int q, int d, float inv_d) {
  int k = (int)((float)q * inv_d);
  const int r = q - k * d;
  if (r < 0) k--;
  else if (r >= d) k++;
  return k;
}

// One plane's brick: global loads into registers (fetch), then LDS stores
// (store).  Element e of the plane's loads is row e / units (a contiguous run
// of v_r rows at one v_t) and unit e % units of it.
struct BrickFill {
  const float* src;  // the plane's first valid row in V
  int units, total;
  float inv_units;
  int st2;           // V stride between v_t rows
  int lbase;         // LDS offset of the first valid row in slot 0
  int ls2;           // LDS stride between v_t rows
};

template <class Chunk, int kW, int kPf>
__device__ __forceinline__ void brick_fetch(const BrickFill& F, size_t plane_off, int slot_off, Chunk (&pf)[kPf],
                                            int (&pl)[kPf]) {
#pragma unroll
  for (int k = 0; k < kPf; k++) {
    const int e = threadIdx.x + k * kBrickBlock;
    pl[k] = -1;
    if (e < F.total) {
      const int row = small_div(e, F.units, F.inv_units);
      const int u = e - row * F.units;
      pf[k] = *reinterpret_cast<const Chunk*>(F.src + plane_off + (size_t)row * F.st2 + u * kW);
      pl[k] = slot_off + F.lbase + row * F.ls2 + u * kW;
    }
  }
}

template <class Chunk, int kPf>
__device__ __forceinline__ void brick_store(float* lds, const Chunk (&pf)[kPf], const int (&pl)[kPf]) {
#pragma unroll
  for (int k = 0; k < kPf; k++)
    if (pl[k] >= 0) *reinterpret_cast<Chunk*>(lds + pl[k]) = pf[k];
}

template <bool kResid, bool kVec, bool kNt>
__global__ __launch_bounds__(kBrickBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_brick(SweepArgs a, BrickPlan B,
                                                            const uint8_t* __restrict__ kind) {
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  // the native vector type (not HIP's float4 struct), so the prefetch array
  // stays in registers
  typedef float native4 __attribute__((ext_vector_type(4)));
  typedef typename std::conditional<kVec, native4, float>::type Chunk;
  constexpr int kW = kVec ? 4 : 1;               // floats per load
  constexpr int kPf = kVec ? kBrickMaxPf : 4 * kBrickMaxPf;

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int at = tile % B.n_at;
  const int ct = (tile / B.n_at) % B.n_ct;
  const int mc = tile / (B.n_at * B.n_ct);
  const int n0 = a.G.n[0], n1 = a.G.n[1], n2 = a.G.n[2], n3 = a.G.n[3];
  const int st1 = a.G.st[1], st2 = a.G.st[2], st3 = a.G.st[3];
  const int A = at * B.tr, C = ct * B.tt;
  const int p0 = mc * B.planes, p1 = min(p0 + B.planes, n3);
  const int4 halo = B.halo[at + B.n_at * ct];
  const int br = B.tr + halo.x + halo.y, bt = B.tt + halo.z + halo.w;  // this tile's brick rows
  const int r_lo = A - halo.x, t_lo = C - halo.z;  // brick origin along v_r, v_t (may be negative)
  const int vr0 = max(0, r_lo), vr1 = min(n1, A + B.tr + halo.y);
  const int vt0 = max(0, t_lo), vt1 = min(n2, C + B.tt + halo.w);
  const int ls1 = n0, ls2 = br * n0;             // LDS strides along v_r and v_t
  BrickFill F;
  F.src = a.V_in + (size_t)vt0 * st2 + (size_t)vr0 * n0;
  F.units = (vr1 - vr0) * n0 / kW;               // loads per contiguous run of v_r rows
  F.total = (vt1 - vt0) * F.units;               // loads per plane
  F.inv_units = 1.0f / (float)F.units;
  F.st2 = st2;
  F.lbase = (vt0 - t_lo) * ls2 + (vr0 - r_lo) * n0;
  F.ls2 = ls2;
  Chunk pf[kPf];
  int pl[kPf];

  const int first = max(p0 - 1, 0);
  brick_fetch<Chunk, kW, kPf>(F, (size_t)first * st3, (first & 1) * B.slot, pf, pl);
  brick_store<Chunk, kPf>(lds, pf, pl);
  if (first < p0) {
    brick_fetch<Chunk, kW, kPf>(F, (size_t)p0 * st3, (p0 & 1) * B.slot, pf, pl);
    brick_store<Chunk, kPf>(lds, pf, pl);
  }
  __syncthreads();

  const int per_plane = n0 * B.tr * B.tt;
  const float inv_n0 = 1.0f / (float)n0, inv_tr = 1.0f / (float)B.tr;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  for (int p = p0; p < p1; p++) {
    const bool more = p + 1 < p1;
    if (more) brick_fetch<Chunk, kW, kPf>(F, (size_t)(p + 1) * st3, ((p + 1) & 1) * B.slot, pf, pl);
    // the plane's nodes of this thread: coordinates, kind and control first,
    // so that their loads are in flight together
    int jj[kNodesPerThread], ii[kNodesPerThread][3];
    uint8_t th[kNodesPerThread];
    float uu[kNodesPerThread];
#pragma unroll
    for (int k = 0; k < kNodesPerThread; k++) {
      const int q = threadIdx.x + k * kBrickBlock;
      jj[k] = -1;
      if (q < per_plane) {
        const int rr = small_div(q, n0, inv_n0);
        const int i0 = q - rr * n0;
        const int rt = small_div(rr, B.tr, inv_tr);
        const int i1 = A + rr - rt * B.tr, i2 = C + rt;
        if (i1 < n1 && i2 < n2) {
          const int j = i0 + i1 * st1 + i2 * st2 + p * st3;
          if (kind[j] == 0) {
            jj[k] = j;
            ii[k][0] = i0;
            ii[k][1] = i1;
            ii[k][2] = i2;
            if (kNt) {
              th[k] = __builtin_nontemporal_load(a.pol_thr_in + j);
              uu[k] = __builtin_nontemporal_load(a.pol_ang_in + j);
            } else {
              th[k] = a.pol_thr_in[j];
              uu[k] = a.pol_ang_in[j];
            }
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kNodesPerThread; k++) {
      if (jj[k] < 0) continue;
      NodeTerms T;
      T.i[0] = ii[k][0];
      T.i[1] = ii[k][1];
      T.i[2] = ii[k][2];
      T.i[3] = p;
      node_terms_at(a, T);
      const int thr = th[k] ? 1 : 0;
      float sn = 0.0f, cs = 1.0f;
      if (thr) policy_sincos(a, uu[k], sn, cs);
      HeunTerms H;
      float off[4];
      foot_off<false>(T, H, thr, sn, cs, off);
      int base[4];
      float t[4];
      float I = a.P.M;
      if (foot_cell(a.G, T.i, off, base, t)) {
        const int y = base[2] - t_lo, x = base[1] - r_lo;
        if ((unsigned)y <= (unsigned)(bt - 2) && (unsigned)x <= (unsigned)(br - 2)) {
          const int o = y * ls2 + x * n0 + base[0];
          const float e0 = plane_value(lds + (base[3] & 1) * B.slot + o, ls1, ls2, t[0], t[1], t[2]);
          // lerp(e0, e1, 0) is e0 for any finite e1: a coast foot (t3 = 0) on
          // plane p reads only that plane
          const float e1 = t[3] != 0.0f ? plane_value(lds + ((base[3] + 1) & 1) * B.slot + o, ls1, ls2, t[0], t[1], t[2])
                                        : e0;
          I = lerp(e0, e1, t[3]);
        } else {
          // beyond the brick (the host's reach bound makes this unreachable):
          // the same cell from global memory
          I = cell_value(a.V_in + (base[0] + base[1] * st1 + base[2] * st2 + base[3] * st3), a.G, t, st3);
        }
      }
      const float out = fmaf(a.P.gamma, I, thr ? a.P.q_thr : a.P.q_coast);
      if (kNt) __builtin_nontemporal_store(out, a.V_out + jj[k]);
      else a.V_out[jj[k]] = out;
      if (kResid) {
        const float vin = lds[(p & 1) * B.slot + (ii[k][2] - t_lo) * ls2 + (ii[k][1] - r_lo) * n0 + ii[k][0]];
        node_residual(vin, out, rel, sum, mabs, bad);
      }
    }
    __syncthreads();  // every node of plane p is done with the slot plane p + 1 overwrites
    if (more) {
      brick_store<Chunk, kPf>(lds, pf, pl);
      __syncthreads();
    }
  }
  if (kResid) block_residual(rel, sum, mabs, bad, 0.0, a.partial, blockIdx.x);
}

// The same column walk driven by the foot descriptors of the greedy step
// (the packed per-node form: cell offsets and cell coordinates along v_r and
// v_t in eight bytes): per node one descriptor is streamed instead of the
// control, and the corners come from the brick.  Everything about a node
// that does not change from one mass plane to the next -- its offset in the
// plane, its brick row, its r cell and weight (r' = v_r does not depend on
// the control) -- is formed once per tile; the m cell and weight depend only
// on the plane and the throttle.  The next plane's descriptors are loaded
// together with its brick, while the current plane is computed.
// Same values, bit for bit, as the descriptor sweep that gathers from global
// memory (k_policy_eval_d16): the same cells, weights and lerps.
template <bool kVec, bool kNt>
__global__ __launch_bounds__(kBrickBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_brick_desc(
    SweepArgs a, BrickPlan B) {
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  typedef float native4 __attribute__((ext_vector_type(4)));
  typedef typename std::conditional<kVec, native4, float>::type Chunk;
  constexpr int kW = kVec ? 4 : 1;
  constexpr int kPf = kVec ? kBrickMaxPf : 4 * kBrickMaxPf;
  constexpr int kN = kNodesPerThread;

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int at = tile % B.n_at;
  const int ct = (tile / B.n_at) % B.n_ct;
  const int mc = tile / (B.n_at * B.n_ct);
  const int n0 = a.G.n[0], n1 = a.G.n[1], n2 = a.G.n[2], n3 = a.G.n[3];
  const int st1 = a.G.st[1], st2 = a.G.st[2], st3 = a.G.st[3];
  const int A = at * B.tr, C = ct * B.tt;
  const int p0 = mc * B.planes, p1 = min(p0 + B.planes, n3);
  const int4 halo = B.halo[at + B.n_at * ct];
  const int br = B.tr + halo.x + halo.y, bt = B.tt + halo.z + halo.w;
  const int r_lo = A - halo.x, t_lo = C - halo.z;
  const int vr0 = max(0, r_lo), vr1 = min(n1, A + B.tr + halo.y);
  const int vt0 = max(0, t_lo), vt1 = min(n2, C + B.tt + halo.w);
  const int ls1 = n0, ls2 = br * n0;

  // brick fill: each thread's loads at fixed offsets within a plane
  const float* src = a.V_in + (size_t)vt0 * st2 + (size_t)vr0 * n0;
  const int units = (vr1 - vr0) * n0 / kW, total = (vt1 - vt0) * units;
  const int lbase = (vt0 - t_lo) * ls2 + (vr0 - r_lo) * n0;
  // load k of a plane: its row run (bits 0-7) and float offset in the run
  // (bits 8-30); a thread's loads beyond the brick read its first element
  // again and are not stored (no branch around a load, so the wait counts
  // of the prefetch stay exact)
  int ld[kPf];
  int nld = 0;  // this thread's loads that are stored
  {
    const float inv_units = 1.0f / (float)units;
#pragma unroll
    for (int k = 0; k < kPf; k++) {
      const int e = threadIdx.x + k * kBrickBlock;
      ld[k] = 0;
      if (e < total) {
        const int row = small_div(e, units, inv_units);
        ld[k] = row | ((e - row * units) * kW << 8);
        nld = k + 1;
      }
    }
  }
  auto fetch = [&](int q, Chunk (&pf)[kPf]) {
    const float* sp = src + (size_t)q * st3;
#pragma unroll
    for (int k = 0; k < kPf; k++) pf[k] = *reinterpret_cast<const Chunk*>(sp + (ld[k] & 255) * st2 + (ld[k] >> 8));
  };
  auto store = [&](int q, const Chunk (&pf)[kPf]) {
    float* dp = lds + (q & 1) * B.slot + lbase;
#pragma unroll
    for (int k = 0; k < kPf; k++)
      if (k < nld) *reinterpret_cast<Chunk*>(dp + (ld[k] & 255) * ls2 + (ld[k] >> 8)) = pf[k];
  };

  // this thread's nodes of the tile (the same in every plane): rc packs the
  // node's r index (bits 0-7), its brick row along v_r (8-15) and v_t (16-23)
  // and its r cell (24-31); -1 (all ones, which no node has: the r cell is at
  // most 254) for none; t0 the r weight
  int rc[kN];
  float t0[kN];
  {
    const int per_plane = n0 * B.tr * B.tt;
    const float inv_n0 = 1.0f / (float)n0, inv_tr = 1.0f / (float)B.tr;
#pragma unroll
    for (int k = 0; k < kN; k++) {
      const int q = threadIdx.x + k * kBrickBlock;
      rc[k] = -1;
      t0[k] = 0.0f;
      if (q < per_plane) {
        const int rr = small_div(q, n0, inv_n0);
        const int i0 = q - rr * n0;
        const int rt = small_div(rr, B.tr, inv_tr);
        const int i1 = A + rr - rt * B.tr, i2 = C + rt;
        if (i1 < n1 && i2 < n2) {
          // r cell and weight exactly as the greedy sweep formed them (a
          // foot outside along r carries the outside bit; its cell is unused)
          int b0 = 0;
          float w0 = 0.0f;
          axis_cell(i0, n0, drift_r(a, i1), b0, w0);
          rc[k] = i0 | ((i1 - r_lo) << 8) | ((i2 - t_lo) << 16) | ((b0 & 255) << 24);
          t0[k] = w0;
        }
      }
    }
  }
  // the node's offset in a plane; a missing node reads the tile's first node
  auto node_of = [&](int k) {
    const int r = rc[k] == -1 ? (A - r_lo) << 8 | (C - t_lo) << 16 : rc[k];
    return (r & 255) + (((r >> 8) & 255) + r_lo) * st1 + (((r >> 16) & 255) + t_lo) * st2;
  };

  // the stream of one plane: the packed descriptors of this thread's nodes
  // (unconditional loads; a missing node's code is replaced by the skip code)
  typedef unsigned native_u2 __attribute__((ext_vector_type(2)));
  struct Stream {
    uint2 d[kN];
  };
  auto stream = [&](int q, Stream& S) {
    const size_t po = (size_t)q * st3;
#pragma unroll
    for (int k = 0; k < kN; k++) {
      const size_t j = po + node_of(k);
      native_u2 v;
      if (kNt) v = __builtin_nontemporal_load(reinterpret_cast<const native_u2*>(a.desc_pk_in) + j);
      else v = reinterpret_cast<const native_u2*>(a.desc_pk_in)[j];
      S.d[k] = make_uint2(v.x, v.y);
    }
  };

  // one plane from LDS; then, with the next plane's brick and stream already
  // in registers, the swap of LDS slots
  auto plane = [&](int p, const Stream& S) {
    // m cell and weight of the plane's coast and thrust feet (axis_cell, as
    // the greedy sweep formed them; a thrust foot below plane 0 is outside
    // and carries the outside bit)
    int bc, bth;
    float tc, tth;
    axis_cell(p, n3, 0.0f, bc, tc);
    axis_cell(p, n3, a.gm, bth, tth);
    const float* lc0 = lds + (bc & 1) * B.slot;
    const float* lc1 = lds + ((bc + 1) & 1) * B.slot;
    const float* lt0 = lds + (bth & 1) * B.slot;
    const float* lt1 = lds + ((bth + 1) & 1) * B.slot;
    float* vout = a.V_out + (size_t)p * st3;
#pragma unroll
    for (int k = 0; k < kN; k++) {
      // keep the packed node words packed: unpacking them once per tile
      // (loop-invariant hoisting) would take more registers than there are
      asm volatile("" : "+v"(rc[k]));
      const uint32_t c = desc_pk_code(S.d[k]);
      if (rc[k] == -1 || c == kDescPkSkip) continue;
      const float w1 = desc_pk_w1(S.d[k]), w2 = desc_pk_w2(S.d[k]);
      const bool thr = (c & kDescThr) != 0;
      float I = a.P.M;
      if (!(c & kDescOut)) {
        const int x = ((rc[k] >> 8) & 255) + (int)(c & 63u) - 32;
        const int y = ((rc[k] >> 16) & 255) + (int)((c >> 6) & 63u) - 32;
        const int b0 = (rc[k] >> 24) & 255;
        const float t3 = thr ? tth : tc;
        if ((unsigned)y <= (unsigned)(bt - 2) && (unsigned)x <= (unsigned)(br - 2)) {
          const int o = y * ls2 + x * n0 + b0;
          const float e0 = plane_value((thr ? lt0 : lc0) + o, ls1, ls2, t0[k], w1, w2);
          // lerp(e0, e1, 0) is e0 for any finite e1: a coast foot on plane p
          // reads only that plane
          const float e1 = t3 != 0.0f ? plane_value((thr ? lt1 : lc1) + o, ls1, ls2, t0[k], w1, w2) : e0;
          I = lerp(e0, e1, t3);
        } else {
          // beyond the brick (the host's reach bound makes this unreachable)
          const int b3 = thr ? bth : bc;
          const float t[4] = {t0[k], w1, w2, t3};
          const int b1 = x + r_lo, b2 = y + t_lo;
          I = cell_value(a.V_in + (b0 + b1 * st1 + b2 * st2 + b3 * st3), a.G, t, st3);
        }
      }
      const float out = fmaf(a.P.gamma, I, thr ? a.P.q_thr : a.P.q_coast);
      if (kNt) __builtin_nontemporal_store(out, vout + node_of(k));
      else vout[node_of(k)] = out;
      // one node at a time: interleaving the nodes' 16 corner reads would
      // need more registers than four waves per SIMD leave
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  Chunk pf[kPf];
  Stream s0, s1;
  const int first = max(p0 - 1, 0);
  fetch(first, pf);
  store(first, pf);
  if (first < p0) {
    fetch(p0, pf);
    store(p0, pf);
  }
  stream(p0, s0);
  __syncthreads();
  // planes in pairs, the two stream buffers alternating (no copies)
  for (int p = p0; p < p1; p += 2) {
    if (p + 1 < p1) {
      fetch(p + 1, pf);
      stream(p + 1, s1);
    }
    plane(p, s0);
    __syncthreads();
    if (p + 1 >= p1) break;
    store(p + 1, pf);
    __syncthreads();
    if (p + 2 < p1) {
      fetch(p + 2, pf);
      stream(p + 2, s0);
    }
    plane(p + 1, s1);
    __syncthreads();
    if (p + 2 >= p1) break;
    store(p + 2, pf);
    __syncthreads();
  }
}

}  // namespace

size_t brick_lds_bytes(const BrickPlan& B) { return sizeof(float) * 2 * (size_t)B.slot; }

hipError_t launch_eval_brick_desc(const SweepArgs& a, const BrickPlan& B, bool streamed, hipStream_t s) {
  const int grid = B.n_at * B.n_ct * B.n_mc;
  const size_t lds = brick_lds_bytes(B);
  const bool vec = (a.G.n[0] % 4) == 0;
#define DPO_BRICK_D(V, N) hipLaunchKernelGGL((k_eval_brick_desc<V, N>), dim3(grid), dim3(kBrickBlock), lds, s, a, B)
  if (streamed) {
    if (vec) DPO_BRICK_D(true, true);
    else DPO_BRICK_D(false, true);
  } else {
    if (vec) DPO_BRICK_D(true, false);
    else DPO_BRICK_D(false, false);
  }
#undef DPO_BRICK_D
  return hipGetLastError();
}

hipError_t launch_eval_brick(const SweepArgs& a, const BrickPlan& B, const uint8_t* kind, bool want_resid,
                             bool streamed, hipStream_t s) {
  const int grid = B.n_at * B.n_ct * B.n_mc;
  const size_t lds = brick_lds_bytes(B);
  const bool vec = (a.G.n[0] % 4) == 0;
#define DPO_BRICK(R, V, N) \
  hipLaunchKernelGGL((k_eval_brick<R, V, N>), dim3(grid), dim3(kBrickBlock), lds, s, a, B, kind)
  if (want_resid) {
    if (vec) DPO_BRICK(true, true, false);
    else DPO_BRICK(true, false, false);
  } else if (streamed) {
    if (vec) DPO_BRICK(false, true, true);
    else DPO_BRICK(false, false, true);
  } else {
    if (vec) DPO_BRICK(false, true, false);
    else DPO_BRICK(false, false, false);
  }
#undef DPO_BRICK
  return hipGetLastError();
}

// Kernel attribute set-up: the largest dynamic LDS a launch of the plan
// takes (two plane slots); a refusal is cleared from the runtime's error
// state and returned.
hipError_t prepare_eval_brick(const BrickPlan& B) {
  const int bytes = (int)brick_lds_bytes(B);
  hipError_t e = hipSuccess;
#define DPO_BRICK_ATTR(R, V, N)                                                                        \
  if (e == hipSuccess)                                                                                 \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eval_brick<R, V, N>),                       \
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes)
  DPO_BRICK_ATTR(true, true, false);
  DPO_BRICK_ATTR(true, false, false);
  DPO_BRICK_ATTR(false, true, true);
  DPO_BRICK_ATTR(false, false, true);
  DPO_BRICK_ATTR(false, true, false);
  DPO_BRICK_ATTR(false, false, false);
#undef DPO_BRICK_ATTR
#define DPO_BRICK_D_ATTR(V, N)                                                                        \
  if (e == hipSuccess)                                                                                \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eval_brick_desc<V, N>),                    \
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes)
  DPO_BRICK_D_ATTR(true, true);
  DPO_BRICK_D_ATTR(false, true);
  DPO_BRICK_D_ATTR(true, false);
  DPO_BRICK_D_ATTR(false, false);
#undef DPO_BRICK_D_ATTR
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

}  // namespace dpo
