// Kernels and C ABI of the control-proposal network (see dpo_mlp.h).
//
// One workgroup of 4 waves handles a tile of 64 samples.  Layer 1 (K = 4)
// and layer 3 (N = 3) run on the vector units; the 128 x 128 layer and the
// two products of its backward pass run on the matrix cores
// (v_mfma_f32_16x16x16_bf16): wave w owns samples 16w .. 16w+15.  Operand
// fragments come from LDS tiles stored K-contiguous, so each lane loads its
// four bf16 values with one 8-byte read; rows are padded by 8 elements to
// spread the 16 rows of a fragment over the LDS banks.
//
// Gradients are summed per tile and then over tiles in a fixed order, so a
// training run is deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dpo.h"
#include "dpo_kernels.h"
#include "dpo_mlp.h"

namespace dpo {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLdA = kHid + 8;       // row stride of sample-major tiles [64][128]
constexpr int kLdT = kMlpTile + 8;   // row stride of unit-major tiles [128][64]
constexpr int kRed = 3 * kHid + 4 + kHid + 5 * kHid;  // per-wave reduction slots

// float -> bfloat16, round to nearest, ties to even (finite inputs).
__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Pre-activation of hidden unit k of layer 1 (the same expression in the
// forward and the backward pass).
__device__ inline float z1_of(const float4& w, float b, const float4& x) {
  return fmaf(w.w, x.w, fmaf(w.z, x.z, fmaf(w.y, x.y, fmaf(w.x, x.x, b))));
}

// Grid position of a node scaled to [-1, 1] per axis.
__device__ inline float4 unit_coords(const Grid& G, const int i[4]) {
  return make_float4((float)(2 * i[0]) / (float)(G.n[0] - 1) - 1.0f, (float)(2 * i[1]) / (float)(G.n[1] - 1) - 1.0f,
                     (float)(2 * i[2]) / (float)(G.n[2] - 1) - 1.0f, (float)(2 * i[3]) / (float)(G.n[3] - 1) - 1.0f);
}

// One wave: D[16][128] = A[16][K] * Bt[128][K]^T with A and Bt bf16,
// row-major, K-contiguous.  Lane (r = lane % 16, g = lane / 16) ends with
// D[4g + i][16 nt + r] in acc[nt][i].
template <int K>
__device__ inline void wave_gemm(const uint16_t* A, int lda, const uint16_t* Bt, int ldb, f32x4 acc[8]) {
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < 8; nt++) acc[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kk = 0; kk < K; kk += 16) {
    const bf16x4 a = *reinterpret_cast<const bf16x4*>(A + r * lda + kk + 4 * g);
#pragma unroll
    for (int nt = 0; nt < 8; nt++) {
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(Bt + (nt * 16 + r) * ldb + kk + 4 * g);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nt], 0, 0, 0);
    }
  }
}

// Layer 1 for the tile: h1 = GELU(W1 x + b1) as bf16, sample-major into h1
// and, when kT, unit-major into h1t.  256 threads: unit k = tid % 128, half
// of the samples each.
template <bool kT>
__device__ inline void layer1(const float* theta, const float4* xs, uint16_t* h1, uint16_t* h1t) {
  const int k = threadIdx.x & (kHid - 1), half = threadIdx.x >> 7;
  const float4 w = reinterpret_cast<const float4*>(theta + kOW1)[k];
  const float b = theta[kOB1 + k];
  for (int s = half * 32; s < half * 32 + 32; s += 2) {
    const uint16_t p = bf16_rne(gelu(z1_of(w, b, xs[s])));
    const uint16_t q = bf16_rne(gelu(z1_of(w, b, xs[s + 1])));
    h1[s * kLdA + k] = p;
    h1[(s + 1) * kLdA + k] = q;
    if (kT) *reinterpret_cast<uint32_t*>(h1t + k * kLdT + s) = (uint32_t)p | ((uint32_t)q << 16);
  }
}

// Layer 2 bias + GELU and layer 3 for the wave's 16 samples.  z2 (in: the
// matrix product, out: with bias) and h2 are in the MFMA output layout; y[i]
// holds the three outputs of sample 16w + 4g + i in all 16 lanes of group g.
__device__ inline void layer3(const float* theta, f32x4 z2[8], f32x4 h2[8], float y[4][3]) {
  const int r = threadIdx.x & 15;
  float p[4][3];
#pragma unroll
  for (int i = 0; i < 4; i++) p[i][0] = p[i][1] = p[i][2] = 0.0f;
#pragma unroll
  for (int nt = 0; nt < 8; nt++) {
    const int n = nt * 16 + r;
    const float b2 = theta[kOB2 + n];
    const float w0 = theta[kOW3 + n], w1 = theta[kOW3 + kHid + n], w2 = theta[kOW3 + 2 * kHid + n];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const float z = z2[nt][i] + b2;
      const float h = gelu(z);
      z2[nt][i] = z;
      h2[nt][i] = h;
      p[i][0] = fmaf(h, w0, p[i][0]);
      p[i][1] = fmaf(h, w1, p[i][1]);
      p[i][2] = fmaf(h, w2, p[i][2]);
    }
  }
#pragma unroll
  for (int m = 8; m >= 1; m >>= 1)
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int o = 0; o < 3; o++) p[i][o] += __shfl_xor(p[i][o], m, 64);
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int o = 0; o < 3; o++) y[i][o] = p[i][o] + theta[kOB3 + o];
}

template <int kN>
__device__ inline void group_sum(float (&v)[kN]) {
#pragma unroll
  for (int m = 16; m <= 32; m <<= 1)
#pragma unroll
    for (int q = 0; q < kN; q++) v[q] += __shfl_xor(v[q], m, 64);
}

__global__ __launch_bounds__(256) void k_mlp_forward(MlpArgs a) {
  __shared__ float4 xs[kMlpTile];
  __shared__ __attribute__((aligned(16))) uint16_t h1[kMlpTile * kLdA];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int s0 = blockIdx.x * kMlpTile;
  if (tid < kMlpTile) xs[tid] = (s0 + tid < a.n) ? a.x[s0 + tid] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  __syncthreads();
  layer1<false>(a.theta, xs, h1, nullptr);
  __syncthreads();
  f32x4 z2[8], h2[8];
  float y[4][3];
  wave_gemm<kHid>(h1 + 16 * w * kLdA, kLdA, a.w2, kHid, z2);
  layer3(a.theta, z2, h2, y);
  if (r < 4) {
    const int s = s0 + 16 * w + 4 * g + r;
    if (s < a.n) {
#pragma unroll
      for (int i = 0; i < 4; i++)
        if (i == r) {
          a.y[3 * (size_t)s + 0] = y[i][0];
          a.y[3 * (size_t)s + 1] = y[i][1];
          a.y[3 * (size_t)s + 2] = y[i][2];
        }
    }
  }
}

// Forward and backward of one tile of a batch; writes the tile's gradient
// sums (and its summed loss) to partial[blockIdx.x].
__global__ __launch_bounds__(256) void k_mlp_grad(MlpArgs a) {
  __shared__ float4 xs[kMlpTile];
  __shared__ float4 tg[kMlpTile];
  __shared__ __attribute__((aligned(16))) uint16_t act[kMlpTile * kLdA];  // h1, then d2 (sample-major)
  __shared__ __attribute__((aligned(16))) uint16_t h1t[kHid * kLdT];
  __shared__ __attribute__((aligned(16))) uint16_t d2t[kHid * kLdT];
  __shared__ float red[4][kRed];
  __shared__ __attribute__((aligned(16))) uint16_t w2s[kHid * kLdA];   // W2 [out][in]
  __shared__ __attribute__((aligned(16))) uint16_t w2ts[kHid * kLdA];  // W2 [in][out]
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int s0 = blockIdx.x * kMlpTile;
  float* part = a.partial + (size_t)blockIdx.x * kPStride;
  // both bf16 copies of W2 staged once: 128 rows of 16 chunks of 8 bf16 each
  for (int c = tid; c < kHid * 16; c += 256) {
    const int row = c >> 4, col = (c & 15) * 8;
    *reinterpret_cast<uint4*>(w2s + row * kLdA + col) = *reinterpret_cast<const uint4*>(a.w2 + row * kHid + col);
    *reinterpret_cast<uint4*>(w2ts + row * kLdA + col) = *reinterpret_cast<const uint4*>(a.w2t + row * kHid + col);
  }
  if (tid < kMlpTile) {
    float4 xv = make_float4(0.0f, 0.0f, 0.0f, 0.0f), tv = xv;
    if (s0 + tid < a.n) {
      const int src = a.perm ? a.perm[s0 + tid] : s0 + tid;
      xv = a.x[src];
      tv = a.tgt[src];
    }
    xs[tid] = xv;
    tg[tid] = tv;
  }
  __syncthreads();
  layer1<true>(a.theta, xs, act, h1t);
  __syncthreads();

  // ---- forward of the wave's 16 samples
  f32x4 z2[8], h2[8];
  float y[4][3];
  wave_gemm<kHid>(act + 16 * w * kLdA, kLdA, w2s, kLdA, z2);
  layer3(a.theta, z2, h2, y);

  // ---- loss and its derivative with respect to (c, s, logit)
  float dy[4][3], lsum = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int s = 16 * w + 4 * g + i;
    const bool valid = s0 + s < a.n;
    const float4 t4 = tg[s];
    const float e0 = y[i][0] - t4.x, e1 = y[i][1] - t4.y, lg = y[i][2], th = t4.z;
    const float li = th * (e0 * e0 + e1 * e1) + fmaxf(lg, 0.0f) - lg * th + log1pf(expf(-fabsf(lg)));
    const float sig = 1.0f / (1.0f + expf(-lg));
    dy[i][0] = valid ? 2.0f * th * e0 * a.inv_n : 0.0f;
    dy[i][1] = valid ? 2.0f * th * e1 * a.inv_n : 0.0f;
    dy[i][2] = valid ? (sig - th) * a.inv_n : 0.0f;
    lsum += valid ? li : 0.0f;
  }

  // ---- W3, b3 and the loss: sums over the wave's samples
  {
    float q[8 * 3];
#pragma unroll
    for (int nt = 0; nt < 8; nt++)
#pragma unroll
      for (int o = 0; o < 3; o++) {
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; i++) acc = fmaf(dy[i][o], h2[nt][i], acc);
        q[nt * 3 + o] = acc;
      }
    group_sum(q);
    float e[4] = {0.0f, 0.0f, 0.0f, lsum};
#pragma unroll
    for (int i = 0; i < 4; i++) {
      e[0] += dy[i][0];
      e[1] += dy[i][1];
      e[2] += dy[i][2];
    }
    group_sum(e);
    if (g == 0) {
#pragma unroll
      for (int nt = 0; nt < 8; nt++)
#pragma unroll
        for (int o = 0; o < 3; o++) red[w][o * kHid + nt * 16 + r] = q[nt * 3 + o];
      if (r == 0)
#pragma unroll
        for (int o = 0; o < 4; o++) red[w][3 * kHid + o] = e[o];
    }
  }

  // ---- delta of layer 2: (W3^T dy) * GELU'(z2)
  f32x4 d2[8];
#pragma unroll
  for (int nt = 0; nt < 8; nt++) {
    const int n = nt * 16 + r;
    const float w0 = a.theta[kOW3 + n], w1 = a.theta[kOW3 + kHid + n], w2 = a.theta[kOW3 + 2 * kHid + n];
#pragma unroll
    for (int i = 0; i < 4; i++)
      d2[nt][i] = fmaf(dy[i][2], w2, fmaf(dy[i][1], w1, dy[i][0] * w0)) * gelu_grad(z2[nt][i]);
  }
  __syncthreads();  // every wave is done with h1 in act
  {
    float e[8];
#pragma unroll
    for (int nt = 0; nt < 8; nt++) {
      const int n = nt * 16 + r;
      uint16_t b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) {
        b[i] = bf16_rne(d2[nt][i]);
        act[(16 * w + 4 * g + i) * kLdA + n] = b[i];
      }
      *reinterpret_cast<uint2*>(d2t + n * kLdT + 16 * w + 4 * g) =
          make_uint2((uint32_t)b[0] | ((uint32_t)b[1] << 16), (uint32_t)b[2] | ((uint32_t)b[3] << 16));
      e[nt] = (d2[nt][0] + d2[nt][1]) + (d2[nt][2] + d2[nt][3]);
    }
    group_sum(e);
    if (g == 0)
#pragma unroll
      for (int nt = 0; nt < 8; nt++) red[w][3 * kHid + 4 + nt * 16 + r] = e[nt];
  }
  __syncthreads();

  // ---- W2 gradient d2^T h1 (K = the tile's 64 samples); wave w owns units 32w .. 32w+31
#pragma unroll
  for (int mt = 0; mt < 2; mt++) {
    f32x4 acc[8];
    const int row0 = 32 * w + 16 * mt;
    wave_gemm<kMlpTile>(d2t + row0 * kLdT, kLdT, h1t, kLdT, acc);
#pragma unroll
    for (int nt = 0; nt < 8; nt++)
#pragma unroll
      for (int i = 0; i < 4; i++) part[kOW2 + (row0 + 4 * g + i) * kHid + nt * 16 + r] = acc[nt][i];
  }

  // ---- back through W2: dh1 = d2 W2, then delta of layer 1 and the W1, b1 sums
  {
    f32x4 dh[8];
    wave_gemm<kHid>(act + 16 * w * kLdA, kLdA, w2ts, kLdA, dh);
    float q[8 * 5];
#pragma unroll
    for (int nt = 0; nt < 8; nt++) {
      const int k = nt * 16 + r;
      const float4 wk = reinterpret_cast<const float4*>(a.theta + kOW1)[k];
      const float bk = a.theta[kOB1 + k];
      float acc[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const float4 x = xs[16 * w + 4 * g + i];
        const float d1 = dh[nt][i] * gelu_grad(z1_of(wk, bk, x));
        acc[0] = fmaf(d1, x.x, acc[0]);
        acc[1] = fmaf(d1, x.y, acc[1]);
        acc[2] = fmaf(d1, x.z, acc[2]);
        acc[3] = fmaf(d1, x.w, acc[3]);
        acc[4] += d1;
      }
#pragma unroll
      for (int c = 0; c < 5; c++) q[nt * 5 + c] = acc[c];
    }
    group_sum(q);
    if (g == 0)
#pragma unroll
      for (int nt = 0; nt < 8; nt++)
#pragma unroll
        for (int c = 0; c < 5; c++) red[w][4 * kHid + 4 + (nt * 16 + r) * 5 + c] = q[nt * 5 + c];
  }
  __syncthreads();

  // ---- combine the four waves (fixed order) and write the tile's row
  for (int e = tid; e < kRed; e += 256) {
    const float v = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    int p;
    if (e < 3 * kHid) p = kOW3 + e;
    else if (e < 3 * kHid + 3) p = kOB3 + (e - 3 * kHid);
    else if (e == 3 * kHid + 3) p = kNParam;  // summed loss
    else if (e < 4 * kHid + 4) p = kOB2 + (e - 3 * kHid - 4);
    else {
      const int u = e - 4 * kHid - 4, k = u / 5, c = u % 5;
      p = c < 4 ? kOW1 + 4 * k + c : kOB1 + k;
    }
    part[p] = v;
  }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(ReduceArgs a) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > kNParam) return;
  // tile sums in a fixed order; eight loads in flight per thread
  float s = 0.0f;
  int t = 0;
  for (; t + 8 <= a.tiles; t += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = a.partial[(size_t)(t + u) * kPStride + p];
#pragma unroll
    for (int u = 0; u < 8; u++) s += v[u];
  }
  for (; t < a.tiles; t++) s += a.partial[(size_t)t * kPStride + p];
  if (p == kNParam) {
    if (a.loss) *a.loss = s * a.inv_n;
    return;
  }
  if (a.grad) a.grad[p] = s;
  if (!a.update) return;
  const float m = a.b1 * a.m[p] + (1.0f - a.b1) * s;
  const float v = a.b2 * a.v[p] + (1.0f - a.b2) * s * s;
  a.m[p] = m;
  a.v[p] = v;
  const float th = a.theta[p] - a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
  a.theta[p] = th;
  if (p >= kOW2 && p < kOB2) {
    const int q = p - kOW2, o = q / kHid, i = q % kHid;
    const uint16_t b = bf16_rne(th);
    a.w2[q] = b;
    a.w2t[i * kHid + o] = b;
  }
}

__global__ __launch_bounds__(256) void k_mlp_cast(const float* __restrict__ theta, uint16_t* __restrict__ w2,
                                                  uint16_t* __restrict__ w2t) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= kHid * kHid) return;
  const uint16_t b = bf16_rne(theta[kOW2 + q]);
  w2[q] = b;
  w2t[(q % kHid) * kHid + q / kHid] = b;
}

__global__ __launch_bounds__(256) void k_mlp_propose(const float* __restrict__ theta, const uint16_t* __restrict__ w2,
                                                     Grid G, const uint32_t* __restrict__ nodes, int n,
                                                     float* __restrict__ seed) {
  __shared__ __attribute__((aligned(16))) uint16_t w2s[kHid * kLdA];
  __shared__ __attribute__((aligned(16))) uint16_t h1[kMlpTile * kLdA];
  __shared__ float4 xs[kMlpTile];
  __shared__ int js[kMlpTile];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  // W2 staged once per workgroup: 128 rows of 16 chunks of 8 bf16
  for (int c = tid; c < kHid * 16; c += 256) {
    const int row = c >> 4, col = (c & 15) * 8;
    *reinterpret_cast<uint4*>(w2s + row * kLdA + col) = *reinterpret_cast<const uint4*>(w2 + row * kHid + col);
  }
  const int tiles = (n + kMlpTile - 1) / kMlpTile;
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    if (tid < kMlpTile) {
      const int t = tile * kMlpTile + tid;
      if (t < n) {
        int i[4];
        js[tid] = unpack_node(G, nodes[t], i);
        xs[tid] = unit_coords(G, i);
      } else {
        js[tid] = -1;
        xs[tid] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
    }
    __syncthreads();
    layer1<false>(theta, xs, h1, nullptr);
    __syncthreads();
    f32x4 z2[8], h2[8];
    float y[4][3];
    wave_gemm<kHid>(h1 + 16 * w * kLdA, kLdA, w2s, kLdA, z2);
    layer3(theta, z2, h2, y);
    if (r < 4) {
      const int j = js[16 * w + 4 * g + r];
      float c = y[0][0], s = y[0][1];
#pragma unroll
      for (int i = 1; i < 4; i++)
        if (i == r) {
          c = y[i][0];
          s = y[i][1];
        }
      if (j >= 0) seed[j] = atan2f(s, c);
    }
    __syncthreads();  // xs, js and h1 are rewritten by the next tile
  }
}

__global__ __launch_bounds__(kBlock) void k_feasible_flags(const uint8_t* __restrict__ kind,
                                                           const float* __restrict__ V, float thresh,
                                                           uint8_t* __restrict__ flag, int N) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < N) flag[j] = (kind[j] == 0 && V[j] < thresh) ? 0 : 1;
}

__global__ __launch_bounds__(kBlock) void k_gather_pairs(Grid G, const uint32_t* __restrict__ nodes,
                                                         const int* __restrict__ sel, int n,
                                                         const float* __restrict__ ang,
                                                         const uint8_t* __restrict__ thr, float4* __restrict__ x,
                                                         float4* __restrict__ tgt) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  int i[4];
  const int j = unpack_node(G, nodes[sel[t]], i);
  x[t] = unit_coords(G, i);
  float s, c;
  sincosf(ang[j], &s, &c);
  tgt[t] = make_float4(c, s, thr[j] ? 1.0f : 0.0f, 0.0f);
}

int mlp_tiles(int n) { return (n + kMlpTile - 1) / kMlpTile; }

hipError_t launch_mlp_forward(const MlpArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(mlp_tiles(a.n)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(mlp_tiles(a.n)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mlp_reduce(const ReduceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParam + 1 + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mlp_cast(const float* theta, uint16_t* w2, uint16_t* w2t, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_cast, dim3(kHid * kHid / 256), dim3(256), 0, s, theta, w2, w2t);
  return hipGetLastError();
}

hipError_t launch_mlp_propose(const float* theta, const uint16_t* w2, const Grid& G, const uint32_t* nodes, int n,
                              float* seed, int max_blocks, hipStream_t s) {
  const int blocks = std::max(1, std::min(max_blocks, mlp_tiles(n)));
  hipLaunchKernelGGL(k_mlp_propose, dim3(blocks), dim3(256), 0, s, theta, w2, G, nodes, n, seed);
  return hipGetLastError();
}

hipError_t launch_feasible_flags(const uint8_t* kind, const float* V, float thresh, uint8_t* flag, int N,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_feasible_flags, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, kind, V, thresh, flag,
                     N);
  return hipGetLastError();
}

hipError_t launch_gather_pairs(const Grid& G, const uint32_t* nodes, const int* sel, int n, const float* ang,
                               const uint8_t* thr, float4* x, float4* tgt, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_pairs, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, G, nodes, sel, n, ang, thr,
                     x, tgt);
  return hipGetLastError();
}

}  // namespace dpo

// ------------------------------------------------------------------ C ABI
using namespace dpo;

struct dpo_mlp {
  float* theta = nullptr;  // FP32 parameters
  float* m = nullptr;      // Adam moments
  float* v = nullptr;
  float* grad = nullptr;   // gradient of the last batch
  float* loss = nullptr;   // scratch loss of dpo_mlp_grad / train without history
  uint16_t* w2 = nullptr;
  uint16_t* w2t = nullptr;
  float* partial = nullptr;
  int partial_tiles = 0;
  int* perm = nullptr;
  int64_t perm_cap = 0;
  int* perm_host = nullptr;           // pinned staging of the epoch's order (host copy of perm)
  hipEvent_t perm_copied = nullptr;   // the staging buffer's last upload has completed
  hipEvent_t work_done = nullptr;     // the network's last queued work (any stream) has completed
  int max_blocks = 512;
  double lr = 1e-3, b1 = 0.9, b2 = 0.999, eps = 1e-8;
  int64_t step = 0;
  std::string err;
};

namespace {

thread_local std::string g_mlp_err;

int mfail(dpo_mlp* m, int code, const std::string& msg) {
  if (m) m->err = msg;
  else g_mlp_err = msg;
  return code;
}

#define MLP_HIP(m, call)                                                                        \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return mfail((m), DPO_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

hipStream_t MS(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int64_t kMaxBatch = 65536;

int ensure_partial(dpo_mlp* m, int tiles) {
  if (tiles <= m->partial_tiles) return DPO_OK;
  if (m->partial) (void)hipFree(m->partial);
  m->partial = nullptr;
  m->partial_tiles = 0;
  if (hipMalloc(&m->partial, (size_t)tiles * kPStride * sizeof(float)) != hipSuccess)
    return mfail(m, DPO_ENOMEM, "partial gradient buffer");
  m->partial_tiles = tiles;
  return DPO_OK;
}

int ensure_perm(dpo_mlp* m, int64_t n) {
  if (!m->perm_copied && hipEventCreateWithFlags(&m->perm_copied, hipEventDisableTiming) != hipSuccess) {
    m->perm_copied = nullptr;
    return mfail(m, DPO_EHIP, "permutation event");
  }
  if (n <= m->perm_cap) return DPO_OK;
  // the buffers may still be in use by steps and an upload queued by the last call
  if (hipDeviceSynchronize() != hipSuccess) return mfail(m, DPO_EHIP, "permutation buffer");
  if (m->perm) (void)hipFree(m->perm);
  if (m->perm_host) (void)hipHostFree(m->perm_host);
  m->perm = nullptr;
  m->perm_host = nullptr;
  m->perm_cap = 0;
  if (hipMalloc(&m->perm, (size_t)n * sizeof(int)) != hipSuccess ||
      hipHostMalloc(&m->perm_host, (size_t)n * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return mfail(m, DPO_ENOMEM, "permutation buffer");
  m->perm_cap = n;
  return DPO_OK;
}

ReduceArgs reduce_args(dpo_mlp* m, int tiles, int n, float* loss, int update) {
  ReduceArgs r{};
  r.partial = m->partial;
  r.tiles = tiles;
  r.inv_n = 1.0f / (float)n;
  r.grad = m->grad;
  r.loss = loss;
  r.update = update;
  r.theta = m->theta;
  r.m = m->m;
  r.v = m->v;
  r.w2 = m->w2;
  r.w2t = m->w2t;
  r.lr = (float)m->lr;
  r.b1 = (float)m->b1;
  r.b2 = (float)m->b2;
  r.eps = (float)m->eps;
  r.c1 = 1.0f;
  r.c2 = 1.0f;
  return r;
}

MlpArgs mlp_args(dpo_mlp* m, const float* x, const float* tgt, const int* perm, int n) {
  MlpArgs a{};
  a.theta = m->theta;
  a.w2 = m->w2;
  a.w2t = m->w2t;
  a.x = reinterpret_cast<const float4*>(x);
  a.tgt = reinterpret_cast<const float4*>(tgt);
  a.perm = perm;
  a.n = n;
  a.inv_n = 1.0f / (float)n;
  a.partial = m->partial;
  return a;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Work on the network's buffers (parameters, Adam state, gradient rows, the
// device copy of the order) is ordered across streams: each asynchronous call
// first makes its stream wait for the previous call's last queued work, and
// records its own at the end.  Calls on one stream are ordered anyway.
hipError_t after_previous(dpo_mlp* m, hipStream_t s) { return hipStreamWaitEvent(s, m->work_done, 0); }
hipError_t mark_done(dpo_mlp* m, hipStream_t s) { return hipEventRecord(m->work_done, s); }

}  // namespace

extern "C" {

int dpo_mlp_create(const float* params, dpo_mlp** out) {
  if (!out) return mfail(nullptr, DPO_EINVAL, "out is NULL");
  *out = nullptr;
  dpo_mlp* m = new dpo_mlp();
  const size_t bytes = (size_t)kNParam * sizeof(float);
  bool ok = hipMalloc(&m->theta, bytes) == hipSuccess && hipMalloc(&m->m, bytes) == hipSuccess &&
            hipMalloc(&m->v, bytes) == hipSuccess && hipMalloc(&m->grad, bytes) == hipSuccess &&
            hipMalloc(&m->loss, sizeof(float)) == hipSuccess &&
            hipMalloc(&m->w2, kHid * kHid * sizeof(uint16_t)) == hipSuccess &&
            hipMalloc(&m->w2t, kHid * kHid * sizeof(uint16_t)) == hipSuccess;
  if (!ok) {
    dpo_mlp_destroy(m);
    return mfail(nullptr, DPO_ENOMEM, "network parameter buffers");
  }
  if (hipEventCreateWithFlags(&m->work_done, hipEventDisableTiming) != hipSuccess) {
    m->work_done = nullptr;
    dpo_mlp_destroy(m);
    return mfail(nullptr, DPO_EHIP, "network event");
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    m->max_blocks = 2 * cus;
  std::vector<float> zeros(kNParam, 0.0f);
  int rc = dpo_mlp_set_params(m, params ? params : zeros.data());
  if (rc != DPO_OK) {
    g_mlp_err = m->err;
    dpo_mlp_destroy(m);
    return rc;
  }
  *out = m;
  return DPO_OK;
}

void dpo_mlp_destroy(dpo_mlp* m) {
  if (!m) return;
  (void)hipFree(m->theta);
  (void)hipFree(m->m);
  (void)hipFree(m->v);
  (void)hipFree(m->grad);
  (void)hipFree(m->loss);
  (void)hipFree(m->w2);
  (void)hipFree(m->w2t);
  (void)hipFree(m->partial);
  (void)hipFree(m->perm);
  if (m->perm_copied) {
    (void)hipEventSynchronize(m->perm_copied);
    (void)hipEventDestroy(m->perm_copied);
  }
  if (m->work_done) {
    (void)hipEventSynchronize(m->work_done);
    (void)hipEventDestroy(m->work_done);
  }
  if (m->perm_host) (void)hipHostFree(m->perm_host);
  delete m;
}

const char* dpo_mlp_last_error(const dpo_mlp* m) { return m ? m->err.c_str() : g_mlp_err.c_str(); }

int dpo_mlp_set_params(dpo_mlp* m, const float* params) {
  if (!m || !params) return mfail(m, DPO_EINVAL, "NULL argument");
  for (int p = 0; p < kNParam; p++)
    if (!std::isfinite(params[p])) return mfail(m, DPO_EINVAL, "parameters must be finite");
  const size_t bytes = (size_t)kNParam * sizeof(float);
  MLP_HIP(m, hipMemcpy(m->theta, params, bytes, hipMemcpyHostToDevice));
  MLP_HIP(m, hipMemset(m->m, 0, bytes));
  MLP_HIP(m, hipMemset(m->v, 0, bytes));
  MLP_HIP(m, hipMemset(m->grad, 0, bytes));
  MLP_HIP(m, launch_mlp_cast(m->theta, m->w2, m->w2t, nullptr));
  MLP_HIP(m, hipDeviceSynchronize());
  m->step = 0;
  return DPO_OK;
}

int dpo_mlp_get_params(dpo_mlp* m, float* params) {
  if (!m || !params) return mfail(m, DPO_EINVAL, "NULL argument");
  MLP_HIP(m, hipDeviceSynchronize());
  MLP_HIP(m, hipMemcpy(params, m->theta, (size_t)kNParam * sizeof(float), hipMemcpyDeviceToHost));
  return DPO_OK;
}

int dpo_mlp_get_grad(dpo_mlp* m, float* grad) {
  if (!m || !grad) return mfail(m, DPO_EINVAL, "NULL argument");
  MLP_HIP(m, hipDeviceSynchronize());
  MLP_HIP(m, hipMemcpy(grad, m->grad, (size_t)kNParam * sizeof(float), hipMemcpyDeviceToHost));
  return DPO_OK;
}

int dpo_mlp_set_adam(dpo_mlp* m, double lr, double beta1, double beta2, double eps) {
  if (!m) return mfail(m, DPO_EINVAL, "NULL argument");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return mfail(m, DPO_EINVAL, "adam: need lr > 0, 0 <= beta < 1, eps > 0");
  m->lr = lr;
  m->b1 = beta1;
  m->b2 = beta2;
  m->eps = eps;
  return DPO_OK;
}

int64_t dpo_mlp_steps(const dpo_mlp* m) { return m ? m->step : -1; }

int dpo_mlp_forward(dpo_mlp* m, const float* x, int64_t n, float* y, void* stream) {
  if (!m || (n > 0 && (!x || !y))) return mfail(m, DPO_EINVAL, "NULL argument");
  if (n < 0 || n > 0x7fffffffLL - kMlpTile) return mfail(m, DPO_EINVAL, "n out of range");
  if (!aligned16(x)) return mfail(m, DPO_EINVAL, "x must be 16-byte aligned");
  if (n == 0) return DPO_OK;
  MlpArgs a = mlp_args(m, x, nullptr, nullptr, (int)n);
  a.y = y;
  MLP_HIP(m, after_previous(m, MS(stream)));
  MLP_HIP(m, launch_mlp_forward(a, MS(stream)));
  MLP_HIP(m, mark_done(m, MS(stream)));
  return DPO_OK;
}

int dpo_mlp_grad(dpo_mlp* m, const float* x, const float* tgt, int64_t n, float* grad, float* loss, void* stream) {
  if (!m || !x || !tgt) return mfail(m, DPO_EINVAL, "NULL argument");
  if (n < 1 || n > kMaxBatch) return mfail(m, DPO_EINVAL, "n must be in [1, 65536]");
  if (!aligned16(x) || !aligned16(tgt)) return mfail(m, DPO_EINVAL, "x and tgt must be 16-byte aligned");
  const int tiles = mlp_tiles((int)n);
  int rc = ensure_partial(m, tiles);
  if (rc != DPO_OK) return rc;
  MlpArgs a = mlp_args(m, x, tgt, nullptr, (int)n);
  a.partial = m->partial;
  MLP_HIP(m, after_previous(m, MS(stream)));
  MLP_HIP(m, launch_mlp_grad(a, MS(stream)));
  ReduceArgs r = reduce_args(m, tiles, (int)n, loss ? loss : m->loss, 0);
  MLP_HIP(m, launch_mlp_reduce(r, MS(stream)));
  if (grad)
    MLP_HIP(m, hipMemcpyAsync(grad, m->grad, (size_t)kNParam * sizeof(float), hipMemcpyDeviceToDevice, MS(stream)));
  MLP_HIP(m, mark_done(m, MS(stream)));
  return DPO_OK;
}

int dpo_mlp_train(dpo_mlp* m, const float* x, const float* tgt, int64_t n, const int32_t* perm, int32_t batch,
                  float* loss_hist, void* stream) {
  if (!m || !x || !tgt) return mfail(m, DPO_EINVAL, "NULL argument");
  if (n < 1 || n > 0x7fffffffLL - kMlpTile) return mfail(m, DPO_EINVAL, "n out of range");
  if (batch < 1 || batch > kMaxBatch) return mfail(m, DPO_EINVAL, "batch must be in [1, 65536]");
  if (!aligned16(x) || !aligned16(tgt)) return mfail(m, DPO_EINVAL, "x and tgt must be 16-byte aligned");
  const int64_t steps = (n + batch - 1) / batch;
  int rc = ensure_partial(m, mlp_tiles(batch));
  if (rc != DPO_OK) return rc;
  const int* dperm = nullptr;
  if (perm) {
    for (int64_t t = 0; t < n; t++)
      if (perm[t] < 0 || perm[t] >= n) return mfail(m, DPO_EINVAL, "perm entries must lie in [0, n)");
    rc = ensure_perm(m, n);
    if (rc != DPO_OK) return rc;
    // Stage the order in pinned memory so that the upload is asynchronous and
    // the caller may prepare the next epoch's order while this one trains.
    // The previous call's upload must have left the staging buffer first.  The
    // new upload waits for the previous call's steps (on whatever stream they
    // were queued), which read the device copy it overwrites.
    MLP_HIP(m, hipEventSynchronize(m->perm_copied));
    std::memcpy(m->perm_host, perm, (size_t)n * sizeof(int));
    MLP_HIP(m, after_previous(m, MS(stream)));
    MLP_HIP(m, hipMemcpyAsync(m->perm, m->perm_host, (size_t)n * sizeof(int), hipMemcpyHostToDevice, MS(stream)));
    MLP_HIP(m, hipEventRecord(m->perm_copied, MS(stream)));
    dperm = m->perm;
  } else {
    MLP_HIP(m, after_previous(m, MS(stream)));
  }
  for (int64_t b = 0; b < steps; b++) {
    const int64_t lo = b * batch;
    const int nb = (int)std::min<int64_t>(batch, n - lo);
    MlpArgs a = mlp_args(m, x, tgt, nullptr, nb);
    if (dperm) {
      a.perm = dperm + lo;
    } else {
      a.x = reinterpret_cast<const float4*>(x) + lo;
      a.tgt = reinterpret_cast<const float4*>(tgt) + lo;
    }
    MLP_HIP(m, launch_mlp_grad(a, MS(stream)));
    m->step++;
    ReduceArgs r = reduce_args(m, mlp_tiles(nb), nb, loss_hist ? loss_hist + b : m->loss, 1);
    r.c1 = (float)(1.0 / (1.0 - std::pow(m->b1, (double)m->step)));
    r.c2 = (float)(1.0 / (1.0 - std::pow(m->b2, (double)m->step)));
    MLP_HIP(m, launch_mlp_reduce(r, MS(stream)));
  }
  MLP_HIP(m, mark_done(m, MS(stream)));
  return DPO_OK;
}

int dpo_mlp_propose(dpo_mlp* m, const dpo_ctx* ctx, float* seed_angle, void* stream) {
  if (!m || !ctx || !seed_angle) return mfail(m, DPO_EINVAL, "NULL argument");
  const CtxView c = ctx_view(ctx);
  if (c.n_free == 0) return DPO_OK;
  MLP_HIP(m, after_previous(m, MS(stream)));
  MLP_HIP(m, launch_mlp_propose(m->theta, m->w2, c.G, c.free_node, (int)c.n_free, seed_angle, m->max_blocks,
                                MS(stream)));
  MLP_HIP(m, mark_done(m, MS(stream)));
  return DPO_OK;
}

}  // extern "C"
