// Kernels of the exact policy evaluation (paper Section 3: eq:p_eval is a
// sparse linear system, v - exp(-lambda dt) P v = b, solved by GMRES).
// Vectors are full-grid float arrays that are zero at fixed nodes; the
// operator is applied matrix-free by the frozen-policy sweep without its
// affine part (no running cost, a foot outside contributes 0 instead of M,
// fixed corners read the zeros), and the dot products of the Gram-Schmidt
// steps are accumulated in FP64 per workgroup and reduced in a fixed order.
#include <hip/hip_runtime.h>

#include "dpo_krylov.h"
#include "dpo_search.h"

namespace dpo {

// y_j = exp(-lambda dt) * I[x](foot of node j under its frozen control), at
// free nodes; fixed entries of y are not written.
template <bool kHeun>
__global__ __launch_bounds__(kBlock) void k_eval_hom(SweepArgs a, const float* __restrict__ x, float* __restrict__ y) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int t = tile * kBlock + threadIdx.x;
  if (t >= a.n_free) return;
  NodeTerms T;
  const int j = node_terms_tab(a, a.free_node[t], T);
  HeunTerms H;
  if (kHeun) {
    double xs[4];
    for (int k = 0; k < 4; k++) xs[k] = a.G.lo[k] + (double)T.i[k] * a.G.h[k];
    heun_terms(a.G, a.P, xs, a.P.dt, H);
  }
  const int thr = a.pol_thr_in[j] ? 1 : 0;
  float sn = 0.0f, cs = 1.0f;
  if (thr) policy_sincos(a, a.pol_ang_in[j], sn, cs);
  float off[4];
  foot_off<kHeun>(T, H, thr, sn, cs, off);
  int base[4];
  float tt[4];
  float v = 0.0f;
  if (foot_cell(a.G, T.i, off, base, tt)) {
    const int s3 = (a.G.periodic3 && base[3] == a.G.n[3] - 1) ? -base[3] * a.G.st[3] : a.G.st[3];
    v = a.P.gamma * cell_value(x + (base[0] + base[1] * a.G.st[1] + base[2] * a.G.st[2] + base[3] * a.G.st[3]),
                               a.G, tt, s3);
  }
  y[j] = v;
}

// r = b - x + y  (with y = gamma P x: the residual b - A x)
__global__ __launch_bounds__(kBlock) void k_residual(const float* __restrict__ b, const float* __restrict__ x,
                                                     const float* __restrict__ y, float* __restrict__ r, int N) {
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < N; j += gridDim.x * kBlock) r[j] = (b[j] - x[j]) + y[j];
}

// w = v - y (A v, with y = gamma P v) and, in the same pass, the partial dot
// products of the new w with the first k <= kDotGroup basis vectors (the
// layout of k_dots): the Gram-Schmidt coefficients of w without a second
// read of it.
__global__ __launch_bounds__(kBlock) void k_sub_dots(const float* __restrict__ v, const float* __restrict__ y,
                                                     float* __restrict__ w, const float* __restrict__ basis, int k,
                                                     size_t ld, int N, double* __restrict__ partial) {
  double acc[kDotGroup];
#pragma unroll
  for (int i = 0; i < kDotGroup; i++) acc[i] = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < N; j += gridDim.x * kBlock) {
    const float nw = v[j] - y[j];
    w[j] = nw;
    const double wj = (double)nw;
#pragma unroll
    for (int i = 0; i < kDotGroup; i++)
      if (i < k) acc[i] += (double)basis[(size_t)i * ld + j] * wj;
  }
  __shared__ double red[kBlock / 64][kDotGroup];
#pragma unroll
  for (int i = 0; i < kDotGroup; i++) {
    double a = acc[i];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][i] = a;
  }
  __syncthreads();
  if (threadIdx.x < kDotGroup) {
    double t = 0.0;
    for (int q = 0; q < kBlock / 64; q++) t += red[q][threadIdx.x];
    partial[(size_t)blockIdx.x * kDotGroup + threadIdx.x] = t;
  }
}

// Partial dot products of w with up to kDotGroup basis vectors (rows of
// `basis`, leading dimension ld): partial[blockIdx.x * kDotGroup + i].
__global__ __launch_bounds__(kBlock) void k_dots(const float* __restrict__ basis, int k, size_t ld,
                                                 const float* __restrict__ w, int N, double* __restrict__ partial) {
  double acc[kDotGroup];
#pragma unroll
  for (int i = 0; i < kDotGroup; i++) acc[i] = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < N; j += gridDim.x * kBlock) {
    const double wj = (double)w[j];
#pragma unroll
    for (int i = 0; i < kDotGroup; i++)
      if (i < k) acc[i] += (double)basis[(size_t)i * ld + j] * wj;
  }
  __shared__ double red[kBlock / 64][kDotGroup];
#pragma unroll
  for (int i = 0; i < kDotGroup; i++) {
    double v = acc[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < kDotGroup) {
    double s = 0.0;
    for (int q = 0; q < kBlock / 64; q++) s += red[q][threadIdx.x];
    partial[(size_t)blockIdx.x * kDotGroup + threadIdx.x] = s;
  }
}

// Per-workgroup max of |r_j| / max(1, |x_j|) (the node-wise relative
// residual, the library's stop measure): partial[blockIdx.x].
__global__ __launch_bounds__(kBlock) void k_relmax(const float* __restrict__ r, const float* __restrict__ x, int N,
                                                   double* __restrict__ partial) {
  double m = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < N; j += gridDim.x * kBlock) {
    const double v = fabs((double)r[j]) / fmax(1.0, fabs((double)x[j]));
    m = (v > m || v != v) ? v : m;  // a NaN propagates
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double u = __shfl_xor(m, o, 64);
    m = (u > m || u != u) ? u : m;
  }
  __shared__ double red[kBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kBlock / 64; q++) s = (red[q] > s || red[q] != red[q]) ? red[q] : s;
    partial[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_relmax_final(const double* __restrict__ partial, int nblocks,
                                                         double* __restrict__ out) {
  __shared__ double red[kBlock];
  double m = 0.0;
  for (int q = threadIdx.x; q < nblocks; q += kBlock) m = (partial[q] > m || partial[q] != partial[q]) ? partial[q] : m;
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double u = red[threadIdx.x + w];
      if (u > red[threadIdx.x] || u != u) red[threadIdx.x] = u;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// out[i] = sum over blocks of partial[b * kDotGroup + i], fixed order; one
// workgroup per output.
__global__ __launch_bounds__(kBlock) void k_dots_final(const double* __restrict__ partial, int nblocks,
                                                       double* __restrict__ out) {
  __shared__ double red[kBlock];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int q = threadIdx.x; q < nblocks; q += kBlock) s += partial[(size_t)q * kDotGroup + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// w -= sum_i coef[i] * basis_i  (k <= kMaxBasis terms, FP64 sum per element);
// with nrm_partial, also the FP64 sum of squares of the new w per workgroup
// (nrm_partial[blockIdx.x * kDotGroup], the layout k_dots_final reads).
__global__ __launch_bounds__(kBlock) void k_axpys(float* __restrict__ w, const float* __restrict__ basis, int k,
                                                  size_t ld, const double* __restrict__ coef, int N,
                                                  double* __restrict__ nrm_partial) {
  __shared__ double c[kMaxBasis];
  __shared__ double red[kBlock / 64];
  for (int i = threadIdx.x; i < k; i += kBlock) c[i] = coef[i];
  __syncthreads();
  double acc = 0.0;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < N; j += gridDim.x * kBlock) {
    double s = 0.0;
    for (int i = 0; i < k; i++) s += c[i] * (double)basis[(size_t)i * ld + j];
    const float nw = (float)((double)w[j] - s);
    w[j] = nw;
    acc += (double)nw * (double)nw;
  }
  if (!nrm_partial) return;  // uniform over the workgroup
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kBlock / 64; q++) t += red[q];
    nrm_partial[(size_t)blockIdx.x * kDotGroup] = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_scale(const float* __restrict__ src, double s, float* __restrict__ dst,
                                                  int N) {
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < N; j += gridDim.x * kBlock) dst[j] = (float)((double)src[j] * s);
}

// dst = src * (*sc), the factor read from device memory.
__global__ __launch_bounds__(kBlock) void k_scale_dev(const float* __restrict__ src, const double* __restrict__ sc,
                                                      float* __restrict__ dst, int N) {
  const double s = *sc;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < N; j += gridDim.x * kBlock) dst[j] = (float)((double)src[j] * s);
}

// Column k of the Arnoldi process, on the device (one thread, FP64): the
// Hessenberg entries h_ik = d_i (the classical Gram-Schmidt coefficients)
// for i <= k and h_(k+1)k = sqrt(*nrm2) (the norm of the new basis vector
// before scaling), the earlier Givens rotations applied to the column, a new
// one zeroing h_(k+1)k, and the rotated right-hand side g.
// H is (m + 1) x m, row-major.  Writes *inv_hn = 1/h_(k+1)k (0 at a
// breakdown) for the scaling of the new vector, and status = (|g_(k+1)|,
// h_(k+1)k) for the host's stop test.
__global__ void k_arnoldi_col(int k, int m, const double* __restrict__ d, const double* __restrict__ nrm2,
                              double* __restrict__ H, double* __restrict__ cs,
                              double* __restrict__ sn, double* __restrict__ g, double* __restrict__ inv_hn,
                              double* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double hn = sqrt(fmax(nrm2[0], 0.0));
  for (int i = 0; i <= k; i++) H[(size_t)i * m + k] = d[i];
  H[(size_t)(k + 1) * m + k] = hn;
  for (int i = 0; i < k; i++) {
    const double t0 = H[(size_t)i * m + k], t1 = H[(size_t)(i + 1) * m + k];
    H[(size_t)i * m + k] = cs[i] * t0 + sn[i] * t1;
    H[(size_t)(i + 1) * m + k] = -sn[i] * t0 + cs[i] * t1;
  }
  const double a = H[(size_t)k * m + k], b = H[(size_t)(k + 1) * m + k];
  const double den = hypot(a, b);
  cs[k] = den > 0 ? a / den : 1.0;
  sn[k] = den > 0 ? b / den : 0.0;
  H[(size_t)k * m + k] = den;
  H[(size_t)(k + 1) * m + k] = 0.0;
  g[k + 1] = -sn[k] * g[k];
  g[k] = cs[k] * g[k];
  inv_hn[0] = hn > 0 ? 1.0 / hn : 0.0;
  status[0] = fabs(g[k + 1]);
  status[1] = hn;
}

// dst[j] = src[j] at the free nodes j; fixed entries untouched.
__global__ __launch_bounds__(kBlock) void k_free_copy(const uint32_t* __restrict__ free_node, int n_free, Grid G,
                                                      const float* __restrict__ src, float* __restrict__ dst) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n_free) return;
  int i[4];
  const int j = unpack_node(G, free_node[t], i);
  dst[j] = src[j];
}

// dst[j] = 0 at the free nodes j (the affine part's argument: V with its free
// entries zeroed).
__global__ __launch_bounds__(kBlock) void k_free_zero(const uint32_t* __restrict__ free_node, int n_free, Grid G,
                                                      float* __restrict__ dst) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n_free) return;
  int i[4];
  dst[unpack_node(G, free_node[t], i)] = 0.0f;
}

// ------------------------------------------------------------ launchers
namespace {
int stream_blocks(int N) { return std::min(blocks_for(N), kStreamBlocks); }
}  // namespace

hipError_t launch_eval_hom(const SweepArgs& a, const float* x, float* y, hipStream_t s) {
  if (a.n_free == 0) return hipSuccess;
  if (a.P.heun) hipLaunchKernelGGL(k_eval_hom<true>, dim3(blocks_for(a.n_free)), dim3(kBlock), 0, s, a, x, y);
  else hipLaunchKernelGGL(k_eval_hom<false>, dim3(blocks_for(a.n_free)), dim3(kBlock), 0, s, a, x, y);
  return hipGetLastError();
}

hipError_t launch_residual(const float* b, const float* x, const float* y, float* r, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(stream_blocks(N)), dim3(kBlock), 0, s, b, x, y, r, N);
  return hipGetLastError();
}

hipError_t launch_sub_dots(const float* v, const float* y, float* w, const float* basis, int k, size_t ld, int N,
                           double* partial, double* out, hipStream_t s) {
  if (k > kDotGroup) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sub_dots, dim3(kStreamBlocks), dim3(kBlock), 0, s, v, y, w, basis, k, ld, N, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dots_final, dim3(k), dim3(kBlock), 0, s, partial, kStreamBlocks, out);
  return hipGetLastError();
}

hipError_t launch_dots(const float* basis, int k, size_t ld, const float* w, int N, double* partial, double* out,
                       hipStream_t s) {
  for (int g = 0; g < k; g += kDotGroup) {
    const int kg = std::min(kDotGroup, k - g);
    hipLaunchKernelGGL(k_dots, dim3(kStreamBlocks), dim3(kBlock), 0, s, basis + (size_t)g * ld, kg, ld, w, N, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dots_final, dim3(kg), dim3(kBlock), 0, s, partial, kStreamBlocks, out + g);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_relmax(const float* r, const float* x, int N, double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_relmax, dim3(kStreamBlocks), dim3(kBlock), 0, s, r, x, N, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_relmax_final, dim3(1), dim3(kBlock), 0, s, partial, kStreamBlocks, out);
  return hipGetLastError();
}

hipError_t launch_axpys(float* w, const float* basis, int k, size_t ld, const double* coef, int N, hipStream_t s,
                       double* partial, double* nrm_out) {
  const int nb = stream_blocks(N);
  hipLaunchKernelGGL(k_axpys, dim3(nb), dim3(kBlock), 0, s, w, basis, k, ld, coef, N, nrm_out ? partial : nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !nrm_out) return e;
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(kBlock), 0, s, partial, nb, nrm_out);
  return hipGetLastError();
}

hipError_t launch_scale(const float* src, double sc, float* dst, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(stream_blocks(N)), dim3(kBlock), 0, s, src, sc, dst, N);
  return hipGetLastError();
}

hipError_t launch_scale_dev(const float* src, const double* sc, float* dst, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_dev, dim3(stream_blocks(N)), dim3(kBlock), 0, s, src, sc, dst, N);
  return hipGetLastError();
}

hipError_t launch_arnoldi_col(int k, int m, const double* d, const double* nrm2, double* H, double* cs, double* sn,
                              double* g, double* inv_hn, double* status, hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi_col, dim3(1), dim3(64), 0, s, k, m, d, nrm2, H, cs, sn, g, inv_hn, status);
  return hipGetLastError();
}

hipError_t launch_free_copy(const SweepArgs& a, const float* src, float* dst, hipStream_t s) {
  if (a.n_free == 0) return hipSuccess;
  hipLaunchKernelGGL(k_free_copy, dim3(blocks_for(a.n_free)), dim3(kBlock), 0, s, a.free_node, a.n_free, a.G, src, dst);
  return hipGetLastError();
}

hipError_t launch_free_zero(const SweepArgs& a, float* dst, hipStream_t s) {
  if (a.n_free == 0) return hipSuccess;
  hipLaunchKernelGGL(k_free_zero, dim3(blocks_for(a.n_free)), dim3(kBlock), 0, s, a.free_node, a.n_free, a.G, dst);
  return hipGetLastError();
}

}  // namespace dpo
