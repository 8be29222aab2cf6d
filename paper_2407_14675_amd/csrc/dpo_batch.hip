// Batched solve: many transfer problems (different grids, thrust levels and
// targets) swept by one kernel launch per sweep, value iteration per problem
// (arXiv 2407.14675, Section 3, "Policy Iteration", first display), with a
// per-problem FP64 residual and stop flag so converged problems drop out.
// The host captures S sweeps into one hipGraph and replays it until every
// problem has stopped.
#include "dpo_search.h"

namespace dpo {

// Workgroup -> (problem, tile): tiles are numbered problem by problem; the
// XCD remap keeps each XCD on a contiguous run of tiles.
template <int kMode>
__global__ __launch_bounds__(kMaxBlock) void k_batch_sweep(BatchArgs B, int parity) {
  extern __shared__ float4 dyn_lds[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  int p = 0;
  while (p + 1 < B.n_prob && B.tile_begin[p + 1] <= tile) p++;
  if (B.done[p]) return;  // whole workgroup: its problem has stopped
  SweepArgs a = B.probs[p].a;
  if (parity) {
    float* tmp = const_cast<float*>(a.V_in);
    a.V_in = a.V_out;
    a.V_out = tmp;
  }
  const int t = (tile - B.tile_begin[p]) * blockDim.x + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  int fell_back = 0;
  if (t < a.n_free) fast_node<kMode>(a, t, dyn_lds, rel, sum, mabs, bad, fell_back);
  block_residual(rel, sum, mabs, bad, (double)fell_back, B.partial, tile);
}

// One workgroup per problem: FP64 reduction of its tiles' partials in a
// fixed order, then the stop decision.
__global__ __launch_bounds__(kBlock) void k_batch_reduce(BatchArgs B, int parity) {
  __shared__ double red[kPartial][kBlock];
  const int p = blockIdx.x;
  if (B.done[p]) return;
  const int lo = B.tile_begin[p], hi = B.tile_begin[p + 1];
  double acc[kPartial] = {0, 0, 0, 0, 0};
  for (int i = lo + (int)threadIdx.x; i < hi; i += kBlock) {
    acc[0] = fmax(acc[0], B.partial[kPartial * i + 0]);
    acc[1] += B.partial[kPartial * i + 1];
    acc[2] = fmax(acc[2], B.partial[kPartial * i + 2]);
    acc[3] += B.partial[kPartial * i + 3];
    acc[4] += B.partial[kPartial * i + 4];
  }
  for (int q = 0; q < kPartial; q++) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int s = kBlock / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + s]);
      red[3][threadIdx.x] += red[3][threadIdx.x + s];
      red[4][threadIdx.x] += red[4][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int q = 0; q < kPartial; q++) B.resid[kPartial * p + q] = red[q][0];
    B.sweeps[p] += 1;
    if (red[3][0] > 0) {
      B.done[p] = 2;
      B.done_buf[p] = parity ^ 1;
    } else if (red[0][0] < B.tol) {
      B.done[p] = 1;
      B.done_buf[p] = parity ^ 1;
    }
  }
}

hipError_t launch_batch_sweep(const BatchArgs& b, int mode, int block, int n_tiles, int parity, hipStream_t s) {
  const size_t lds = sizeof(float4) * 4 * block;
  if (mode == 0) hipLaunchKernelGGL(k_batch_sweep<0>, dim3(n_tiles), dim3(block), lds, s, b, parity);
  else hipLaunchKernelGGL(k_batch_sweep<1>, dim3(n_tiles), dim3(block), lds, s, b, parity);
  return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchArgs& b, int parity, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reduce, dim3(b.n_prob), dim3(kBlock), 0, s, b, parity);
  return hipGetLastError();
}

}  // namespace dpo
