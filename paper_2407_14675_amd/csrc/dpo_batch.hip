// Batched solve: many transfer problems (different grids, thrust levels and
// targets) swept by one kernel launch per sweep, value iteration per problem
// (arXiv 2407.14675, Section 3, "Policy Iteration", first display), with a
// per-problem FP64 residual and stop flag so converged problems drop out.
// The host captures S sweeps into one hipGraph and replays it until every
// problem has stopped.
#include "dpo_search.h"

namespace dpo {

// One workgroup per tile of the running problems (numbered problem by
// problem, XCD-contiguous); the problem's record holds offsets into the
// concatenated buffers, whose bases are kernel arguments.  The tile's problem
// is one table lookup, so a workgroup's set-up waits on two dependent loads
// (table entry, then record) whatever the number of running problems.
template <int kMode>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_sweep(BatchArgs B, int parity, int want_resid) {
  extern __shared__ float4 dyn_lds[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const BatchProblem& R = B.probs[B.tile_run[tile]];
  SweepArgs a;
  a.G = R.G;
  a.P = R.P;
  a.V_in = (parity ? B.Vb : B.Va) + R.v_off;
  a.V_out = (parity ? B.Va : B.Vb) + R.v_off;
  a.pol_ang = B.ang_all ? B.ang_all + R.v_off : nullptr;
  a.pol_thr = B.thr_all ? B.thr_all + R.v_off : nullptr;
  a.free_node = B.free_all + R.free_off;
  a.n_free = R.n_free;
  a.rinv = B.rinv_all + R.rinv_off;
  a.g1tab = B.g_all + R.g_off;
  a.g2tab = B.g_all + R.g_off + R.G.n[3];
  a.c0 = R.c0;
  a.c1 = R.c1;
  a.c2 = R.c2;
  a.gm = R.gm;
  a.tab_sin = B.tab;
  a.tab_cos = B.tab + B.n_ang;
  a.tab_ang = B.tab + 2 * B.n_ang;
  a.n_ang = B.n_ang;
  a.n_golden = B.n_golden;
  a.half_width = B.half_width;
  a.rot_scan = B.rot_scan;
  a.desc_code = nullptr;
  a.desc16 = nullptr;
  a.desc_pk = nullptr;
  a.desc_pk_in = nullptr;
  a.desc_dense = 0;
  a.seed = nullptr;
  a.pol_ang_in = nullptr;
  a.pol_thr_in = nullptr;
  a.fb_list = nullptr;
  a.fb_count = nullptr;
  a.walk_from = nullptr;
  a.eval_acc = nullptr;
  const int t = (tile - R.tile_begin) * blockDim.x + threadIdx.x;
  double rel = 0, sum = 0, mabs = 0, bad = 0;
  int fell_back = 0, deferred = 0, evals = 0;
  if (t < a.n_free) fast_node<kMode>(a, t, dyn_lds, rel, sum, mabs, bad, fell_back, deferred, evals);
  // only the last sweep of a graph replay feeds the stop decision
  if (want_resid) block_residual(rel, sum, mabs, bad, (double)fell_back, B.partial, tile);
}

// One workgroup per running problem: FP64 reduction of its tiles' partials
// (the residual of the last sweep) in a fixed order, then the stop decision.
__global__ __launch_bounds__(kBlock) void k_batch_reduce(BatchArgs B) {
  __shared__ double red[kPartial][kBlock];
  const int k = blockIdx.x;
  const int p = B.run[k];
  const int lo = B.tile_begin[k], hi = B.tile_begin[k + 1];
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
    if (red[3][0] > 0) B.done[p] = 2;
    else if (red[0][0] < B.tol) B.done[p] = 1;
  }
}

hipError_t launch_batch_sweep(const BatchArgs& b, int mode, int block, int parity, int want_resid, hipStream_t s) {
  const size_t lds = sizeof(float4) * 4 * block;
  if (mode == 0) hipLaunchKernelGGL(k_batch_sweep<0>, dim3(b.n_tiles), dim3(block), lds, s, b, parity, want_resid);
  else hipLaunchKernelGGL(k_batch_sweep<1>, dim3(b.n_tiles), dim3(block), lds, s, b, parity, want_resid);
  return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchArgs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reduce, dim3(b.n_run), dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

}  // namespace dpo
