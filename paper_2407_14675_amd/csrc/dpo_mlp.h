// Internal interface of the control-proposal network: a 4 -> 128 -> 128 -> 3
// perceptron with exact (erf) GELU that maps a node's grid position, scaled
// to [-1, 1] per axis, to (cos u, sin u, throttle logit).  Its angle seeds
// the short local search of the seeded sweep (the learned counterpart of the
// paper's warm-started minimisation, Section 3, "Efficient computation of
// the minimum").
//
// Parameters live in one FP32 array in the order W1[128][4], b1[128],
// W2[128][128], b2[128], W3[3][128], b3[3] (row = output unit).  The
// 128 x 128 layer runs on the matrix cores with bfloat16 operands and FP32
// accumulation, so W2 is also kept as bfloat16 in both [out][in] and
// [in][out] order; everything else is FP32 on the vector units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpo_device.h"

namespace dpo {

constexpr int kHid = 128;
constexpr int kOW1 = 0;
constexpr int kOB1 = kOW1 + kHid * 4;
constexpr int kOW2 = kOB1 + kHid;
constexpr int kOB2 = kOW2 + kHid * kHid;
constexpr int kOW3 = kOB2 + kHid;
constexpr int kOB3 = kOW3 + 3 * kHid;
constexpr int kNParam = kOB3 + 3;  // 17539
constexpr int kPStride = 17544;    // per-tile partial row: gradient, summed loss, padding
constexpr int kMlpTile = 64;       // samples per workgroup

// Gradient of the mean loss over one batch, one workgroup per tile of 64
// samples; each writes its partial gradient row.  Forward-only kernels use
// x, y and n.
struct MlpArgs {
  const float* theta;   // FP32 parameters
  const uint16_t* w2;   // bf16 W2 [out][in]
  const uint16_t* w2t;  // bf16 W2 [in][out]
  const float4* x;      // scaled inputs
  const float4* tgt;    // (cos u*, sin u*, thr*, unused)
  const int* perm;      // sample order, nullable
  int n;                // samples in the batch
  float inv_n;          // 1 / n
  float* y;             // forward output [n][3]
  float* partial;       // [tiles][kPStride]
};

// Tile sums -> gradient (and the batch loss), then optionally one Adam step
// on the FP32 parameters and a refresh of the bf16 copies of W2.
struct ReduceArgs {
  const float* partial;
  int tiles;
  float inv_n;
  float* grad;  // nullable
  float* loss;  // nullable: mean loss of the batch
  int update;
  float* theta;
  float* m;
  float* v;
  uint16_t* w2;
  uint16_t* w2t;
  float lr, b1, b2, eps, c1, c2;  // c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t)
};

int mlp_tiles(int n);
hipError_t launch_mlp_forward(const MlpArgs& a, hipStream_t s);
hipError_t launch_mlp_grad(const MlpArgs& a, hipStream_t s);
hipError_t launch_mlp_reduce(const ReduceArgs& a, hipStream_t s);
hipError_t launch_mlp_cast(const float* theta, uint16_t* w2, uint16_t* w2t, hipStream_t s);
// Proposed thrust angle atan2(sin, cos) at every listed node (packed
// coordinates), written to seed[flat index]; persistent workgroups.
hipError_t launch_mlp_propose(const float* theta, const uint16_t* w2, const Grid& G, const uint32_t* nodes, int n,
                              float* seed, int max_blocks, hipStream_t s);
// flag[j] = 0 where node j is free and V[j] < thresh, else 1 (input of the
// ordered compaction).
hipError_t launch_feasible_flags(const uint8_t* kind, const float* V, float thresh, uint8_t* flag, int N,
                                 hipStream_t s);
// Training pairs: scaled position and (cos, sin, throttle) of the policy at
// nodes[sel[t]].
hipError_t launch_gather_pairs(const Grid& G, const uint32_t* nodes, const int* sel, int n, const float* ang,
                               const uint8_t* thr, float4* x, float4* tgt, hipStream_t s);

}  // namespace dpo

struct dpo_ctx;
namespace dpo {
// Read-only view of a context for the network entry points.
struct CtxView {
  Grid G;
  const uint32_t* free_node;
  int64_t n_free;
  int64_t N;
  const uint8_t* kind;
};
CtxView ctx_view(const dpo_ctx* c);
}  // namespace dpo
