// Internal interface between the host library and the HIP kernels of libdpo.
#pragma once

#include "dpo_device.h"

namespace dpo {

struct TargetBox {
  double c[4], w[4];
};

// Everything a node kernel needs, passed by value as the kernel argument.
struct SweepArgs {
  Grid G;
  Phys P;
  const float* V_in;
  float* V_out;
  float* pol_ang;             // out, nullable
  uint8_t* pol_thr;           // out, nullable
  const float* pol_ang_in;    // frozen policy (evaluation sweep); greedy sweeps: incumbent, nullable
  const uint8_t* pol_thr_in;  // frozen policy (evaluation sweep); greedy sweeps: incumbent, nullable
  const float* seed;          // seeded search
  const float* walk_from;     // table walk: each node's previous angle (may alias pol_ang)
  unsigned long long* eval_acc;  // table walk: per-workgroup running count of thrust evaluations, nullable
  int* fb_list;               // seeded search on the factorised path: nodes whose full search is deferred, nullable
  int* fb_count;              // their count (zeroed before the sweep)
  const uint32_t* free_node;  // packed coordinates (8 bits per axis, r lowest) of the free nodes
  int n_free;
  // per-axis / per-plane tables (FP64 1/r; thrust displacement per unit sin/cos per mass plane)
  const double* rinv;
  const float* g1tab;
  const float* g2tab;
  double c0, c1, c2, c3;  // dt / h_k for axes r, v_r, v_t and axis 3
  const float* qnode;     // crown problem: dt times the orbital-element running cost per node, nullable
  float gm;           // thrust displacement along m (cells)
  const float* tab_sin;  // tabulated controls (TABLE) or scan samples (SCAN_GOLDEN)
  const float* tab_cos;
  const float* tab_ang;
  int n_ang;
  int n_golden;
  float half_width;  // golden bracket half width, 2*pi/n_scan
  const float* rot_scan;   // golden-section rotation constants for half_width (see golden())
  const float* rot_local;  // the same for local_half_width
  int n_local;
  float local_half_width;
  float fallback_tol;
  double* partial;  // kPartial doubles per workgroup; null: the sweep skips the residual
  // Foot descriptor of each free node's chosen control (free-list order),
  // written by the greedy sweep when desc_code is set and read by the
  // frozen-policy sweep.  desc_code: bits 0-29 flat index of the cell's lowest
  // corner, bit 30 foot outside the domain, bit 31 throttle.  desc_w: the
  // cell coordinates along v_r and v_t; those along r and m follow from the
  // node and the throttle and are recomputed bit-identically.
  int* desc_code;
  float2* desc_w;
  const int* desc_code_in;
  const float2* desc_w_in;
  // Compact form used when every foot lies within 31 cells of its node along
  // v_r and v_t: a 16-bit code with the cell's offset from the node along v_r
  // (bits 0-5) and v_t (bits 6-11), each plus 32, bit 12 foot outside, bit
  // 13 throttle.  Indexed by free-list position, or by node (desc_dense: the
  // sweep then runs over every node and skips the code kDescSkip).
  uint16_t* desc16;
  const uint16_t* desc16_in;
  // Packed form, stored per node (desc_dense): the 14 low bits of the compact
  // code (kDescPkSkip for a node that is not free), then the two cell
  // coordinates as 25-bit fixed-point numbers in units of 2^-24 of a cell
  // (see desc_pack).
  uint2* desc_pk;
  const uint2* desc_pk_in;
  int desc_dense;
  int mode;         // search mode (feedback)
  double w_time, w_fuel, lambda;
};

inline int blocks_for(long long n, int per = kBlock) { return (int)((n + per - 1) / per); }

constexpr uint16_t kDescOut = 1u << 12;
constexpr uint16_t kDescThr = 1u << 13;
constexpr uint16_t kDescSkip = 0xffffu;  // not a free node (dense form)
constexpr uint32_t kDescPkSkip = 0x3fffu;  // not a free node (packed form; no code of a free node has it)

// Packed descriptor of one node: code (14 bits), then the cell coordinates w1
// and w2 in [0, 1] rounded to the nearest multiple of 2^-24 (25 bits each:
// exact for coordinates in [0.5, 1], within 2^-25 of a cell below that, which
// is half a float32 unit at 0.25-0.5).  Eight bytes per node instead of ten.
__device__ inline uint2 desc_pack(uint32_t code, float w1, float w2) {
  const uint32_t q1 = (uint32_t)rintf(fminf(fmaxf(w1, 0.0f), 1.0f) * 16777216.0f);
  const uint32_t q2 = (uint32_t)rintf(fminf(fmaxf(w2, 0.0f), 1.0f) * 16777216.0f);
  return make_uint2(code | (q1 << 14), (q1 >> 18) | (q2 << 7));
}
__device__ inline uint32_t desc_pk_code(uint2 d) { return d.x & kDescPkSkip; }
__device__ inline float desc_pk_w1(uint2 d) {
  return (float)(__builtin_amdgcn_alignbit(d.y, d.x, 14) & 0x1ffffffu) * 5.9604644775390625e-8f;
}
__device__ inline float desc_pk_w2(uint2 d) { return (float)(d.y >> 7) * 5.9604644775390625e-8f; }
// Feedback and closed loop: up to this many states one wave per state (the
// lanes split the table), beyond it one thread per state.
constexpr int kWaveStates = 8192;
constexpr int kResidStage = 256;          // workgroups of the first stage of the residual reduction
constexpr int kDescReach = 31;           // largest cell offset the compact code holds

// Per-problem record of the batched sweep (device table).  It holds no
// pointers: every array of the batch is one concatenated allocation passed
// as a kernel argument, and the record gives this problem's offsets into it.
struct BatchProblem {
  Grid G;
  Phys P;
  double c0, c1, c2;
  float gm;
  int n_free;
  long long v_off;  // offset of node 0 in the value / policy arrays
  int free_off;     // offset in the concatenated free-node list
  int rinv_off;     // offset in the concatenated 1/r table
  int g_off;        // offset in the concatenated thrust tables ([2][n_m] per problem)
  int tile_begin;   // first tile of this problem
};

struct BatchArgs {
  const BatchProblem* probs;  // records of the running problems, in run order (n_run entries)
  const int* run;             // problem number of each running problem (n_run entries)
  const int* tile_begin;      // first tile of each running problem (n_run + 1 entries)
  const int* tile_run;        // running problem of each tile (n_tiles entries)
  int n_run;
  int n_tiles;
  const uint32_t* free_all;
  const double* rinv_all;
  const float* g_all;
  float* Va;  // value buffer A (concatenated)
  float* Vb;  // value buffer B
  float* ang_all;
  uint8_t* thr_all;
  const float* tab;  // shared search table [3][n_ang]
  int n_ang;
  int n_golden;
  float half_width;
  const float* rot_scan;
  int* done;      // per problem: 0 running, 1 converged, 2 non-finite values
  double* partial;
  double* resid;  // kPartial per problem
  double tol;
};

hipError_t launch_batch_sweep(const BatchArgs& b, int mode, int block, int parity, int want_resid, hipStream_t s);
hipError_t launch_batch_reduce(const BatchArgs& b, hipStream_t s);

// Launch wrappers (asynchronous on `stream`); each returns the launch status.
hipError_t launch_classify(const Grid& G, const TargetBox& tb, const uint8_t* mask, uint8_t* kind, int N,
                           hipStream_t s);
int compact_chunks(int N);
hipError_t launch_compact(const Grid& G, const uint8_t* kind, int N, int* counts, int* offsets,
                          uint32_t* free_node, hipStream_t s);
hipError_t launch_init_value(const uint8_t* kind, float M, float* V, int N, hipStream_t s);
// Direct-path sweep; mode 0 table, 1 scan + golden, 2 seeded, 3 table walk
// (the integrator comes from a.P.heun).
hipError_t launch_sweep_direct(const SweepArgs& a, int mode, hipStream_t s);
hipError_t launch_policy_eval(const SweepArgs& a, bool want_resid, hipStream_t s);
// crown problem: qnode[j] = dt * running cost at node j (FP64, rounded)
hipError_t launch_node_cost(const Grid& G, const Phys& P, float* qnode, int N, hipStream_t s);
// out[0] = sum of acc[0..n) (fixed order, one workgroup)
hipError_t launch_sum_counts(const unsigned long long* acc, int n, unsigned long long* out, hipStream_t s);
hipError_t launch_policy_eval_desc(const SweepArgs& a, bool streamed, hipStream_t s);
// format 1: compact codes by free-list position; 2: compact codes by node
hipError_t launch_policy_eval_desc16(const SweepArgs& a, int format, bool streamed, hipStream_t s);
hipError_t launch_zero_count(int* count, hipStream_t s);
hipError_t launch_sweep_fallback(const SweepArgs& a, int block, int blocks, hipStream_t s);
hipError_t launch_sweep_fast(const SweepArgs& a, int mode, int block, hipStream_t s);
// Final FP64 reduction of nblocks residual partials into out[kPartial];
// `stage` holds kResidStage * kPartial doubles for the first of two stages.
hipError_t launch_resid_final(const double* partial, int nblocks, double* stage, double* out, hipStream_t s);
hipError_t launch_value_at(const float* V, const Grid& G, double M, const double x[4], double* out,
                           hipStream_t s);
hipError_t launch_feedback(const SweepArgs& a, const double* states, int n, double tau, float* ang,
                           uint8_t* thr, float* q, hipStream_t s);
hipError_t launch_simulate(const SweepArgs& a, double* states, int n, double tau, int steps, int substeps,
                           double drag, double* traj, uint8_t* thr_hist, float* ang_hist, hipStream_t s);
hipError_t launch_mask_seed(const float* Vc, const Grid& Gc, double M, const Grid& Gf, double thresh,
                            uint8_t* seed, int Nf, hipStream_t s);
hipError_t launch_dilate_axis(const uint8_t* in, uint8_t* out, const Grid& G, int axis, int d, int N,
                              hipStream_t s);
hipError_t launch_probe_interp(const float* V, const Grid& G, float M, const float* pts, int n,
                               float* out, hipStream_t s);
hipError_t launch_probe_q(const SweepArgs& a, const int* nodes, const uint8_t* thr, const float* ang,
                          int n, float* q_out, float* off_out, hipStream_t s);

// Frozen-policy sweep over a dense grid with value bricks in LDS
// (dpo_brick.hip).  A workgroup of kBrickBlock threads owns every r of a
// tile of tr v_r rows and tt v_t rows and walks `planes` mass planes upwards;
// its LDS holds two planes of the brick its feet can reach: the tile plus,
// per tile, halo.x rows below and halo.y above along v_r, halo.z below and
// halo.w above along v_t (the reach of the feet of that tile's nodes).
constexpr int kBrickBlock = 512;
constexpr int kBrickMaxPf = 4;  // 16-byte loads per thread for one plane's brick, at most
constexpr int kBrickNodes = 6;  // nodes of one plane of a tile per thread, at most
constexpr int kBrickMaxRows = 32;  // v_r rows of a tile, at most
struct BrickPlan {
  int tr, tt, planes;
  int n_at, n_ct, n_mc;  // tiles along v_r, v_t, mass chunks (workgroups = their product)
  int slot;              // floats of one plane slot: the largest brick's rows times n0
  const int4* halo;      // device, n_at * n_ct entries (tile at + n_at * ct)
};
size_t brick_lds_bytes(const BrickPlan& B);
hipError_t launch_eval_brick(const SweepArgs& a, const BrickPlan& B, const uint8_t* kind, bool want_resid,
                             bool streamed, hipStream_t s);
// the same sweep driven by the dense per-node foot descriptors of the
// greedy step (SweepArgs::desc16_in / desc_w_in, desc_dense)
hipError_t launch_eval_brick_desc(const SweepArgs& a, const BrickPlan& B, bool streamed, hipStream_t s);
hipError_t prepare_eval_brick(const BrickPlan& B);

// Machine ceilings (dpo_ceiling.hip): a float4 streaming copy and read of n
// floats (n a multiple of 4, 16-byte aligned) and a plain FP32 FMA loop of
// blocks x 256 threads, each issuing iters x 8 FMAs.
hipError_t launch_ceil_copy(const float* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_ceil_read(const float* src, int64_t n, float* sink, hipStream_t s);
hipError_t launch_ceil_fma(int blocks, int iters, float* sink, hipStream_t s);

}  // namespace dpo
