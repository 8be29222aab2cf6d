// Host side of libdpo: the C ABI declared in include/dpo.h.
//
// Owns the per-context device scratch (node kinds, compacted free-node list,
// control tables, residual partials, a second value buffer for the solvers)
// and runs the value- and policy-iteration loops of arXiv 2407.14675,
// Section 3 ("Policy Iteration"): sweeps are queued asynchronously and the
// host synchronises only to read the FP64 residual every few sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dpo.h"
#include "dpo_kernels.h"
#include "dpo_mlp.h"
#include "dpo_krylov.h"

using namespace dpo;

struct dpo_ctx {
  dpo_grid grid;
  dpo_problem prob;
  dpo_search search;
  Grid G;
  Phys P;
  TargetBox tb;
  int64_t N = 0, n_free = 0;
  uint8_t* kind = nullptr;
  uint32_t* free_node = nullptr;  // packed coordinates of the free nodes, node order
  double* rinv = nullptr;         // 1/r per r node (FP64)
  float* gtab = nullptr;          // [2][n_m]: thrust displacement per unit sin (v_r) / cos (v_t)
  double c0 = 0, c1 = 0, c2 = 0;  // dt/h for r, v_r, v_t
  float gm = 0;                   // thrust displacement along m
  bool fast_ok = false;           // the factorised thrust kernel applies
  int path = 0;                   // 0 auto, 1 direct, 2 fast
  BrickPlan brick{};              // frozen-policy sweep with LDS value bricks (dense grids)
  bool brick_ok = false;          // the plan applies to this problem
  int4* brick_halo = nullptr;     // its per-tile halo table
  double brick_over = 0;          // brick floats loaded per node, per plane
  int eval_path = 0;              // 0 auto, 1 free-list / descriptor kernels, 2 LDS bricks
  int block = kBlock;             // workgroup size of the factorised sweeps
  int last_blocks = 0;            // workgroups of the last kernel that wrote residual partials
  float* tab = nullptr;  // [3][n_ang]: sin, cos, angle
  float* rot = nullptr;  // [2][kRot]: golden-section rotation constants (scan bracket, local bracket)
  int n_ang = 0;
  int tab_cap = 0;
  double* partial = nullptr;
  int partial_blocks = 0;
  double* resid = nullptr;  // kPartial doubles
  float* work = nullptr;    // second value buffer of the solvers
  float* work2 = nullptr;   // third value buffer (policy iteration keeps the greedy output while evaluating ahead)
  double* resid_host = nullptr;  // pinned copy of the residual for the overlapped read-back
  int* fb_list = nullptr;         // seeded sweeps: nodes whose full search is deferred to a second pass
  int* fb_count = nullptr;
  hipEvent_t resid_ready = nullptr;
  hipEvent_t step_ev[2][4] = {};  // policy iteration: greedy start/end, evaluation start/end, two steps deep
  int* desc_code = nullptr;  // foot descriptors of the greedy step's controls (policy iteration)
  uint16_t* desc16 = nullptr;  // compact codes (desc_format 1)
  int desc_format = -1;        // 0 flat 32-bit codes, 1 compact by free node, 2 packed by node
  float2* desc_w = nullptr;    // cell coordinates (desc_format 0 and 1)
  uint2* desc_pk = nullptr;    // packed descriptors, one per node (desc_format 2)
  bool desc_valid = false;    // a sweep has written them
  float* qnode = nullptr;                  // crown problem: dt * running cost per node
  float* kry = nullptr;      // exact policy evaluation: Krylov basis, (kry_m + 1) x N
  float* kbuf = nullptr;     // its b, x, y vectors (3 x N)
  double* kpart = nullptr;   // dot-product partials
  double* kdots = nullptr;   // dot products (kMaxBasis)
  double* kcoef = nullptr;   // update coefficients (kMaxBasis)
  double* karn = nullptr;    // device Arnoldi state (see gmres_eval)
  double* karn_host = nullptr;  // pinned: each step's (|g_(k+1)|, h_(k+1)k)
  hipEvent_t karn_ev[2] = {nullptr, nullptr};
  int kry_m = 0;
  unsigned long long* eval_acc = nullptr;  // table walk: per-workgroup thrust-evaluation counts
  unsigned long long* eval_sum = nullptr;
  std::string err;
};

namespace {

thread_local std::string g_err;

int fail(dpo_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_err = msg;
  return code;
}

int hip_fail(dpo_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, DPO_EHIP, m);
}

#define HIP_TRY(ctx, call)                                         \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);       \
  } while (0)

int validate_grid(dpo_ctx* c, const dpo_grid* g) {
  if (!g) return fail(c, DPO_EINVAL, "grid is NULL");
  long long N = 1;
  for (int k = 0; k < 4; k++) {
    if (g->n[k] < 2) return fail(c, DPO_EINVAL, "grid: n[k] must be >= 2");
    if (!(g->lo[k] < g->hi[k]) || !std::isfinite(g->lo[k]) || !std::isfinite(g->hi[k]))
      return fail(c, DPO_EINVAL, "grid: need finite lo[k] < hi[k]");
    if (g->n[k] > 256) return fail(c, DPO_EINVAL, "grid: at most 256 nodes per axis");
    N *= g->n[k];
  }
  if (N > 0x7fffffffLL / 2) return fail(c, DPO_EINVAL, "grid: too many nodes (limit 2^30)");
  return DPO_OK;
}

int validate_problem(dpo_ctx* c, const dpo_problem* p) {
  if (!p) return fail(c, DPO_EINVAL, "problem is NULL");
  if (p->model != DPO_MODEL_ORBIT && p->model != DPO_MODEL_EIKONAL && p->model != DPO_MODEL_CROWN)
    return fail(c, DPO_EINVAL, "problem: unknown model");
  if (p->model == DPO_MODEL_CROWN && !(p->mu > 0 && p->accel >= 0))
    return fail(c, DPO_EINVAL, "problem: the crown model needs mu > 0 and accel >= 0");
  if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(c, DPO_EINVAL, "problem: dt must be > 0");
  if (!(p->lambda >= 0)) return fail(c, DPO_EINVAL, "problem: lambda must be >= 0");
  if (!std::isfinite(p->M)) return fail(c, DPO_EINVAL, "problem: M must be finite");
  if (p->model == DPO_MODEL_ORBIT && !(p->accel >= 0 && p->mdot >= 0))
    return fail(c, DPO_EINVAL, "problem: accel and mdot must be >= 0");
  if (p->integrator != DPO_STEP_EULER && p->integrator != DPO_STEP_HEUN)
    return fail(c, DPO_EINVAL, "problem: unknown integrator");
  return DPO_OK;
}

int validate_search(dpo_ctx* c, const dpo_search* s) {
  if (!s) return fail(c, DPO_EINVAL, "search is NULL");
  if (s->mode == DPO_SEARCH_TABLE || s->mode == DPO_SEARCH_TABLE_WALK) {
    if (s->n_angles < 1 || s->n_angles > 1024) return fail(c, DPO_EINVAL, "search: n_angles in [1, 1024]");
  } else if (s->mode == DPO_SEARCH_SCAN_GOLDEN || s->mode == DPO_SEARCH_SEEDED) {
    if (s->n_scan < 8 || s->n_scan > 1024) return fail(c, DPO_EINVAL, "search: n_scan in [8, 1024]");
    if (s->n_golden < 0 || s->n_golden > 64) return fail(c, DPO_EINVAL, "search: n_golden in [0, 64]");
    if (s->mode == DPO_SEARCH_SEEDED) {
      if (s->n_local < 3 || s->n_local > 64) return fail(c, DPO_EINVAL, "search: n_local in [3, 64]");
      if (!(s->local_half_width > 0 && s->local_half_width <= 0.785398))
        return fail(c, DPO_EINVAL, "search: local_half_width in (0, pi/4]");
      if (!(s->fallback_tol >= 0)) return fail(c, DPO_EINVAL, "search: fallback_tol >= 0");
    }
  } else {
    return fail(c, DPO_EINVAL, "search: unknown mode");
  }
  return DPO_OK;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int kRot = 2 + 2 * 64;

// Workgroups of the second (fallback) pass of a seeded sweep; the residual
// partial buffer has room for them after the first pass's.
constexpr int kFallbackBlocks = 2048;

// MI355X Infinity Cache (last-level cache shared by the XCDs).
constexpr double kLastLevelCacheBytes = 256.0 * 1024 * 1024;

// Rotation constants of the golden section on [u0 - half, u0 + half]: sin/cos
// of half*rho^3 (the two interior points), then of L0*rho^(k+4), L0 = 2*half,
// the move of the new point at step k (FP64, rounded to float).
void golden_rotations(double half, float* out) {
  const double rho = (std::sqrt(5.0) - 1.0) / 2.0;
  const double first = half * rho * rho * rho;
  out[0] = (float)std::sin(first);
  out[1] = (float)std::cos(first);
  double step = 2.0 * half * rho * rho * rho * rho;
  for (int k = 0; k < 64; k++) {
    out[2 + 2 * k] = (float)std::sin(step);
    out[3 + 2 * k] = (float)std::cos(step);
    step *= rho;
  }
}

// Tabulated angles u_k = -pi + 2*pi*k/K (FP64, rounded to float).
int upload_table(dpo_ctx* c) {
  if (!c->rot && hipMalloc(&c->rot, sizeof(float) * 2 * kRot) != hipSuccess) return fail(c, DPO_ENOMEM, "rotation table alloc");
  {
    std::vector<float> r(2 * kRot, 0.0f);
    const double pi = 3.14159265358979323846;
    golden_rotations(2.0 * pi / (double)(c->search.n_scan > 0 ? c->search.n_scan : 8), r.data());
    golden_rotations(c->search.local_half_width > 0 ? c->search.local_half_width : 0.1, r.data() + kRot);
    HIP_TRY(c, hipMemcpy(c->rot, r.data(), sizeof(float) * 2 * kRot, hipMemcpyHostToDevice));
  }
  const bool table = c->search.mode == DPO_SEARCH_TABLE || c->search.mode == DPO_SEARCH_TABLE_WALK;
  const int K = table ? c->search.n_angles : c->search.n_scan;
  if (K > c->tab_cap) {
    if (c->tab) hipFree(c->tab);
    c->tab = nullptr;
    if (hipMalloc(&c->tab, sizeof(float) * 3 * K) != hipSuccess) return fail(c, DPO_ENOMEM, "table alloc");
    c->tab_cap = K;
  }
  std::vector<float> h(3 * K);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < K; k++) {
    const double u = -pi + 2.0 * pi * (double)k / (double)K;
    h[k] = (float)std::sin(u);
    h[K + k] = (float)std::cos(u);
    h[2 * K + k] = (float)u;
  }
  HIP_TRY(c, hipMemcpy(c->tab, h.data(), sizeof(float) * 3 * K, hipMemcpyHostToDevice));
  c->n_ang = K;
  return DPO_OK;
}

// periodic3: axis 3 wraps, node i at lo + i*(hi - lo)/n (hi is lo's image).
Grid make_grid(const dpo_grid& g, bool periodic3 = false) {
  Grid G;
  for (int k = 0; k < 4; k++) {
    G.n[k] = g.n[k];
    G.lo[k] = g.lo[k];
    G.h[k] = (g.hi[k] - g.lo[k]) / (double)(k == 3 && periodic3 ? g.n[k] : g.n[k] - 1);
    G.inv_h[k] = 1.0 / G.h[k];
  }
  G.periodic3 = periodic3 ? 1 : 0;
  G.clamp12 = periodic3 ? 1 : 0;  // the crown problem
  G.st[0] = 1;
  G.st[1] = g.n[0];
  G.st[2] = g.n[0] * g.n[1];
  G.st[3] = g.n[0] * g.n[1] * g.n[2];
  return G;
}

SweepArgs base_args(const dpo_ctx* c) {
  SweepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.G = c->G;
  a.P = c->P;
  a.free_node = c->free_node;
  a.n_free = (int)c->n_free;
  a.rinv = c->rinv;
  a.g1tab = c->gtab;
  a.g2tab = c->gtab + c->grid.n[3];
  a.c0 = c->c0;
  a.c1 = c->c1;
  a.c2 = c->c2;
  a.c3 = c->prob.dt * c->G.inv_h[3];
  a.qnode = c->qnode;
  a.gm = c->gm;
  a.tab_sin = c->tab;
  a.tab_cos = c->tab + c->n_ang;
  a.tab_ang = c->tab + 2 * c->n_ang;
  a.n_ang = c->n_ang;
  a.n_golden = c->search.n_golden;
  a.rot_scan = c->rot;
  a.rot_local = c->rot + kRot;
  a.half_width = (float)(2.0 * 3.14159265358979323846 / (double)(c->search.n_scan > 0 ? c->search.n_scan : 1));
  a.n_local = c->search.n_local;
  a.local_half_width = (float)c->search.local_half_width;
  a.fallback_tol = (float)c->search.fallback_tol;
  a.partial = c->partial;
  a.mode = c->search.mode;
  a.w_time = c->prob.w_time;
  a.w_fuel = c->prob.w_fuel;
  a.lambda = c->prob.lambda;
  return a;
}

bool use_fast(const dpo_ctx* c);

// The LDS-brick evaluation sweeps are planned for the orbit model with the
// Euler foot, a thrust step of less than one mass cell, and bricks of the
// feet's reach that fit half of a CU's LDS.  The descriptor-driven form
// (policy iteration) is the automatic choice wherever the descriptors are
// stored per node (at least half of the nodes free); the form that recomputes
// the foot from the control arrays only on request (eval path 2): the foot's
// FP64 node terms and sin/cos make it arithmetic-bound, and the free-list
// kernel is faster there.
bool use_brick_desc(const dpo_ctx* c) { return c->brick_ok && c->eval_path != 1 && c->desc_format == 2; }
bool use_brick_policy(const dpo_ctx* c) { return c->brick_ok && c->eval_path == 2; }

// Halo of one brick tile: the signed reach of its nodes' feet along v_r and
// v_t (in cells, over every r node and every control, from the FP64 node
// terms the sweeps round, widened by 1e-3 cell), as rows below and above
// the tile.  At least one row below: a foot clamped to the last cell (n - 2)
// of a node on the last row reads the row below it.
struct TileHalo {
  int r0, r1, t0, t1;
};

TileHalo tile_halo(const dpo_ctx* c, int A, int tr, int C, int tt) {
  const dpo_grid& g = c->grid;
  const dpo_problem& p = c->prob;
  const int a1 = std::min(A + tr, g.n[1]) - 1, c1 = std::min(C + tt, g.n[2]) - 1;
  const double vr_a = g.lo[1] + A * c->G.h[1], vr_b = g.lo[1] + a1 * c->G.h[1];
  const double vt_a = g.lo[2] + C * c->G.h[2], vt_b = g.lo[2] + c1 * c->G.h[2];
  const double q_a = vt_a * vt_a, q_b = vt_b * vt_b;
  const double vt2_max = std::max(q_a, q_b), vt2_min = (vt_a <= 0 && vt_b >= 0) ? 0.0 : std::min(q_a, q_b);
  double lo1 = INFINITY, hi1 = -INFINITY, lo2 = INFINITY, hi2 = -INFINITY;
  for (int i = 0; i < g.n[0]; i++) {
    const double ri = 1.0 / (g.lo[0] + i * c->G.h[0]);
    for (double vt2 : {vt2_min, vt2_max}) {
      const double d = c->c1 * (vt2 * ri - p.mu * ri * ri);
      lo1 = std::min(lo1, d);
      hi1 = std::max(hi1, d);
    }
    for (double vr : {vr_a, vr_b})
      for (double vt : {vt_a, vt_b}) {
        const double d = -c->c2 * vr * vt * ri;
        lo2 = std::min(lo2, d);
        hi2 = std::max(hi2, d);
      }
  }
  const double acc = p.accel / g.lo[3];
  const double g1 = std::fabs(p.dt * acc * c->G.inv_h[1]) + 1e-3, g2 = std::fabs(p.dt * acc * c->G.inv_h[2]) + 1e-3;
  TileHalo h;
  h.r0 = std::max(1, -(int)std::floor(lo1 - g1));
  h.r1 = std::max(0, (int)std::floor(hi1 + g1) + 1);
  h.t0 = std::max(1, -(int)std::floor(lo2 - g2));
  h.t1 = std::max(0, (int)std::floor(hi2 + g2) + 1);
  return h;
}

// The brick tile (tr v_r rows by tt v_t rows, every r) with the least LDS
// traffic per node whose largest brick fits half of a CU's LDS (two
// workgroups per CU), and its per-tile halo table on the device.
void plan_brick(dpo_ctx* c) {
  c->brick_ok = false;
  const dpo_grid& g = c->grid;
  const dpo_problem& p = c->prob;
  if (p.model != DPO_MODEL_ORBIT || p.integrator != DPO_STEP_EULER) return;
  if (!(c->gm > -1.0f && c->gm <= 0.0f) || !(g.lo[0] > 0) || !(g.lo[3] > 0)) return;
  // reach over the whole grid: a sanity bound on the halo sizes
  const TileHalo all = tile_halo(c, 0, g.n[1], 0, g.n[2]);
  if (all.r0 + all.r1 > 64 || all.t0 + all.t1 > 64) return;
  const int n0 = g.n[0];
  const size_t lds_cap = 80 * 1024;
  double best = INFINITY;
  BrickPlan B{};
  std::vector<int4> best_halo;
  for (int tr : {32, 16, 8, 4, 2, 1})
    for (int tt : {16, 8, 4, 2, 1}) {
      if (tr > g.n[1] || tt > g.n[2]) continue;
      if (n0 * tr * tt > kBrickBlock * kBrickNodes) continue;
      const int n_at = (g.n[1] + tr - 1) / tr, n_ct = (g.n[2] + tt - 1) / tt;
      std::vector<int4> halo((size_t)n_at * n_ct);
      size_t slot = 0;
      double rows = 0;
      for (int ct = 0; ct < n_ct; ct++)
        for (int at = 0; at < n_at; at++) {
          const TileHalo h = tile_halo(c, at * tr, tr, ct * tt, tt);
          halo[(size_t)at + (size_t)n_at * ct] = make_int4(h.r0, h.r1, h.t0, h.t1);
          const size_t br = tr + h.r0 + h.r1, bt = tt + h.t0 + h.t1;
          slot = std::max(slot, br * bt * n0);
          rows += (double)br * bt;
        }
      if (2 * slot * sizeof(float) > lds_cap) continue;
      const size_t loads = (n0 % 4 == 0) ? slot / 4 : slot;
      if (loads > (size_t)kBrickBlock * ((n0 % 4 == 0) ? kBrickMaxPf : 4 * kBrickMaxPf)) continue;
      const double over = rows / ((double)n_at * n_ct * tr * tt);
      if (over < best - 1e-9) {
        best = over;
        B.tr = tr;
        B.tt = tt;
        B.n_at = n_at;
        B.n_ct = n_ct;
        B.slot = (int)slot;
        best_halo.swap(halo);
      }
    }
  if (!(best < INFINITY)) return;
  // mass planes per workgroup: 8 (each plane's brick loaded once per 9/8
  // planes) while that leaves at least 8 workgroups per CU, else 4, else 2
  // with at least 4 per CU, else 1, so that thin grids (one GPU's slab of a
  // sharded grid) still fill the chip.  At 96^3 x 64 runs of 8 planes take
  // 0.201 ms per sweep against 0.214-0.217 ms with 9 or 10; with 10-byte
  // descriptors 0.207 ms against 0.216 ms with 4 and 0.224 ms with 16 (half
  // the workgroups: the last round leaves CUs idle).
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1) {
    (void)hipGetLastError();
    cus = 256;
  }
  const int64_t columns = (int64_t)B.n_at * B.n_ct;
  B.planes = 1;
  for (int P : {8, 4, 2}) {
    if (columns * ((g.n[3] + P - 1) / P) >= (int64_t)(P >= 4 ? 8 : 4) * cus) {
      B.planes = P;
      break;
    }
  }
  B.n_mc = (g.n[3] + B.planes - 1) / B.planes;
  if ((int64_t)B.n_at * B.n_ct * B.n_mc > 0x7fffffff) return;
  if (prepare_eval_brick(B) != hipSuccess) return;
  int4* d = nullptr;
  if (hipMalloc(&d, sizeof(int4) * best_halo.size()) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  if (hipMemcpy(d, best_halo.data(), sizeof(int4) * best_halo.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(d);
    return;
  }
  B.halo = d;
  c->brick_halo = d;
  c->brick = B;
  c->brick_over = best;
  c->brick_ok = true;
}

int brick_blocks(const dpo_ctx* c) { return c->brick.n_at * c->brick.n_ct * c->brick.n_mc; }

// Final FP64 reduction of the last node kernel's partials into `out`.
int finish_resid(dpo_ctx* c, double* out, hipStream_t s) {
  if (!out) return DPO_OK;
  const int nb = c->last_blocks;
  if (nb == 0) {
    HIP_TRY(c, hipMemsetAsync(out, 0, sizeof(double) * kPartial, s));
    return DPO_OK;
  }
  HIP_TRY(c, launch_resid_final(c->partial, nb, c->partial + (size_t)kPartial * c->partial_blocks, out, s));
  return DPO_OK;
}

int ensure_work(dpo_ctx* c) {
  if (c->work) return DPO_OK;
  if (hipMalloc(&c->work, sizeof(float) * (size_t)c->N) != hipSuccess)
    return fail(c, DPO_ENOMEM, "solver work buffer alloc");
  return DPO_OK;
}

int ensure_pi_buffers(dpo_ctx* c) {
  if (!c->work2 && hipMalloc(&c->work2, sizeof(float) * (size_t)c->N) != hipSuccess)
    return fail(c, DPO_ENOMEM, "solver work buffer alloc");
  if (!c->resid_host && hipHostMalloc(&c->resid_host, sizeof(double) * kPartial, hipHostMallocDefault) != hipSuccess)
    return fail(c, DPO_ENOMEM, "pinned residual buffer alloc");
  if (!c->resid_ready && hipEventCreateWithFlags(&c->resid_ready, hipEventDisableTiming) != hipSuccess)
    return fail(c, DPO_EHIP, "residual event create");
  for (auto& row : c->step_ev)
    for (auto& e : row)
      if (!e && hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
        return fail(c, DPO_EHIP, "step timing event create");
      }
  return DPO_OK;
}

// Descriptor form: the compact 16-bit code needs every foot within
// kDescReach cells of its node along v_r and v_t.  The bound is taken over the
// grid's r nodes and the extreme v_r, v_t values (the drift along v_r is
// linear in v_t^2, the one along v_t in v_r*v_t), plus the thrust step, plus
// one cell for the cell base and one of margin.  With at least half of the
// nodes free, the codes are stored per node and the sweep needs no free list.
int desc_format_for(const dpo_ctx* c) {
  const dpo_grid& g = c->grid;
  const dpo_problem& p = c->prob;
  const double h1 = c->G.h[1], h2 = c->G.h[2];
  double mv = 0, mt = 0;
  if (p.model == DPO_MODEL_ORBIT) {
    if (!(g.lo[3] > 0)) return 0;
    const double a2 = g.lo[2] * g.lo[2], b2 = g.hi[2] * g.hi[2];
    const double vt2_max = std::max(a2, b2), vt2_min = (g.lo[2] <= 0 && g.hi[2] >= 0) ? 0.0 : std::min(a2, b2);
    const double vrvt = std::max(std::fabs(g.lo[1]), std::fabs(g.hi[1])) * std::max(std::fabs(g.lo[2]), std::fabs(g.hi[2]));
    for (int i = 0; i < g.n[0]; i++) {
      const double r = g.lo[0] + i * c->G.h[0];
      if (!(r > 0)) return 0;
      const double ri = 1.0 / r;
      mv = std::max(mv, std::max(std::fabs(vt2_max * ri - p.mu * ri * ri), std::fabs(vt2_min * ri - p.mu * ri * ri)));
      mt = std::max(mt, vrvt * ri);
    }
    const double thrust = p.accel / g.lo[3];
    mv = p.dt * (mv + thrust) / h1;
    mt = p.dt * (mt + thrust) / h2;
  } else {
    mv = p.dt * std::fabs(p.speed) / h1;
    mt = p.dt * std::fabs(p.speed) / h2;
  }
  if (!std::isfinite(mv) || !std::isfinite(mt) || mv + 2 > kDescReach || mt + 2 > kDescReach) return 0;
  return 2 * c->n_free >= c->N ? 2 : 1;
}

int ensure_desc(dpo_ctx* c) {
  if (c->desc_format >= 0) return DPO_OK;
  const int format = desc_format_for(c);
  const size_t n = (size_t)std::max<int64_t>(1, format == 2 ? c->N : c->n_free);
  bool ok = true;
  if (format == 2) {
    // every descriptor starts as the skip code (all bits set); greedy sweeps
    // overwrite the free nodes'
    ok = hipMalloc(&c->desc_pk, sizeof(uint2) * n) == hipSuccess &&
         hipMemset(c->desc_pk, 0xff, sizeof(uint2) * n) == hipSuccess;
  } else {
    ok = hipMalloc(&c->desc_w, sizeof(float2) * n) == hipSuccess;
    if (format == 0) ok = ok && hipMalloc(&c->desc_code, sizeof(int) * n) == hipSuccess;
    else ok = ok && hipMalloc(&c->desc16, sizeof(uint16_t) * n) == hipSuccess;
  }
  if (!ok) return fail(c, DPO_ENOMEM, "descriptor alloc");
  c->desc_format = format;
  return DPO_OK;
}

void set_desc_out(dpo_ctx* c, SweepArgs& a) {
  if (c->desc_format == 2) {
    a.desc_pk = c->desc_pk;
    a.desc_dense = 1;
  } else {
    a.desc_w = c->desc_w;
    if (c->desc_format == 0) a.desc_code = c->desc_code;
    else a.desc16 = c->desc16;
  }
  c->desc_valid = true;
}

int read_resid(dpo_ctx* c, double h[kPartial], hipStream_t s) {
  HIP_TRY(c, hipMemcpyAsync(h, c->resid, sizeof(double) * kPartial, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  return DPO_OK;
}

int64_t evals_per_full_search(const dpo_ctx* c) {
  if (c->search.mode == DPO_SEARCH_TABLE || c->search.mode == DPO_SEARCH_TABLE_WALK) return 1 + c->search.n_angles;
  return 1 + c->search.n_scan + (c->search.n_golden > 0 ? 2 + c->search.n_golden : 0);
}

bool use_fast(const dpo_ctx* c) { return c->path == 2 || (c->path == 0 && c->fast_ok); }

// Foot descriptors record the r and m cells as functions of the node and the
// throttle alone, which holds for the Euler foot only.
bool desc_ok(const dpo_ctx* c) { return !c->P.heun && c->P.model != DPO_MODEL_CROWN; }

// Table walk evaluation counters: one entry per workgroup of the largest grid
// any sweep launches (workgroups of 64 threads and up).
int ensure_walk(dpo_ctx* c) {
  if (c->eval_acc) return DPO_OK;
  const size_t n = (size_t)blocks_for(std::max<int64_t>(1, c->n_free), 64);
  if (hipMalloc(&c->eval_acc, sizeof(unsigned long long) * n) != hipSuccess ||
      hipMalloc(&c->eval_sum, sizeof(unsigned long long)) != hipSuccess)
    return fail(c, DPO_ENOMEM, "walk counter alloc");
  return DPO_OK;
}

int walk_counts_zero(dpo_ctx* c, hipStream_t s) {
  const size_t n = (size_t)blocks_for(std::max<int64_t>(1, c->n_free), 64);
  HIP_TRY(c, hipMemsetAsync(c->eval_acc, 0, sizeof(unsigned long long) * n, s));
  return DPO_OK;
}

// Sum of the walk's thrust evaluations since walk_counts_zero (synchronises s).
int walk_counts_read(dpo_ctx* c, hipStream_t s, int64_t* out) {
  const int n = blocks_for(std::max<int64_t>(1, c->n_free), 64);
  unsigned long long h = 0;
  HIP_TRY(c, launch_sum_counts(c->eval_acc, n, c->eval_sum, s));
  HIP_TRY(c, hipMemcpyAsync(&h, c->eval_sum, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  *out = (int64_t)h;
  return DPO_OK;
}

// walk_from: TABLE_WALK sweeps walk from these angles (null: the full table);
// count: add the walk's thrust evaluations to the context's counters.
int sweep_full(dpo_ctx* c, const float* Vin, float* Vout, float* ang, uint8_t* thr, hipStream_t s,
               bool desc = false, bool incumbent = false, bool want_resid = true, const float* walk_from = nullptr,
               bool count = false) {
  SweepArgs a = base_args(c);
  if (!want_resid) a.partial = nullptr;
  a.V_in = Vin;
  a.V_out = Vout;
  a.pol_ang = ang;
  a.pol_thr = thr;
  if (incumbent) {
    a.pol_ang_in = ang;
    a.pol_thr_in = thr;
  }
  // descriptors describe the policy of the last sweep that wrote them
  if (desc && desc_ok(c)) set_desc_out(c, a);
  else c->desc_valid = false;
  if (a.n_free == 0) return DPO_OK;
  // a SEEDED context's full steps (the first step of a seeded solve and the
  // steps that certify it) take its scan + golden parameters
  int mode = (c->search.mode == DPO_SEARCH_SCAN_GOLDEN || c->search.mode == DPO_SEARCH_SEEDED) ? 1 : 0;
  if (c->search.mode == DPO_SEARCH_TABLE_WALK && walk_from) {
    mode = 3;
    a.walk_from = walk_from;
    if (count) a.eval_acc = c->eval_acc;
  }
  hipError_t e;
  if (use_fast(c)) e = launch_sweep_fast(a, mode, c->block, s);
  else e = launch_sweep_direct(a, mode, s);
  c->last_blocks = blocks_for(c->n_free, use_fast(c) ? c->block : kBlock);
  if (e != hipSuccess) return hip_fail(c, e, "bellman sweep launch");
  return DPO_OK;
}

int sweep_seeded(dpo_ctx* c, const float* Vin, float* Vout, float* ang, uint8_t* thr, const float* seed,
                 hipStream_t s, bool desc = false, bool incumbent = false) {
  SweepArgs a = base_args(c);
  a.V_in = Vin;
  a.V_out = Vout;
  a.pol_ang = ang;
  a.pol_thr = thr;
  if (incumbent) {
    a.pol_ang_in = ang;
    a.pol_thr_in = thr;
  }
  a.seed = seed;
  if (desc && desc_ok(c)) set_desc_out(c, a);
  else c->desc_valid = false;
  if (a.n_free == 0) return DPO_OK;
  if (!use_fast(c)) {
    hipError_t e = launch_sweep_direct(a, 2, s);
    c->last_blocks = blocks_for(c->n_free, kBlock);
    if (e != hipSuccess) return hip_fail(c, e, "seeded sweep launch");
    return DPO_OK;
  }
  // factorised path: the local searches first, then the full search at the
  // nodes that fall back, as a second launch over the list the first built
  if (!c->fb_list) {
    if (hipMalloc(&c->fb_list, sizeof(int) * (size_t)c->n_free) != hipSuccess ||
        hipMalloc(&c->fb_count, sizeof(int)) != hipSuccess)
      return fail(c, DPO_ENOMEM, "fallback list alloc");
  }
  a.fb_list = c->fb_list;
  a.fb_count = c->fb_count;
  const int nb1 = blocks_for(c->n_free, c->block);
  const int nb2 = std::min(kFallbackBlocks, nb1);
  hipError_t e = launch_zero_count(c->fb_count, s);
  if (e == hipSuccess) e = launch_sweep_fast(a, 2, c->block, s);
  if (e == hipSuccess) {
    SweepArgs b = a;
    b.partial = c->partial + (size_t)kPartial * nb1;
    e = launch_sweep_fallback(b, c->block, nb2, s);
  }
  c->last_blocks = nb1 + nb2;
  if (e != hipSuccess) return hip_fail(c, e, "seeded sweep launch");
  return DPO_OK;
}

int sweep_eval(dpo_ctx* c, const float* Vin, float* Vout, const float* ang, const uint8_t* thr, bool want_resid,
               hipStream_t s) {
  SweepArgs a = base_args(c);
  a.V_in = Vin;
  a.V_out = Vout;
  a.pol_ang_in = ang;
  a.pol_thr_in = thr;
  if (a.n_free == 0) return DPO_OK;
  if (use_brick_policy(c)) {
    // streamed per sweep: angle, throttle and kind, and two value arrays
    const bool streamed = 14.0 * (double)c->N > kLastLevelCacheBytes;
    hipError_t e = launch_eval_brick(a, c->brick, c->kind, want_resid, streamed, s);
    if (want_resid) c->last_blocks = brick_blocks(c);
    if (e != hipSuccess) return hip_fail(c, e, "policy eval (brick) launch");
    return DPO_OK;
  }
  hipError_t e = launch_policy_eval(a, want_resid, s);
  if (want_resid) c->last_blocks = blocks_for(c->n_free, kBlock);
  if (e != hipSuccess) return hip_fail(c, e, "policy eval launch");
  return DPO_OK;
}

// Bytes of the per-node stream of one descriptor sweep (coordinates, codes,
// weights), not counting the values.
int64_t eval_stream_bytes(const dpo_ctx* c) {
  const int format = c->desc_format >= 0 ? c->desc_format : desc_format_for(c);
  if (format == 0) return 16 * c->n_free;
  if (format == 1) return 14 * c->n_free;
  return 8 * c->N;
}

// Frozen-policy sweep driven by the descriptors of the last greedy sweep.
int sweep_eval_desc(dpo_ctx* c, const float* Vin, float* Vout, hipStream_t s) {
  SweepArgs a = base_args(c);
  a.V_in = Vin;
  a.V_out = Vout;
  a.desc_code_in = c->desc_code;
  a.desc16_in = c->desc16;
  a.desc_w_in = c->desc_w;
  a.desc_pk_in = c->desc_pk;
  if (a.n_free == 0) return DPO_OK;
  // streamed per sweep: the per-node stream and two value arrays
  const double bytes = (double)eval_stream_bytes(c) + 8.0 * (double)c->N;
  const bool streamed = bytes > kLastLevelCacheBytes;
  if (use_brick_desc(c)) {
    a.desc_dense = 1;
    hipError_t e = launch_eval_brick_desc(a, c->brick, streamed, s);
    if (e != hipSuccess) return hip_fail(c, e, "policy eval (descriptor brick) launch");
    return DPO_OK;
  }
  hipError_t e = c->desc_format == 0 ? launch_policy_eval_desc(a, streamed, s)
                                     : launch_policy_eval_desc16(a, c->desc_format, streamed, s);
  if (e != hipSuccess) return hip_fail(c, e, "policy eval (descriptor) launch");
  return DPO_OK;
}

// ---- exact policy evaluation: restarted GMRES(m) on (I - gamma P) v = b
// over the free nodes (paper Section 3: eq:p_eval is a sparse linear system;
// GMRES is the solver the paper names).  b is the frozen-policy sweep of V
// with its free entries zeroed (running cost plus the fixed corners and M);
// the operator is the sweep without that affine part.  Classical
// Gram-Schmidt in one pass, its coefficients formed in the same pass as
// w = v - gamma P v: with a basis of at most 8 vectors the loss of
// orthogonality a second pass would repair costs no operator applications
// here (Example 1: 1681 with one pass, 1690 with two), and the stop test
// uses the true residual b - A x, not the Hessenberg estimate.  The
// coefficients, the Hessenberg matrix and its Givens rotations stay on the
// device in FP64, so a step needs no host synchronisation; the triangular
// solve of a cycle runs on the host.  Stop measure: the node-wise relative
// residual max_j |b - A v|_j / max(1, |v_j|), checked between cycles; a cycle
// ends after m steps or once its 2-norm residual has fallen by kCycleDrop
// (read one step late, so at most one step more).

constexpr int kGmresRestart = 8;
static_assert(kGmresRestart <= kDotGroup, "one fused dot-product pass covers the basis");
constexpr double kCycleDrop = 1e-2;
constexpr double kExactEvalTol = 5e-7;  // node-wise residual of the evaluations inside policy iteration

// Device Arnoldi state of gmres_eval: the Gram-Schmidt dot products, the
// new vector's squared norm, the Hessenberg matrix, the Givens rotations, the
// rotated right-hand side, 1/h_(k+1)k and the step's status.
constexpr int kArnD = 0, kArnNrm = kMaxBasis, kArnH = kMaxBasis + 1;
constexpr int kArnCs = kArnH + (kMaxBasis + 1) * kMaxBasis, kArnSn = kArnCs + kMaxBasis, kArnG = kArnSn + kMaxBasis;
constexpr int kArnInv = kArnG + kMaxBasis + 1, kArnStat = kArnInv + 1, kArnDoubles = kArnStat + 2;

int ensure_krylov(dpo_ctx* c, int m) {
  const size_t N = (size_t)c->N;
  if (c->kry && c->kry_m >= m) return DPO_OK;
  if (c->kry) hipFree(c->kry);
  c->kry = nullptr;
  if (hipMalloc(&c->kry, sizeof(float) * N * (size_t)(m + 1)) != hipSuccess) return fail(c, DPO_ENOMEM, "Krylov basis alloc");
  c->kry_m = m;
  if (!c->kbuf && hipMalloc(&c->kbuf, sizeof(float) * N * 3) != hipSuccess) return fail(c, DPO_ENOMEM, "Krylov vectors alloc");
  if (!c->kpart && hipMalloc(&c->kpart, sizeof(double) * kStreamBlocks * kDotGroup) != hipSuccess)
    return fail(c, DPO_ENOMEM, "Krylov partials alloc");
  if (!c->kdots && hipMalloc(&c->kdots, sizeof(double) * kMaxBasis) != hipSuccess) return fail(c, DPO_ENOMEM, "alloc");
  if (!c->kcoef && hipMalloc(&c->kcoef, sizeof(double) * kMaxBasis) != hipSuccess) return fail(c, DPO_ENOMEM, "alloc");
  if (!c->karn && hipMalloc(&c->karn, sizeof(double) * kArnDoubles) != hipSuccess) return fail(c, DPO_ENOMEM, "alloc");
  if (!c->karn_host && hipHostMalloc(&c->karn_host, sizeof(double) * 2 * kMaxBasis, hipHostMallocDefault) != hipSuccess)
    return fail(c, DPO_ENOMEM, "pinned Arnoldi status alloc");
  for (auto& e : c->karn_ev)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      return fail(c, DPO_EHIP, "Arnoldi event create");
    }
  return DPO_OK;
}

// h[0..k) = <basis_i, w> on the host (synchronises s)
int host_dots(dpo_ctx* c, const float* basis, int k, const float* w, double* h, hipStream_t s) {
  HIP_TRY(c, launch_dots(basis, k, (size_t)c->N, w, (int)c->N, c->kpart, c->kdots, s));
  HIP_TRY(c, hipMemcpyAsync(h, c->kdots, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  return DPO_OK;
}

int gmres_eval(dpo_ctx* c, float* V, const float* ang, const uint8_t* thr, double tol, int max_iter, int64_t* matvecs,
               double* rel_out, hipStream_t s) {
  const int m = kGmresRestart;
  int rc = ensure_krylov(c, m);
  if (rc != DPO_OK) return rc;
  const int N = (int)c->N;
  const size_t ld = (size_t)N;
  float* B = c->kbuf;
  float* X = c->kbuf + ld;
  float* Y = c->kbuf + 2 * ld;
  float* basis = c->kry;
  SweepArgs a = base_args(c);
  a.pol_ang_in = ang;
  a.pol_thr_in = thr;
  int64_t mv = 0;
  // b: the sweep of V with its free entries zeroed (Y as scratch)
  HIP_TRY(c, hipMemcpyAsync(Y, V, sizeof(float) * ld, hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, launch_free_zero(a, Y, s));
  HIP_TRY(c, hipMemsetAsync(B, 0, sizeof(float) * ld, s));
  {
    SweepArgs e = a;
    e.V_in = Y;
    e.V_out = B;
    e.partial = nullptr;
    if (a.n_free > 0) HIP_TRY(c, launch_policy_eval(e, false, s));
  }
  // x: the current V at free nodes, zero elsewhere
  HIP_TRY(c, hipMemsetAsync(X, 0, sizeof(float) * ld, s));
  HIP_TRY(c, launch_free_copy(a, V, X, s));
  std::vector<double> H((size_t)(m + 1) * m), g(m + 1), y(m);
  double* arn = c->karn;
  double rel = 0;
  int it = 0;
  while (true) {
    // r = b - A x into basis row 0
    HIP_TRY(c, launch_eval_hom(a, X, Y, s));
    mv++;
    HIP_TRY(c, launch_residual(B, X, Y, basis, N, s));
    HIP_TRY(c, launch_relmax(basis, X, N, c->kpart, c->kdots, s));
    HIP_TRY(c, hipMemcpyAsync(&rel, c->kdots, sizeof(double), hipMemcpyDeviceToHost, s));
    double rr = 0;
    if ((rc = host_dots(c, basis, 1, basis, &rr, s)) != DPO_OK) return rc;
    const double beta = std::sqrt(rr);
    if (!(rel > tol) || !(beta > 0) || it >= max_iter) break;
    HIP_TRY(c, launch_scale(basis, 1.0 / beta, basis, N, s));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    HIP_TRY(c, hipMemcpyAsync(arn + kArnG, g.data(), sizeof(double) * (m + 1), hipMemcpyHostToDevice, s));
    // Arnoldi steps with no host synchronisation: classical Gram-Schmidt
    // (the coefficients stay on the device), the Hessenberg column and its
    // Givens rotation in one small kernel; the host reads each step's status
    // one step late, so the device always has the next step queued.
    int k = 0;
    bool stop = false;
    while (k < m && it < max_iter && !stop) {
      float* vk = basis + (size_t)k * ld;
      float* w = basis + (size_t)(k + 1) * ld;
      HIP_TRY(c, launch_eval_hom(a, vk, Y, s));
      mv++;
      it++;
      HIP_TRY(c, launch_sub_dots(vk, Y, w, basis, k + 1, ld, N, c->kpart, arn + kArnD, s));
      HIP_TRY(c, launch_axpys(w, basis, k + 1, ld, arn + kArnD, N, s, c->kpart, arn + kArnNrm));
      HIP_TRY(c, launch_arnoldi_col(k, m, arn + kArnD, arn + kArnNrm, arn + kArnH, arn + kArnCs,
                                    arn + kArnSn, arn + kArnG, arn + kArnInv, arn + kArnStat, s));
      HIP_TRY(c, launch_scale_dev(w, arn + kArnInv, w, N, s));
      HIP_TRY(c, hipMemcpyAsync(c->karn_host + 2 * k, arn + kArnStat, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(c, hipEventRecord(c->karn_ev[k & 1], s));
      k++;
      // the previous step's stop test (this step is already queued behind it)
      if (k >= 2) {
        HIP_TRY(c, hipEventSynchronize(c->karn_ev[k & 1]));
        const double* st = c->karn_host + 2 * (k - 2);
        if (!(st[0] > kCycleDrop * beta) || !(st[1] > 0)) stop = true;
      }
    }
    // x += V_k y with H y = g over the k columns the device formed
    HIP_TRY(c, hipMemcpyAsync(H.data(), arn + kArnH, sizeof(double) * (size_t)(m + 1) * m, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(g.data(), arn + kArnG, sizeof(double) * (m + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    for (int i = k - 1; i >= 0; i--) {
      double t = g[i];
      for (int q = i + 1; q < k; q++) t -= H[(size_t)i * m + q] * y[q];
      y[i] = H[(size_t)i * m + i] != 0 ? t / H[(size_t)i * m + i] : 0.0;
    }
    for (int i = 0; i < k; i++) y[i] = -y[i];
    HIP_TRY(c, hipMemcpyAsync(c->kcoef, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    HIP_TRY(c, launch_axpys(X, basis, k, ld, c->kcoef, N, s));
  }
  HIP_TRY(c, launch_free_copy(a, X, V, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (matvecs) *matvecs = mv;
  if (rel_out) *rel_out = rel;
  return DPO_OK;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ===================================================================== ABI
extern "C" {

const char* dpo_last_error(const dpo_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int dpo_create(const dpo_grid* grid, const dpo_problem* prob, const dpo_search* search,
               const uint8_t* active_mask, dpo_ctx** out) {
  if (!out) return fail(nullptr, DPO_EINVAL, "out is NULL");
  *out = nullptr;
  int rc;
  if ((rc = validate_grid(nullptr, grid)) != DPO_OK) return rc;
  if ((rc = validate_problem(nullptr, prob)) != DPO_OK) return rc;
  if ((rc = validate_search(nullptr, search)) != DPO_OK) return rc;
  dpo_ctx* c = new dpo_ctx();
  c->grid = *grid;
  c->prob = *prob;
  c->search = *search;
  const bool crown = prob->model == DPO_MODEL_CROWN;
  if (crown && !(grid->lo[0] > 0)) {
    g_err = "grid: the crown model needs r > 0";
    delete c;
    return DPO_EINVAL;
  }
  c->G = make_grid(*grid, crown);
  c->P.model = prob->model;
  c->P.el_beta = prob->el_beta;
  c->P.el_gamma = prob->el_gamma;
  c->P.el_a = prob->el_a;
  c->P.el_ex = prob->el_e * std::cos(prob->el_omega);
  c->P.el_ey = prob->el_e * std::sin(prob->el_omega);
  c->P.heun = prob->integrator == DPO_STEP_HEUN ? 1 : 0;
  c->P.mu = prob->mu;
  c->P.accel = prob->accel;
  c->P.mdot = prob->mdot;
  c->P.dt = prob->dt;
  c->P.speed = prob->speed;
  c->P.q_coast = (float)(prob->dt * prob->w_time);
  c->P.q_thr = (float)(prob->dt * (prob->w_time + prob->w_fuel));
  c->P.gamma = (float)std::exp(-prob->lambda * prob->dt);
  c->P.M = (float)prob->M;
  for (int k = 0; k < 4; k++) {
    c->tb.c[k] = prob->tgt_c[k];
    c->tb.w[k] = prob->tgt_w[k];
  }
  c->N = (int64_t)grid->n[0] * grid->n[1] * grid->n[2] * grid->n[3];
  const int N = (int)c->N;
  int* counts = nullptr;
  int* offsets = nullptr;
  const int nch = compact_chunks(N);
  auto cleanup = [&](int code) {
    if (counts) hipFree(counts);
    if (offsets) hipFree(offsets);
    if (code != DPO_OK) {
      g_err = c->err;
      dpo_destroy(c);
    }
    return code;
  };
  if (hipMalloc(&c->kind, (size_t)N) != hipSuccess || hipMalloc(&c->free_node, sizeof(uint32_t) * (size_t)N) != hipSuccess ||
      hipMalloc(&c->rinv, sizeof(double) * grid->n[0]) != hipSuccess ||
      hipMalloc(&c->gtab, sizeof(float) * 2 * grid->n[3]) != hipSuccess ||
      hipMalloc(&counts, sizeof(int) * nch) != hipSuccess || hipMalloc(&offsets, sizeof(int) * (nch + 1)) != hipSuccess ||
      hipMalloc(&c->resid, sizeof(double) * kPartial) != hipSuccess) {
    c->err = "device allocation failed in dpo_create";
    return cleanup(DPO_ENOMEM);
  }
  // Per-axis tables: 1/r per r node (FP64), thrust displacement per m plane.
  {
    std::vector<double> rinv(grid->n[0]);
    for (int i = 0; i < grid->n[0]; i++) {
      const double r = grid->lo[0] + i * c->G.h[0];
      rinv[i] = prob->model != DPO_MODEL_EIKONAL ? 1.0 / r : 0.0;
    }
    const int nm = grid->n[3];
    std::vector<float> gt(2 * nm);
    double gmax = 0;
    for (int i = 0; i < nm; i++) {
      const double m = grid->lo[3] + i * c->G.h[3];
      const double acc = prob->model == DPO_MODEL_ORBIT ? prob->accel / m
                         : prob->model == DPO_MODEL_CROWN ? prob->accel : prob->speed;
      const double g1 = prob->dt * acc * c->G.inv_h[1], g2 = prob->dt * acc * c->G.inv_h[2];
      gt[i] = (float)g1;
      gt[nm + i] = (float)g2;
      gmax = std::max(gmax, std::max(std::fabs(g1), std::fabs(g2)));
    }
    c->c0 = prob->dt * c->G.inv_h[0];
    c->c1 = prob->dt * c->G.inv_h[1];
    c->c2 = prob->dt * c->G.inv_h[2];
    const double gm = prob->model == DPO_MODEL_ORBIT ? -prob->dt * prob->mdot * c->G.inv_h[3] : 0.0;
    c->gm = (float)gm;
    // the factorised thrust kernel needs every thrust foot of a node within two
    // cells per moving axis and within one m cell
    c->fast_ok = gmax < 0.45 && gm > -1.0 && gm <= 0.0 && prob->integrator == DPO_STEP_EULER && !crown;
    plan_brick(c);
    hipError_t e1 = hipMemcpy(c->rinv, rinv.data(), sizeof(double) * rinv.size(), hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(c->gtab, gt.data(), sizeof(float) * gt.size(), hipMemcpyHostToDevice);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      c->err = "dpo_create: table upload failed";
      return cleanup(DPO_EHIP);
    }
  }
  hipError_t e = launch_classify(c->G, c->tb, active_mask, c->kind, N, nullptr);
  if (e == hipSuccess) e = launch_compact(c->G, c->kind, N, counts, offsets, c->free_node, nullptr);
  int total = 0;
  if (e == hipSuccess) e = hipMemcpy(&total, offsets + nch, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    c->err = std::string("dpo_create: ") + hipGetErrorString(e);
    return cleanup(DPO_EHIP);
  }
  c->n_free = total;
  if (crown) {
    if (hipMalloc(&c->qnode, sizeof(float) * (size_t)N) != hipSuccess) {
      c->err = "device allocation failed in dpo_create";
      return cleanup(DPO_ENOMEM);
    }
    e = launch_node_cost(c->G, c->P, c->qnode, N, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      c->err = std::string("dpo_create: ") + hipGetErrorString(e);
      return cleanup(DPO_EHIP);
    }
  }
  c->partial_blocks = blocks_for(total > 0 ? total : 1, 64) + kFallbackBlocks;
  // the partials, then the first stage of their reduction
  if (hipMalloc(&c->partial, sizeof(double) * kPartial * (c->partial_blocks + kResidStage)) != hipSuccess) {
    c->err = "device allocation failed in dpo_create";
    return cleanup(DPO_ENOMEM);
  }
  if ((rc = upload_table(c)) != DPO_OK) return cleanup(rc);
  *out = c;
  return cleanup(DPO_OK);
}

void dpo_destroy(dpo_ctx* c) {
  if (!c) return;
  if (c->kind) hipFree(c->kind);
  if (c->brick_halo) hipFree(c->brick_halo);
  if (c->free_node) hipFree(c->free_node);
  if (c->rinv) hipFree(c->rinv);
  if (c->gtab) hipFree(c->gtab);
  if (c->tab) hipFree(c->tab);
  if (c->rot) hipFree(c->rot);
  if (c->partial) hipFree(c->partial);
  if (c->resid) hipFree(c->resid);
  if (c->work) hipFree(c->work);
  if (c->work2) hipFree(c->work2);
  if (c->fb_list) hipFree(c->fb_list);
  if (c->fb_count) hipFree(c->fb_count);
  if (c->resid_host) hipHostFree(c->resid_host);
  if (c->resid_ready) hipEventDestroy(c->resid_ready);
  for (auto& row : c->step_ev)
    for (auto& e : row)
      if (e) hipEventDestroy(e);
  if (c->desc_code) hipFree(c->desc_code);
  if (c->desc16) hipFree(c->desc16);
  if (c->desc_w) hipFree(c->desc_w);
  if (c->desc_pk) hipFree(c->desc_pk);
  if (c->eval_acc) hipFree(c->eval_acc);
  if (c->qnode) hipFree(c->qnode);
  if (c->kry) hipFree(c->kry);
  if (c->kbuf) hipFree(c->kbuf);
  if (c->kpart) hipFree(c->kpart);
  if (c->kdots) hipFree(c->kdots);
  if (c->kcoef) hipFree(c->kcoef);
  if (c->karn) hipFree(c->karn);
  if (c->karn_host) hipHostFree(c->karn_host);
  for (auto& e : c->karn_ev)
    if (e) hipEventDestroy(e);
  if (c->eval_sum) hipFree(c->eval_sum);
  delete c;
}

int dpo_sizes(const dpo_ctx* c, int64_t* n_nodes, int64_t* n_free) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (n_nodes) *n_nodes = c->N;
  if (n_free) *n_free = c->n_free;
  return DPO_OK;
}

int dpo_get_kind(dpo_ctx* c, uint8_t* kind, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!kind) return fail(c, DPO_EINVAL, "kind is NULL");
  HIP_TRY(c, hipMemcpyAsync(kind, c->kind, (size_t)c->N, hipMemcpyDeviceToDevice, S(stream)));
  return DPO_OK;
}

int dpo_set_kernel_path(dpo_ctx* c, int32_t path) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (path < 0 || path > 2) return fail(c, DPO_EINVAL, "path must be 0 (auto), 1 (direct) or 2 (factorised)");
  if (path == 2 && !c->fast_ok) return fail(c, DPO_EINVAL, "the factorised kernel does not apply to this problem");
  c->path = path;
  return DPO_OK;
}

int dpo_set_block(dpo_ctx* c, int32_t block) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (block < 64 || block > 512 || block % 64) return fail(c, DPO_EINVAL, "block must be 64, 128, ..., 512");
  c->block = block;
  return DPO_OK;
}

int dpo_kernel_path(const dpo_ctx* c) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  return use_fast(c) ? 2 : 1;
}

int dpo_eval_sweep_bytes(const dpo_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return fail(const_cast<dpo_ctx*>(c), DPO_EINVAL, "NULL argument");
  if (!desc_ok(c)) {
    // no descriptors: the frozen-policy sweep reads coordinates, angle and
    // throttle (and the crown problem's node cost)
    *bytes = (4 + 4 + 1 + 8 + (c->qnode ? 4 : 0)) * c->n_free;
    return DPO_OK;
  }
  // the stream plus one value read (the gather's share) and one value write per free node
  *bytes = eval_stream_bytes(c) + 8 * c->n_free;
  return DPO_OK;
}

int dpo_set_search(dpo_ctx* c, const dpo_search* search) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  int rc = validate_search(c, search);
  if (rc != DPO_OK) return rc;
  c->search = *search;
  return upload_table(c);
}

int dpo_init_value(dpo_ctx* c, float* V, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V) return fail(c, DPO_EINVAL, "V is NULL");
  HIP_TRY(c, launch_init_value(c->kind, c->P.M, V, (int)c->N, S(stream)));
  return DPO_OK;
}

int dpo_bellman_sweep(dpo_ctx* c, const float* V_in, float* V_out, float* pol_angle, uint8_t* pol_thr,
                      double* resid, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V_in || !V_out) return fail(c, DPO_EINVAL, "V_in / V_out is NULL");
  if (V_in == V_out) return fail(c, DPO_EINVAL, "V_in and V_out must differ (Jacobi sweep)");
  if (c->search.mode == DPO_SEARCH_SEEDED) return fail(c, DPO_EINVAL, "SEEDED mode: use dpo_bellman_sweep_seeded");
  const bool walk = c->search.mode == DPO_SEARCH_TABLE_WALK;
  if (walk && !pol_angle) return fail(c, DPO_EINVAL, "TABLE_WALK: pol_angle holds the walk's start and is required");
  int rc = desc_ok(c) ? ensure_desc(c) : DPO_OK;
  if (rc != DPO_OK) return rc;
  rc = sweep_full(c, V_in, V_out, pol_angle, pol_thr, S(stream), true, false, true, walk ? pol_angle : nullptr);
  if (rc != DPO_OK) return rc;
  return finish_resid(c, resid, S(stream));
}

int dpo_bellman_sweep_seeded(dpo_ctx* c, const float* V_in, float* V_out, float* pol_angle, uint8_t* pol_thr,
                             const float* seed_angle, double* resid, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V_in || !V_out || !seed_angle) return fail(c, DPO_EINVAL, "V_in / V_out / seed_angle is NULL");
  if (V_in == V_out) return fail(c, DPO_EINVAL, "V_in and V_out must differ (Jacobi sweep)");
  if (c->search.mode != DPO_SEARCH_SEEDED) return fail(c, DPO_EINVAL, "search mode is not SEEDED");
  int rc = desc_ok(c) ? ensure_desc(c) : DPO_OK;
  if (rc != DPO_OK) return rc;
  rc = sweep_seeded(c, V_in, V_out, pol_angle, pol_thr, seed_angle, S(stream), true);
  if (rc != DPO_OK) return rc;
  return finish_resid(c, resid, S(stream));
}

int dpo_policy_eval_sweep(dpo_ctx* c, const float* V_in, float* V_out, const float* pol_angle,
                          const uint8_t* pol_thr, double* resid, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V_in || !V_out || !pol_angle || !pol_thr) return fail(c, DPO_EINVAL, "null array argument");
  if (V_in == V_out) return fail(c, DPO_EINVAL, "V_in and V_out must differ (Jacobi sweep)");
  int rc = sweep_eval(c, V_in, V_out, pol_angle, pol_thr, resid != nullptr, S(stream));
  if (rc != DPO_OK) return rc;
  return finish_resid(c, resid, S(stream));
}

int dpo_set_eval_path(dpo_ctx* c, int32_t path) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (path < 0 || path > 2) return fail(c, DPO_EINVAL, "eval path must be 0 (auto), 1 (free list) or 2 (bricks)");
  if (path == 2 && !c->brick_ok)
    return fail(c, DPO_EINVAL, "the LDS-brick evaluation sweep needs the orbit model, the Euler foot and a "
                               "thrust step of less than one mass cell");
  c->eval_path = path;
  return DPO_OK;
}

int dpo_eval_path(const dpo_ctx* c) {
  if (!c) return -1;
  if (desc_ok(c)) {
    const int format = c->desc_format >= 0 ? c->desc_format : desc_format_for(c);
    return c->brick_ok && c->eval_path != 1 && format == 2 ? 2 : 1;
  }
  return use_brick_policy(c) ? 2 : 1;
}

int dpo_policy_eval_sweep_last(dpo_ctx* c, const float* V_in, float* V_out, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V_in || !V_out) return fail(c, DPO_EINVAL, "V_in / V_out is NULL");
  if (V_in == V_out) return fail(c, DPO_EINVAL, "V_in and V_out must differ (Jacobi sweep)");
  if (!desc_ok(c)) return fail(c, DPO_EINVAL, "foot descriptors need the Euler foot; use dpo_policy_eval_sweep");
  if (!c->desc_valid) return fail(c, DPO_EINVAL, "no Bellman sweep has chosen a policy yet");
  return sweep_eval_desc(c, V_in, V_out, S(stream));
}

int dpo_solve_vi(dpo_ctx* c, float* V, float* pol_angle, uint8_t* pol_thr, double tol_rel, int64_t max_sweeps,
                 int32_t check_every, dpo_stats* st, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V || !pol_angle || !pol_thr) return fail(c, DPO_EINVAL, "null array argument");
  if (max_sweeps < 1 || check_every < 1 || !(tol_rel >= 0)) return fail(c, DPO_EINVAL, "bad max_sweeps / check_every / tol");
  if (c->search.mode == DPO_SEARCH_SEEDED) return fail(c, DPO_EINVAL, "value iteration needs TABLE or SCAN_GOLDEN");
  int rc = ensure_work(c);
  if (rc != DPO_OK) return rc;
  hipStream_t s = S(stream);
  const bool walk = c->search.mode == DPO_SEARCH_TABLE_WALK;
  if (walk && ((rc = ensure_walk(c)) != DPO_OK || (rc = walk_counts_zero(c, s)) != DPO_OK)) return rc;
  dpo_stats local;
  std::memset(&local, 0, sizeof(local));
  const double t0 = now_s();
  HIP_TRY(c, hipMemcpyAsync(c->work, V, sizeof(float) * (size_t)c->N, hipMemcpyDeviceToDevice, s));
  float* cur = V;
  float* nxt = c->work;
  double best = INFINITY;
  int since_best = 0;
  int code = DPO_ENOCONV;
  double h[kPartial] = {0, 0, 0, 0, 0};
  int64_t k = 0;
  while (k < max_sweeps) {
    // only the sweeps that end a check interval compute the residual
    const bool check = (k + 1) % check_every == 0 || k + 1 == max_sweeps;
    // TABLE_WALK: the first sweep searches the full table, later ones walk from the previous angles
    rc = sweep_full(c, cur, nxt, pol_angle, pol_thr, s, false, false, check, walk && k > 0 ? pol_angle : nullptr,
                    true);
    if (rc != DPO_OK) return rc;
    k++;
    std::swap(cur, nxt);
    if (k % check_every == 0 || k == max_sweeps) {
      if ((rc = finish_resid(c, c->resid, s)) != DPO_OK) return rc;
      if ((rc = read_resid(c, h, s)) != DPO_OK) return rc;
      if (h[3] > 0) {
        code = DPO_ENUMERIC;
        fail(c, DPO_ENUMERIC, "value iteration produced non-finite values");
        break;
      }
      if (h[0] < tol_rel) {
        code = DPO_OK;
        local.converged = 1;
        break;
      }
      if (h[0] < best) {
        best = h[0];
        since_best = 0;
      } else if (++since_best >= 64) {
        local.stalled = 1;
        break;
      }
    }
  }
  if (cur != V) HIP_TRY(c, hipMemcpyAsync(V, cur, sizeof(float) * (size_t)c->N, hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  local.sweeps = k;
  local.evals = k * c->n_free * evals_per_full_search(c);
  if (walk) {
    int64_t w = 0;
    if ((rc = walk_counts_read(c, s, &w)) != DPO_OK) return rc;
    local.evals = k * c->n_free + (k > 0 ? c->n_free * c->search.n_angles : 0) + w;
  }
  local.resid_max_rel = h[0];
  local.resid_sum_abs = h[1];
  local.resid_max_abs = h[2];
  local.seconds = now_s() - t0;
  if (st) *st = local;
  if (code == DPO_ENOCONV) fail(c, DPO_ENOCONV, local.stalled ? "value iteration stalled" : "max_sweeps reached");
  return code;
}

int dpo_policy_evaluate(dpo_ctx* c, float* V, const float* pol_angle, const uint8_t* pol_thr, double tol_rel,
                        int32_t max_iter, int64_t* matvecs, double* resid_rel, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V || !pol_angle || !pol_thr) return fail(c, DPO_EINVAL, "null array argument");
  if (!(c->prob.lambda > 0)) return fail(c, DPO_EINVAL, "exact policy evaluation needs lambda > 0");
  if (!(tol_rel > 0) || max_iter < 1) return fail(c, DPO_EINVAL, "tol_rel > 0 and max_iter >= 1");
  double rel = 0;
  int rc = gmres_eval(c, V, pol_angle, pol_thr, tol_rel, max_iter, matvecs, &rel, S(stream));
  if (rc != DPO_OK) return rc;
  if (resid_rel) *resid_rel = rel;
  if (!(rel <= tol_rel)) return fail(c, DPO_ENOCONV, "GMRES did not reach tol_rel within max_iter");
  return DPO_OK;
}

namespace {

// Policy iteration with the evaluation solved exactly (eq:p_eval by GMRES):
// greedy step, stop if its residual is below tol_rel, else evaluate the new
// policy to a node-wise relative residual of kExactEvalTol (at most 300
// operator applications) starting from the greedy values.  float32 floors
// that residual at ~3e-7 where values next to the exit faces carry M.
int solve_pi_exact(dpo_ctx* c, float* V, float* pol_angle, uint8_t* pol_thr, double tol_rel, int64_t max_outer,
                   dpo_stats* st, hipStream_t s) {
  int rc = ensure_work(c);
  if (rc != DPO_OK) return rc;
  dpo_stats local;
  std::memset(&local, 0, sizeof(local));
  const double t0 = now_s();
  HIP_TRY(c, hipMemcpyAsync(c->work, V, sizeof(float) * (size_t)c->N, hipMemcpyDeviceToDevice, s));
  float* cur = V;
  float* nxt = c->work;
  double h[kPartial] = {0, 0, 0, 0, 0};
  int code = DPO_ENOCONV;
  int64_t it = 0, evals = 0, mv_total = 0;
  double full_best = INFINITY;
  int full_stall = 0;
  while (it < max_outer) {
    if ((rc = sweep_full(c, cur, nxt, pol_angle, pol_thr, s, false, it > 0)) != DPO_OK) return rc;
    it++;
    if ((rc = finish_resid(c, c->resid, s)) != DPO_OK) return rc;
    if ((rc = read_resid(c, h, s)) != DPO_OK) return rc;
    evals += c->n_free * evals_per_full_search(c);
    std::swap(cur, nxt);
    if (h[3] > 0) {
      code = DPO_ENUMERIC;
      fail(c, DPO_ENUMERIC, "policy iteration produced non-finite values");
      break;
    }
    if (h[0] < tol_rel) {
      code = DPO_OK;
      local.converged = 1;
      break;
    }
    if (h[0] < full_best) {
      full_best = h[0];
      full_stall = 0;
    } else if (++full_stall >= 32) {
      local.stalled = 1;
      break;
    }
    int64_t mv = 0;
    double rel = 0;
    if ((rc = gmres_eval(c, cur, pol_angle, pol_thr, kExactEvalTol, 300, &mv, &rel, s)) != DPO_OK) return rc;
    mv_total += mv;
    evals += mv * c->n_free;
  }
  if (cur != V) HIP_TRY(c, hipMemcpyAsync(V, cur, sizeof(float) * (size_t)c->N, hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  local.sweeps = it;
  local.eval_sweeps = mv_total;
  local.evals = evals;
  local.resid_max_rel = h[0];
  local.resid_sum_abs = h[1];
  local.resid_max_abs = h[2];
  local.seconds = now_s() - t0;
  if (st) *st = local;
  if (code == DPO_ENOCONV) fail(c, DPO_ENOCONV, local.stalled ? "policy iteration stalled" : "max_outer reached");
  return code;
}

}  // namespace

int dpo_solve_pi(dpo_ctx* c, float* V, float* pol_angle, uint8_t* pol_thr, double tol_rel, int32_t eval_sweeps,
                 int64_t max_outer, const float* seed_angle, dpo_stats* st, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V || !pol_angle || !pol_thr) return fail(c, DPO_EINVAL, "null array argument");
  if (max_outer < 1 || !(tol_rel >= 0)) return fail(c, DPO_EINVAL, "bad max_outer / tol");
  if (eval_sweeps < 0) {
    if (seed_angle) return fail(c, DPO_EINVAL, "exact evaluation (eval_sweeps < 0) takes no seed_angle");
    if (c->search.mode == DPO_SEARCH_SEEDED || c->search.mode == DPO_SEARCH_TABLE_WALK)
      return fail(c, DPO_EINVAL, "exact evaluation needs the TABLE or SCAN_GOLDEN search");
    if (!(c->prob.lambda > 0)) return fail(c, DPO_EINVAL, "exact policy evaluation needs lambda > 0");
    return solve_pi_exact(c, V, pol_angle, pol_thr, tol_rel, max_outer, st, S(stream));
  }
  const bool seeded = seed_angle != nullptr;
  if (seeded && c->search.mode != DPO_SEARCH_SEEDED) return fail(c, DPO_EINVAL, "seed_angle given but search mode is not SEEDED");
  if (!seeded && c->search.mode == DPO_SEARCH_SEEDED) return fail(c, DPO_EINVAL, "SEEDED mode needs seed_angle");
  int rc = ensure_work(c);
  if (rc != DPO_OK) return rc;
  // the evaluation sweeps read the greedy step's foot descriptors where the
  // Euler foot applies, else the policy arrays
  const bool desc = desc_ok(c);
  if (desc && (rc = ensure_desc(c)) != DPO_OK) return rc;
  if ((rc = ensure_pi_buffers(c)) != DPO_OK) return rc;
  hipStream_t s = S(stream);
  const bool walk = c->search.mode == DPO_SEARCH_TABLE_WALK;
  if (walk && ((rc = ensure_walk(c)) != DPO_OK || (rc = walk_counts_zero(c, s)) != DPO_OK)) return rc;
  dpo_stats local;
  std::memset(&local, 0, sizeof(local));
  const double t0 = now_s();
  // Three value buffers: the greedy step writes G; the evaluation sweeps of
  // the step alternate between the other two and are queued before the host
  // reads the greedy residual (which travels back through pinned memory), so
  // the round trip overlaps them.  If the step meets the stop rule, G holds
  // T V and the sweeps queued after it are discarded.
  float* buf[3] = {V, c->work, c->work2};
  HIP_TRY(c, hipMemcpyAsync(buf[1], V, sizeof(float) * (size_t)c->N, hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(buf[2], V, sizeof(float) * (size_t)c->N, hipMemcpyDeviceToDevice, s));
  float* cur = V;
  int code = DPO_ENOCONV;
  double h[kPartial] = {0, 0, 0, 0, 0};
  int64_t it = 0, evals = 0, fallback = 0;
  // Seeded solves run seeded greedy steps until their residual meets tol_rel,
  // then full-search steps until a full step meets it: a local search that
  // settled in the wrong basin is self-consistent (its residual is zero), so
  // only the full search can certify the fixed point.
  bool verify = false;
  double seeded_best = INFINITY, full_best = INFINITY;
  int seeded_stall = 0, full_stall = 0;
  // device time of the greedy sweeps and of the counted evaluation sweeps:
  // events around each, read one step later (by then the stream has passed them)
  double greedy_ms = 0, eval_ms = 0;
  auto span_ms = [&](hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? (double)ms : 0.0;
  };
  bool pending = false, pending_eval = false;  // the previous step's events, not yet read
  int prev = 0;
  while (it < max_outer) {
    float* G = cur == buf[0] ? buf[1] : buf[0];
    hipEvent_t* ev = c->step_ev[it & 1];
    // greedy step: policy improvement together with T V
    const bool use_seed = seeded && it > 0 && !verify;
    HIP_TRY(c, hipEventRecord(ev[0], s));
    if (use_seed) rc = sweep_seeded(c, cur, G, pol_angle, pol_thr, seed_angle, s, desc, true);
    else rc = sweep_full(c, cur, G, pol_angle, pol_thr, s, desc, it > 0, true, walk && it > 0 ? pol_angle : nullptr, true);
    if (rc != DPO_OK) return rc;
    HIP_TRY(c, hipEventRecord(ev[1], s));
    it++;
    if ((rc = finish_resid(c, c->resid, s)) != DPO_OK) return rc;
    HIP_TRY(c, hipMemcpyAsync(c->resid_host, c->resid, sizeof(double) * kPartial, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipEventRecord(c->resid_ready, s));
    // evaluation sweeps of this step, queued ahead of the stop decision
    float* src = G;
    HIP_TRY(c, hipEventRecord(ev[2], s));
    for (int e = 0; e < eval_sweeps; e++) {
      float* dst = nullptr;
      for (float* b : buf)
        if (b != G && b != src) {
          dst = b;
          break;
        }
      rc = desc ? sweep_eval_desc(c, src, dst, s) : sweep_eval(c, src, dst, pol_angle, pol_thr, false, s);
      if (rc != DPO_OK) return rc;
      src = dst;
    }
    HIP_TRY(c, hipEventRecord(ev[3], s));
    HIP_TRY(c, hipEventSynchronize(c->resid_ready));
    if (pending) {
      greedy_ms += span_ms(c->step_ev[prev][0], c->step_ev[prev][1]);
      if (pending_eval) eval_ms += span_ms(c->step_ev[prev][2], c->step_ev[prev][3]);
    }
    pending = true;
    pending_eval = false;
    prev = (int)((it - 1) & 1);
    std::memcpy(h, c->resid_host, sizeof(h));
    cur = G;  // T V, the result if this step stops the solve
    if (use_seed) {
      fallback += (int64_t)h[4];
      evals += c->n_free * (1 + c->search.n_local) + (int64_t)h[4] * evals_per_full_search(c);
    } else {
      // walk steps: coast here, the walk's thrust evaluations from the counters at the end
      evals += c->n_free * (walk && it > 1 ? 1 : evals_per_full_search(c));
      if (seeded && it > 1) local.verify_steps++;
    }
    if (h[3] > 0) {
      code = DPO_ENUMERIC;
      fail(c, DPO_ENUMERIC, "policy iteration produced non-finite values");
      break;
    }
    if (use_seed) {
      // seeds that move with the iterate (warm starts) may never settle:
      // leave the seeded phase after 8 seeded steps without a new best residual
      if (h[0] < seeded_best) {
        seeded_best = h[0];
        seeded_stall = 0;
      } else if (++seeded_stall >= 8) {
        verify = true;
      }
    }
    if (h[0] < tol_rel) {
      if (use_seed) {
        verify = true;
      } else {
        code = DPO_OK;
        local.converged = 1;
        break;
      }
    }
    if (!use_seed) {
      // float32 rounding floors the residual; stop after 32 full steps without a new lowest one
      if (h[0] < full_best) {
        full_best = h[0];
        full_stall = 0;
      } else if (++full_stall >= 32) {
        local.stalled = 1;
        break;
      }
    }
    cur = src;
    local.eval_sweeps += eval_sweeps;
    evals += (int64_t)eval_sweeps * c->n_free;
    pending_eval = eval_sweeps > 0;
  }
  if (cur != V) HIP_TRY(c, hipMemcpyAsync(V, cur, sizeof(float) * (size_t)c->N, hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (pending) {
    greedy_ms += span_ms(c->step_ev[prev][0], c->step_ev[prev][1]);
    if (pending_eval) eval_ms += span_ms(c->step_ev[prev][2], c->step_ev[prev][3]);
  }
  local.greedy_seconds = 1e-3 * greedy_ms;
  local.eval_seconds = 1e-3 * eval_ms;
  if (walk) {
    int64_t w = 0;
    if ((rc = walk_counts_read(c, s, &w)) != DPO_OK) return rc;
    evals += w;
  }
  local.sweeps = it;
  local.evals = evals;
  local.fallback_nodes = fallback;
  local.resid_max_rel = h[0];
  local.resid_sum_abs = h[1];
  local.resid_max_abs = h[2];
  local.seconds = now_s() - t0;
  if (st) *st = local;
  if (code == DPO_ENOCONV) fail(c, DPO_ENOCONV, local.stalled ? "policy iteration stalled" : "max_outer reached");
  return code;
}

int dpo_value_at(dpo_ctx* c, const float* V, const double* x, double* out, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V || !x || !out) return fail(c, DPO_EINVAL, "null argument");
  hipStream_t s = S(stream);
  HIP_TRY(c, launch_value_at(V, c->G, c->prob.M, x, c->resid, s));
  HIP_TRY(c, hipMemcpyAsync(out, c->resid, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  return DPO_OK;
}

int dpo_extract_feedback(dpo_ctx* c, const float* V, const double* states, int64_t n, double tau, float* angle_out,
                         uint8_t* thr_out, float* q_out, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V || !states || !angle_out || !thr_out) return fail(c, DPO_EINVAL, "null array argument");
  if (n < 0 || n > 0x7fffffff) return fail(c, DPO_EINVAL, "bad n");
  if (!(tau > 0)) return fail(c, DPO_EINVAL, "tau must be > 0");
  if (c->search.mode == DPO_SEARCH_SEEDED) return fail(c, DPO_EINVAL, "feedback needs TABLE, SCAN_GOLDEN or TABLE_WALK");
  if (n == 0) return DPO_OK;
  SweepArgs a = base_args(c);
  a.V_in = V;
  HIP_TRY(c, launch_feedback(a, states, (int)n, tau, angle_out, thr_out, q_out, S(stream)));
  return DPO_OK;
}

int dpo_simulate(dpo_ctx* c, const float* V, double* states, int64_t n, double tau, int32_t steps, int32_t substeps,
                 double drag, double* traj, uint8_t* thr_hist, float* ang_hist, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V) return fail(c, DPO_EINVAL, "V is NULL");
  if (n < 0 || n > 0x7fffffff - kBlock) return fail(c, DPO_EINVAL, "bad n");
  if (!(tau > 0) || !std::isfinite(tau)) return fail(c, DPO_EINVAL, "tau must be > 0");
  if (steps < 0 || substeps < 1 || substeps > 4096) return fail(c, DPO_EINVAL, "steps >= 0, substeps in [1, 4096]");
  if (c->search.mode == DPO_SEARCH_SEEDED) return fail(c, DPO_EINVAL, "the closed loop needs TABLE, SCAN_GOLDEN or TABLE_WALK");
  if (!(drag >= 0) || !std::isfinite(drag)) return fail(c, DPO_EINVAL, "drag must be finite and >= 0");
  if (drag != 0 && c->prob.model == DPO_MODEL_EIKONAL) return fail(c, DPO_EINVAL, "drag: orbit models only");
  if (n == 0) return DPO_OK;
  if (!states) return fail(c, DPO_EINVAL, "states is NULL");
  SweepArgs a = base_args(c);
  a.V_in = V;
  HIP_TRY(c, launch_simulate(a, states, (int)n, tau, steps, substeps, drag, traj, thr_hist, ang_hist, S(stream)));
  return DPO_OK;
}

int dpo_mask_from_coarse(dpo_ctx* c, const float* Vc, const dpo_grid* fine, double thresh, const int32_t* dilate,
                         uint8_t* mask, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!Vc || !fine || !dilate || !mask) return fail(c, DPO_EINVAL, "null argument");
  int rc = validate_grid(c, fine);
  if (rc != DPO_OK) return rc;
  if (c->P.model == DPO_MODEL_CROWN) return fail(c, DPO_EINVAL, "mask_from_coarse: not for the crown model");
  for (int k = 0; k < 4; k++) {
    if (fine->lo[k] != c->grid.lo[k] || fine->hi[k] != c->grid.hi[k])
      return fail(c, DPO_EINVAL, "fine grid must share the coarse domain box");
    if (dilate[k] < 0) return fail(c, DPO_EINVAL, "dilate must be >= 0");
  }
  const Grid Gf = make_grid(*fine);
  const int Nf = fine->n[0] * fine->n[1] * fine->n[2] * fine->n[3];
  uint8_t* tmp = nullptr;
  if (hipMalloc(&tmp, (size_t)Nf) != hipSuccess) return fail(c, DPO_ENOMEM, "mask scratch alloc");
  hipStream_t s = S(stream);
  hipError_t e = launch_mask_seed(Vc, c->G, c->prob.M, Gf, thresh, mask, Nf, s);
  for (int k = 0; k < 4 && e == hipSuccess; k++) {
    if (dilate[k] == 0) continue;
    e = launch_dilate_axis(mask, tmp, Gf, k, dilate[k], Nf, s);
    if (e == hipSuccess) e = hipMemcpyAsync(mask, tmp, (size_t)Nf, hipMemcpyDeviceToDevice, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(tmp);
  if (e != hipSuccess) return hip_fail(c, e, "dpo_mask_from_coarse");
  return DPO_OK;
}

int dpo_probe_interp(dpo_ctx* c, const float* V, const float* pts, int64_t n, float* out, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V || !pts || !out) return fail(c, DPO_EINVAL, "null argument");
  if (n < 0 || n > 0x7fffffff) return fail(c, DPO_EINVAL, "bad n");
  if (n == 0) return DPO_OK;
  HIP_TRY(c, launch_probe_interp(V, c->G, c->P.M, pts, (int)n, out, S(stream)));
  return DPO_OK;
}

static int probe_nodes_check(dpo_ctx* c, const int32_t* nodes, int64_t n) {
  if (n < 0 || n > 0x7fffffff) return fail(c, DPO_EINVAL, "bad n");
  // Node indices are read on the device; reject out-of-range ones on the host.
  std::vector<int32_t> h((size_t)n);
  if (n > 0 && hipMemcpy(h.data(), nodes, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, DPO_EHIP, "probe: reading node indices");
  for (int32_t v : h)
    if (v < 0 || v >= c->N) return fail(c, DPO_EINVAL, "probe: node index out of range");
  return DPO_OK;
}

int dpo_probe_q(dpo_ctx* c, const float* V, const int32_t* nodes, const uint8_t* thr, const float* angle, int64_t n,
                float* q_out, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V || !nodes || !thr || !angle || !q_out) return fail(c, DPO_EINVAL, "null argument");
  int rc = probe_nodes_check(c, nodes, n);
  if (rc != DPO_OK || n == 0) return rc;
  SweepArgs a = base_args(c);
  a.V_in = V;
  HIP_TRY(c, launch_probe_q(a, nodes, thr, angle, (int)n, q_out, nullptr, S(stream)));
  return DPO_OK;
}

int dpo_probe_foot(dpo_ctx* c, const int32_t* nodes, const uint8_t* thr, const float* angle, int64_t n,
                   float* off_out, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!nodes || !thr || !angle || !off_out) return fail(c, DPO_EINVAL, "null argument");
  int rc = probe_nodes_check(c, nodes, n);
  if (rc != DPO_OK || n == 0) return rc;
  SweepArgs a = base_args(c);
  HIP_TRY(c, launch_probe_q(a, nodes, thr, angle, (int)n, nullptr, off_out, S(stream)));
  return DPO_OK;
}

/* ---------------------------------------------------------------- machine ceilings */

int dpo_probe_copy(const float* src, float* dst, int64_t n, void* stream) {
  if (!src || !dst) return fail(nullptr, DPO_EINVAL, "dpo_probe_copy: NULL argument");
  if (n < 4 || n % 4 != 0) return fail(nullptr, DPO_EINVAL, "dpo_probe_copy: n must be a positive multiple of 4");
  if (n / 4 > (int64_t)0x7fffffff * 1024) return fail(nullptr, DPO_EINVAL, "dpo_probe_copy: n too large");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u)
    return fail(nullptr, DPO_EINVAL, "dpo_probe_copy: buffers must be 16-byte aligned");
  HIP_TRY(nullptr, launch_ceil_copy(src, dst, n, S(stream)));
  return DPO_OK;
}

int dpo_probe_read(const float* src, int64_t n, float* sink, void* stream) {
  if (!src || !sink) return fail(nullptr, DPO_EINVAL, "dpo_probe_read: NULL argument");
  if (n < 4 || n % 4 != 0) return fail(nullptr, DPO_EINVAL, "dpo_probe_read: n must be a positive multiple of 4");
  if (n / 4 > (int64_t)0x7fffffff * 1024) return fail(nullptr, DPO_EINVAL, "dpo_probe_read: n too large");
  if (reinterpret_cast<uintptr_t>(src) & 15u) return fail(nullptr, DPO_EINVAL, "dpo_probe_read: src must be 16-byte aligned");
  HIP_TRY(nullptr, launch_ceil_read(src, n, sink, S(stream)));
  return DPO_OK;
}

int dpo_probe_fma(int32_t blocks, int32_t iters, float* sink, void* stream) {
  if (!sink) return fail(nullptr, DPO_EINVAL, "dpo_probe_fma: NULL argument");
  if (blocks < 1 || iters < 1) return fail(nullptr, DPO_EINVAL, "dpo_probe_fma: blocks and iters must be >= 1");
  HIP_TRY(nullptr, launch_ceil_fma(blocks, iters, sink, S(stream)));
  return DPO_OK;
}

/* ------------------------------------------------- training pairs for the network */

int dpo_feasible_nodes(dpo_ctx* c, const float* V, double thresh, uint32_t* nodes, int64_t* n_out, void* stream) {
  if (!c || !V || !nodes || !n_out) return fail(c, DPO_EINVAL, "NULL argument");
  if (!std::isfinite(thresh)) return fail(c, DPO_EINVAL, "thresh must be finite");
  const int N = (int)c->N;
  const int nch = compact_chunks(N);
  uint8_t* flag = nullptr;
  int* counts = nullptr;
  int* offsets = nullptr;
  auto release = [&]() {
    if (flag) (void)hipFree(flag);
    if (counts) (void)hipFree(counts);
    if (offsets) (void)hipFree(offsets);
  };
  if (hipMalloc(&flag, (size_t)N) != hipSuccess || hipMalloc(&counts, sizeof(int) * nch) != hipSuccess ||
      hipMalloc(&offsets, sizeof(int) * (nch + 1)) != hipSuccess) {
    release();
    return fail(c, DPO_ENOMEM, "dpo_feasible_nodes: scratch allocation");
  }
  hipError_t e = launch_feasible_flags(c->kind, V, (float)thresh, flag, N, S(stream));
  if (e == hipSuccess) e = launch_compact(c->G, flag, N, counts, offsets, nodes, S(stream));
  int total = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&total, offsets + nch, sizeof(int), hipMemcpyDeviceToHost, S(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(S(stream));
  release();
  if (e != hipSuccess) return hip_fail(c, e, "dpo_feasible_nodes");
  *n_out = total;
  return DPO_OK;
}

int dpo_gather_pairs(dpo_ctx* c, const uint32_t* nodes, int64_t n_nodes, const int32_t* sel, int64_t n,
                     const float* pol_angle, const uint8_t* pol_thr, float* x, float* tgt, void* stream) {
  if (!c || !nodes || !pol_angle || !pol_thr || !x || !tgt || (n > 0 && !sel))
    return fail(c, DPO_EINVAL, "NULL argument");
  if (n < 0 || n > 0x7fffffffLL - kBlock) return fail(c, DPO_EINVAL, "n out of range");
  if (n_nodes < 0 || n_nodes > c->n_free) return fail(c, DPO_EINVAL, "n_nodes must be in [0, n_free]");
  if ((reinterpret_cast<uintptr_t>(x) & 15u) || (reinterpret_cast<uintptr_t>(tgt) & 15u))
    return fail(c, DPO_EINVAL, "x and tgt must be 16-byte aligned");
  for (int64_t t = 0; t < n; t++)
    if (sel[t] < 0 || sel[t] >= n_nodes) return fail(c, DPO_EINVAL, "sel entries must lie in [0, n_nodes)");
  if (n == 0) return DPO_OK;
  int* dsel = nullptr;
  if (hipMalloc(&dsel, sizeof(int) * (size_t)n) != hipSuccess) return fail(c, DPO_ENOMEM, "dpo_gather_pairs");
  hipError_t e = hipMemcpyAsync(dsel, sel, sizeof(int) * (size_t)n, hipMemcpyHostToDevice, S(stream));
  if (e == hipSuccess)
    e = launch_gather_pairs(c->G, nodes, dsel, (int)n, pol_angle, pol_thr, reinterpret_cast<float4*>(x),
                            reinterpret_cast<float4*>(tgt), S(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(S(stream));
  (void)hipFree(dsel);
  if (e != hipSuccess) return hip_fail(c, e, "dpo_gather_pairs");
  return DPO_OK;
}

}  // extern "C"

dpo::CtxView dpo::ctx_view(const dpo_ctx* c) {
  CtxView v;
  v.G = c->G;
  v.free_node = c->free_node;
  v.n_free = c->n_free;
  v.N = c->N;
  v.kind = c->kind;
  return v;
}

// ============================================================ batched solve
// The batch keeps every per-problem array in one concatenated device
// allocation (values A and B, policy, free-node lists, 1/r and thrust
// tables) and a pointer-free record per problem with its offsets.
struct dpo_batch {
  int n = 0;
  std::vector<dpo_ctx*> ctx;
  dpo_search search;
  int mode = 0;
  hipStream_t stream = nullptr;
  std::vector<long long> v_off;  // node offsets (n + 1)
  std::vector<int> free_off;     // free-list offsets (n + 1)
  float* Va = nullptr;
  float* Vb = nullptr;
  float* ang = nullptr;
  uint8_t* thr = nullptr;
  uint32_t* free_all = nullptr;
  double* rinv_all = nullptr;
  float* g_all = nullptr;
  std::vector<BatchProblem> rec;  // host copy of the records (tile_begin per config)
  BatchProblem* d_probs = nullptr;  // records of the running problems, in run order (n)
  int* d_tile_begin = nullptr;  // over the running problems (n + 1)
  int* d_tile_run = nullptr;    // running problem of each tile (partial_cap)
  int* d_run = nullptr;         // running problems (n)
  int* d_done = nullptr;        // per problem: 0 running, 1 converged, 2 non-finite
  double* d_partial = nullptr;
  double* d_resid = nullptr;
  int partial_cap = 0;
  int max_blocks = 0;  // compute units of the device (sizes the persistent-style grid)
  std::string err;
};

namespace {

int bfail(dpo_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  else g_err = msg;
  return code;
}

#define BHIP_TRY(b, call)                                                            \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) return bfail((b), DPO_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Tile table over the running problems for workgroup size `block` (records
// uploaded too); returns the tile count.
int batch_tables(dpo_batch* b, int block, const std::vector<int>& run, int* n_tiles) {
  std::vector<int> tb(run.size() + 1, 0);
  std::vector<BatchProblem> rr(run.size());
  for (size_t k = 0; k < run.size(); k++) {
    b->rec[run[k]].tile_begin = tb[k];
    rr[k] = b->rec[run[k]];
    tb[k + 1] = tb[k] + blocks_for(b->ctx[run[k]]->n_free, block);
  }
  if (tb[run.size()] > b->partial_cap) return bfail(b, DPO_EINVAL, "batch: too many tiles for the partial buffer");
  std::vector<int> tr(std::max(1, tb[run.size()]));
  for (size_t k = 0; k < run.size(); k++)
    std::fill(tr.begin() + tb[k], tr.begin() + tb[k + 1], (int)k);
  BHIP_TRY(b, hipMemcpyAsync(b->d_probs, rr.data(), sizeof(BatchProblem) * rr.size(), hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(b->d_run, run.data(), sizeof(int) * run.size(), hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(b->d_tile_begin, tb.data(), sizeof(int) * tb.size(), hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipMemcpyAsync(b->d_tile_run, tr.data(), sizeof(int) * tb[run.size()], hipMemcpyHostToDevice, b->stream));
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  *n_tiles = tb[run.size()];
  return DPO_OK;
}

BatchArgs batch_args(dpo_batch* b, double tol, int n_run, int n_tiles, bool policy) {
  BatchArgs a;
  std::memset(&a, 0, sizeof(a));
  const dpo_ctx* c0 = b->ctx[0];
  a.probs = b->d_probs;
  a.run = b->d_run;
  a.tile_begin = b->d_tile_begin;
  a.tile_run = b->d_tile_run;
  a.n_run = n_run;
  a.n_tiles = n_tiles;
  a.free_all = b->free_all;
  a.rinv_all = b->rinv_all;
  a.g_all = b->g_all;
  a.Va = b->Va;
  a.Vb = b->Vb;
  a.ang_all = policy ? b->ang : nullptr;
  a.thr_all = policy ? b->thr : nullptr;
  a.tab = c0->tab;
  a.n_ang = c0->n_ang;
  a.n_golden = c0->search.n_golden;
  a.half_width = (float)(2.0 * 3.14159265358979323846 / (double)(c0->search.n_scan > 0 ? c0->search.n_scan : 1));
  a.rot_scan = c0->rot;
  a.done = b->d_done;
  a.partial = b->d_partial;
  a.resid = b->d_resid;
  a.tol = tol;
  return a;
}

// Capture S sweeps over the running problems, then one per-problem stop
// decision on the last sweep's residual, into a graph.  S is even, so every
// replay leaves the last iterate in buffer A.
int batch_graph(dpo_batch* b, const BatchArgs& a, int block, int S, hipGraphExec_t* exec) {
  hipGraph_t g = nullptr;
  BHIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int s = 0; s < S && e == hipSuccess; s++) e = launch_batch_sweep(a, b->mode, block, s & 1, s == S - 1, b->stream);
  if (e == hipSuccess) e = launch_batch_reduce(a, b->stream);
  hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return bfail(b, DPO_EHIP, std::string("batch graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return bfail(b, DPO_EHIP, std::string("batch graph instantiate: ") + hipGetErrorString(e));
  return DPO_OK;
}

// Replays until every problem has stopped or max_sweeps; the graph is
// re-captured over the remaining problems whenever one stops.
int batch_run(dpo_batch* b, double tol, int64_t max_sweeps, int S, int block, bool policy,
              std::vector<int64_t>& sweeps, std::vector<int>& done, int64_t* total) {
  const int n = b->n;
  std::vector<int> run(n);
  for (int p = 0; p < n; p++) run[p] = p;
  sweeps.assign(n, 0);
  done.assign(n, 0);
  BHIP_TRY(b, hipMemsetAsync(b->d_done, 0, sizeof(int) * n, b->stream));
  hipGraphExec_t exec = nullptr;
  int rc = DPO_OK;
  int64_t t = 0;
  while (t < max_sweeps && !run.empty()) {
    if (!exec) {
      int n_tiles = 0;
      if ((rc = batch_tables(b, block, run, &n_tiles)) != DPO_OK) break;
      if ((rc = batch_graph(b, batch_args(b, tol, (int)run.size(), n_tiles, policy), block, S, &exec)) != DPO_OK) break;
    }
    hipError_t e = hipGraphLaunch(exec, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(done.data(), b->d_done, sizeof(int) * n, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
      rc = bfail(b, DPO_EHIP, std::string("batch replay: ") + hipGetErrorString(e));
      break;
    }
    t += S;
    std::vector<int> still;
    for (int p : run) {
      sweeps[p] += S;
      if (done[p] == 0) still.push_back(p);
    }
    if (still.size() != run.size()) {
      hipGraphExecDestroy(exec);
      exec = nullptr;
      run.swap(still);
    }
  }
  if (exec) hipGraphExecDestroy(exec);
  *total = t;
  return rc;
}

int check_batch_cfg(dpo_batch* b, int block, int S) {
  if (block < 64 || block > 512 || block % 64) return bfail(b, DPO_EINVAL, "batch: block must be 64, 128, ..., 512");
  if (S < 2 || S > 256 || (S & 1)) return bfail(b, DPO_EINVAL, "batch: sweeps per graph must be even, in [2, 256]");
  return DPO_OK;
}

// Copy the value functions between the caller's per-problem arrays and the
// concatenated buffer `dst_all` (to_all) or back.
int batch_copy_values(dpo_batch* b, float* const* V, float* all, bool to_all) {
  for (int p = 0; p < b->n; p++) {
    const size_t bytes = sizeof(float) * (size_t)b->ctx[p]->N;
    float* seg = all + b->v_off[p];
    BHIP_TRY(b, hipMemcpyAsync(to_all ? seg : V[p], to_all ? V[p] : seg, bytes, hipMemcpyDeviceToDevice, b->stream));
  }
  return DPO_OK;
}

}  // namespace

extern "C" {

int dpo_batch_create(int32_t n_prob, const dpo_grid* grids, const dpo_problem* probs, const dpo_search* search,
                     dpo_batch** out) {
  if (!out) return bfail(nullptr, DPO_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_prob < 1 || n_prob > 4096 || !grids || !probs || !search) return bfail(nullptr, DPO_EINVAL, "batch: bad arguments");
  if (search->mode != DPO_SEARCH_TABLE && search->mode != DPO_SEARCH_SCAN_GOLDEN)
    return bfail(nullptr, DPO_EINVAL, "batch: search must be TABLE or SCAN_GOLDEN");
  dpo_batch* b = new dpo_batch();
  b->n = n_prob;
  b->search = *search;
  b->mode = search->mode == DPO_SEARCH_TABLE ? 0 : 1;
  auto bail = [&](int code) {
    if (code != DPO_OK) {
      g_err = b->err;
      dpo_batch_destroy(b);
    }
    return code;
  };
  b->v_off.assign(n_prob + 1, 0);
  b->free_off.assign(n_prob + 1, 0);
  std::vector<int> r_off(n_prob + 1, 0), g_off(n_prob + 1, 0);
  long long tiles64 = 0;
  for (int p = 0; p < n_prob; p++) {
    dpo_ctx* c = nullptr;
    int rc = dpo_create(&grids[p], &probs[p], search, nullptr, &c);
    if (rc != DPO_OK) {
      b->err = "batch problem " + std::to_string(p) + ": " + g_err;
      return bail(rc);
    }
    b->ctx.push_back(c);
    if (!c->fast_ok) {
      b->err = "batch problem " + std::to_string(p) + ": the factorised sweep does not apply";
      return bail(DPO_EINVAL);
    }
    b->v_off[p + 1] = b->v_off[p] + c->N;
    b->free_off[p + 1] = b->free_off[p] + (int)c->n_free;
    r_off[p + 1] = r_off[p] + grids[p].n[0];
    g_off[p + 1] = g_off[p] + 2 * grids[p].n[3];
    tiles64 += blocks_for(c->n_free, 64);
  }
  const long long NT = b->v_off[n_prob];
  if (NT > 0x7fffffffLL || b->free_off[n_prob] < 0) {
    b->err = "batch: more than 2^31 nodes in total";
    return bail(DPO_EINVAL);
  }
  b->partial_cap = (int)std::max(1LL, tiles64);
  if (hipMalloc(&b->Va, sizeof(float) * NT) != hipSuccess || hipMalloc(&b->Vb, sizeof(float) * NT) != hipSuccess ||
      hipMalloc(&b->ang, sizeof(float) * NT) != hipSuccess || hipMalloc(&b->thr, (size_t)NT) != hipSuccess ||
      hipMalloc(&b->free_all, sizeof(uint32_t) * std::max(1, b->free_off[n_prob])) != hipSuccess ||
      hipMalloc(&b->rinv_all, sizeof(double) * r_off[n_prob]) != hipSuccess ||
      hipMalloc(&b->g_all, sizeof(float) * g_off[n_prob]) != hipSuccess ||
      hipMalloc(&b->d_probs, sizeof(BatchProblem) * n_prob) != hipSuccess ||
      hipMalloc(&b->d_tile_begin, sizeof(int) * (n_prob + 1)) != hipSuccess ||
      hipMalloc(&b->d_tile_run, sizeof(int) * b->partial_cap) != hipSuccess ||
      hipMalloc(&b->d_run, sizeof(int) * n_prob) != hipSuccess ||
      hipMalloc(&b->d_done, sizeof(int) * n_prob) != hipSuccess ||
      hipMalloc(&b->d_partial, sizeof(double) * kPartial * b->partial_cap) != hipSuccess ||
      hipMalloc(&b->d_resid, sizeof(double) * kPartial * n_prob) != hipSuccess) {
    b->err = "batch: device allocation failed";
    return bail(DPO_ENOMEM);
  }
  b->rec.resize(n_prob);
  for (int p = 0; p < n_prob; p++) {
    dpo_ctx* c = b->ctx[p];
    hipError_t e = hipMemcpy(b->free_all + b->free_off[p], c->free_node, sizeof(uint32_t) * c->n_free, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->rinv_all + r_off[p], c->rinv, sizeof(double) * grids[p].n[0], hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->g_all + g_off[p], c->gtab, sizeof(float) * 2 * grids[p].n[3], hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
      b->err = "batch: table copy failed";
      return bail(DPO_EHIP);
    }
    BatchProblem& R = b->rec[p];
    std::memset(&R, 0, sizeof(R));
    R.G = c->G;
    R.P = c->P;
    R.c0 = c->c0;
    R.c1 = c->c1;
    R.c2 = c->c2;
    R.gm = c->gm;
    R.n_free = (int)c->n_free;
    R.v_off = b->v_off[p];
    R.free_off = b->free_off[p];
    R.rinv_off = r_off[p];
    R.g_off = g_off[p];
  }
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  b->max_blocks = ncu;  // compute units; the grid holds 2048 threads per CU
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    b->err = "batch: stream create";
    return bail(DPO_EHIP);
  }
  *out = b;
  return DPO_OK;
}

void dpo_batch_destroy(dpo_batch* b) {
  if (!b) return;
  if (b->stream) hipStreamSynchronize(b->stream);
  for (dpo_ctx* c : b->ctx) dpo_destroy(c);
  void* bufs[] = {b->Va, b->Vb, b->ang, b->thr, b->free_all, b->rinv_all, b->g_all,
                  b->d_probs, b->d_tile_begin, b->d_tile_run, b->d_run, b->d_done, b->d_partial, b->d_resid};
  for (void* v : bufs)
    if (v) hipFree(v);
  if (b->stream) hipStreamDestroy(b->stream);
  delete b;
}

const char* dpo_batch_last_error(const dpo_batch* b) { return b ? b->err.c_str() : g_err.c_str(); }

int dpo_batch_sizes(const dpo_batch* b, int64_t* n_nodes, int64_t* n_free) {
  if (!b) return bfail(nullptr, DPO_EINVAL, "batch is NULL");
  for (int p = 0; p < b->n; p++) {
    if (n_nodes) n_nodes[p] = b->ctx[p]->N;
    if (n_free) n_free[p] = b->ctx[p]->n_free;
  }
  return DPO_OK;
}

int dpo_batch_init_value(dpo_batch* b, float* const* V, void* stream) {
  if (!b) return bfail(nullptr, DPO_EINVAL, "batch is NULL");
  if (!V) return bfail(b, DPO_EINVAL, "V is NULL");
  for (int p = 0; p < b->n; p++) {
    int rc = dpo_init_value(b->ctx[p], V[p], stream);
    if (rc != DPO_OK) return bfail(b, rc, b->ctx[p]->err);
  }
  return DPO_OK;
}

int dpo_batch_solve_vi(dpo_batch* b, float* const* V, float* const* pol_angle, uint8_t* const* pol_thr, double tol_rel,
                       int64_t max_sweeps, int32_t sweeps_per_graph, int32_t block, dpo_batch_stats* stats,
                       double* seconds, void* stream) {
  if (!b) return bfail(nullptr, DPO_EINVAL, "batch is NULL");
  if (!V) return bfail(b, DPO_EINVAL, "V is NULL");
  for (int p = 0; p < b->n; p++)
    if (!V[p] || (pol_angle && !pol_angle[p]) || (pol_thr && !pol_thr[p])) return bfail(b, DPO_EINVAL, "null array");
  if (max_sweeps < 1 || !(tol_rel >= 0)) return bfail(b, DPO_EINVAL, "bad max_sweeps / tol");
  int rc = check_batch_cfg(b, block, sweeps_per_graph);
  if (rc != DPO_OK) return rc;
  const int n = b->n;
  const bool policy = pol_angle && pol_thr;
  BHIP_TRY(b, hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  const double t0 = now_s();
  if ((rc = batch_copy_values(b, V, b->Va, true)) != DPO_OK) return rc;
  if ((rc = batch_copy_values(b, V, b->Vb, true)) != DPO_OK) return rc;
  std::vector<int64_t> sweeps;
  std::vector<int> done;
  int64_t total = 0;
  if ((rc = batch_run(b, tol_rel, max_sweeps, sweeps_per_graph, block, policy, sweeps, done, &total)) != DPO_OK)
    return rc;
  std::vector<double> res(kPartial * n);
  BHIP_TRY(b, hipMemcpy(res.data(), b->d_resid, sizeof(double) * kPartial * n, hipMemcpyDeviceToHost));
  int code = DPO_OK;
  for (int p = 0; p < n; p++) {
    const size_t N = (size_t)b->ctx[p]->N;
    BHIP_TRY(b, hipMemcpyAsync(V[p], b->Va + b->v_off[p], sizeof(float) * N, hipMemcpyDeviceToDevice, b->stream));
    if (policy) {
      BHIP_TRY(b, hipMemcpyAsync(pol_angle[p], b->ang + b->v_off[p], sizeof(float) * N, hipMemcpyDeviceToDevice, b->stream));
      BHIP_TRY(b, hipMemcpyAsync(pol_thr[p], b->thr + b->v_off[p], N, hipMemcpyDeviceToDevice, b->stream));
    }
    if (done[p] == 2) code = DPO_ENUMERIC;
    else if (done[p] == 0 && code == DPO_OK) code = DPO_ENOCONV;
    if (stats) {
      stats[p].sweeps = sweeps[p];
      stats[p].resid_max_rel = res[kPartial * p + 0];
      stats[p].resid_sum_abs = res[kPartial * p + 1];
      stats[p].resid_max_abs = res[kPartial * p + 2];
      stats[p].converged = done[p] == 1;
      stats[p].status = done[p];
    }
  }
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  if (seconds) *seconds = now_s() - t0;
  if (code == DPO_ENUMERIC) bfail(b, code, "batch: non-finite values");
  else if (code == DPO_ENOCONV) bfail(b, code, "batch: max_sweeps reached");
  return code;
}

int dpo_batch_time_config(dpo_batch* b, int32_t block, int32_t sweeps_per_graph, int32_t replays,
                          double* seconds_per_sweep) {
  if (!b) return bfail(nullptr, DPO_EINVAL, "batch is NULL");
  if (!seconds_per_sweep || replays < 1) return bfail(b, DPO_EINVAL, "bad arguments");
  int rc = check_batch_cfg(b, block, sweeps_per_graph);
  if (rc != DPO_OK) return rc;
  const int n = b->n;
  for (int p = 0; p < n; p++) {
    float* A = b->Va + b->v_off[p];
    hipError_t e = launch_init_value(b->ctx[p]->kind, b->ctx[p]->P.M, A, (int)b->ctx[p]->N, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->Vb + b->v_off[p], A, sizeof(float) * (size_t)b->ctx[p]->N, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return bfail(b, DPO_EHIP, "autotune init");
  }
  std::vector<int> run(n);
  for (int p = 0; p < n; p++) run[p] = p;
  int n_tiles = 0;
  if ((rc = batch_tables(b, block, run, &n_tiles)) != DPO_OK) return rc;
  BHIP_TRY(b, hipMemsetAsync(b->d_done, 0, sizeof(int) * n, b->stream));
  hipGraphExec_t exec = nullptr;
  if ((rc = batch_graph(b, batch_args(b, -1.0, n, n_tiles, false), block, sweeps_per_graph, &exec)) != DPO_OK) return rc;
  // replays as the solver issues them: graph, read-back of the stop flags, sync
  std::vector<int> flags(n, 0);
  hipError_t e = hipGraphLaunch(exec, b->stream);  // warm-up
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  const double t0 = now_s();
  for (int r = 0; r < replays && e == hipSuccess; r++) {
    e = hipGraphLaunch(exec, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), b->d_done, sizeof(int) * n, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  }
  const double elapsed = now_s() - t0;
  hipGraphExecDestroy(exec);
  hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, DPO_EHIP, std::string("autotune timing: ") + hipGetErrorString(e));
  *seconds_per_sweep = elapsed / ((double)replays * sweeps_per_graph);
  return DPO_OK;
}

int dpo_batch_solve_sequential(dpo_batch* b, float* const* V, float* const* pol_angle, uint8_t* const* pol_thr,
                               double tol_rel, int64_t max_sweeps, int32_t check_every, dpo_batch_stats* stats,
                               double* seconds, void* stream) {
  if (!b) return bfail(nullptr, DPO_EINVAL, "batch is NULL");
  if (!V || !pol_angle || !pol_thr) return bfail(b, DPO_EINVAL, "null array");
  const double t0 = now_s();
  int code = DPO_OK;
  for (int p = 0; p < b->n; p++) {
    dpo_stats st;
    int rc = dpo_solve_vi(b->ctx[p], V[p], pol_angle[p], pol_thr[p], tol_rel, max_sweeps, check_every, &st, stream);
    if (rc < 0) return bfail(b, rc, b->ctx[p]->err);
    if (rc == DPO_ENOCONV && code == DPO_OK) code = DPO_ENOCONV;
    if (stats) {
      stats[p].sweeps = st.sweeps;
      stats[p].resid_max_rel = st.resid_max_rel;
      stats[p].resid_sum_abs = st.resid_sum_abs;
      stats[p].resid_max_abs = st.resid_max_abs;
      stats[p].converged = st.converged;
      stats[p].status = st.converged ? 1 : 0;
    }
  }
  if (seconds) *seconds = now_s() - t0;
  return code;
}

}  // extern "C"

/* ------------------------------------------- frozen-policy sweep without allocation
 * For callers that cannot allocate device memory (code under graph capture,
 * serving loops, harnesses that forbid hipMalloc): the per-workgroup FP64
 * residual partials of the frozen-policy sweep and the first stage of their
 * reduction live in a file-scope device array instead of the context's
 * buffer.  Each device holds its own copy of the array for the life of the
 * process; host code reaches it only through the address hipGetSymbolAddress
 * returns on that device, taken once per device on the entry point's first
 * call there. */
namespace {

constexpr int kStaticMaxBlocks = 262144;  // workgroups of one sweep: up to 67,108,864 free nodes
constexpr size_t kStaticScratch = (size_t)kPartial * (kStaticMaxBlocks + kResidStage);

__device__ __align__(256) double scratch[kStaticScratch];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (nullptr and a message on error).
double* static_scratch(dpo_ctx* c) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    fail(c, DPO_EHIP, "no current device for the static scratch");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      hip_fail(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int dpo_policy_eval_sweep_static(dpo_ctx* c, const float* V_in, float* V_out, const float* pol_angle,
                                 const uint8_t* pol_thr, double* resid, void* stream) {
  if (!c) return fail(nullptr, DPO_EINVAL, "ctx is NULL");
  if (!V_in || !V_out || !pol_angle || !pol_thr) return fail(c, DPO_EINVAL, "null array argument");
  if (V_in == V_out) return fail(c, DPO_EINVAL, "V_in and V_out must differ (Jacobi sweep)");
  const bool brick = use_brick_policy(c);
  const int nb = brick ? brick_blocks(c) : blocks_for(c->n_free, kBlock);
  if (blocks_for(c->n_free, kBlock) > kStaticMaxBlocks || nb > kStaticMaxBlocks)
    return fail(c, DPO_EINVAL, "dpo_policy_eval_sweep_static: more than 67,108,864 free nodes "
                               "(the static scratch holds 262,144 workgroup partials)");
  double* ptr = static_scratch(c);
  if (!ptr) return DPO_EHIP;
  hipStream_t s = S(stream);
  SweepArgs a = base_args(c);
  a.V_in = V_in;
  a.V_out = V_out;
  a.pol_ang_in = pol_angle;
  a.pol_thr_in = pol_thr;
  a.partial = ptr;
  if (c->n_free > 0) {
    if (brick) HIP_TRY(c, launch_eval_brick(a, c->brick, c->kind, resid != nullptr, false, s));
    else HIP_TRY(c, launch_policy_eval(a, resid != nullptr, s));
  }
  // every workgroup writes its partial before the reduction reads it, so the
  // array needs no clearing; with no free node the reduction of zero
  // partials writes the zeros (a kernel, not a memset)
  if (resid)
    HIP_TRY(c, launch_resid_final(ptr, c->n_free > 0 ? nb : 0, ptr + (size_t)kPartial * kStaticMaxBlocks, resid, s));
  return DPO_OK;
}

}  // extern "C"
