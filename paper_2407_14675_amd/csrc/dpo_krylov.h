// Internal interface of the exact policy evaluation kernels (GMRES on
// eq:p_eval, paper Section 3).
#pragma once

#include <algorithm>

#include "dpo_kernels.h"

namespace dpo {

constexpr int kDotGroup = 8;        // basis vectors per pass of the dot-product kernel
constexpr int kMaxBasis = 64;       // largest Krylov basis (restart length + 1)
constexpr int kStreamBlocks = 1024; // workgroups of the vector kernels (grid-stride loops)

// y = exp(-lambda dt) P x at free nodes (frozen policy a.pol_ang_in / a.pol_thr_in)
hipError_t launch_eval_hom(const SweepArgs& a, const float* x, float* y, hipStream_t s);
// r = b - x + y
hipError_t launch_residual(const float* b, const float* x, const float* y, float* r, int N, hipStream_t s);
// w = v - y, then out[i] = <basis_i, w> in FP64 for i < k <= kDotGroup, in one pass
// (partial: kStreamBlocks * kDotGroup doubles)
hipError_t launch_sub_dots(const float* v, const float* y, float* w, const float* basis, int k, size_t ld, int N,
                           double* partial, double* out, hipStream_t s);
// out[i] = <basis_i, w> in FP64 for i < k (partial: kStreamBlocks * kDotGroup doubles)
hipError_t launch_dots(const float* basis, int k, size_t ld, const float* w, int N, double* partial, double* out,
                       hipStream_t s);
// out[0] = max_j |r_j| / max(1, |x_j|) (partial: kStreamBlocks doubles)
hipError_t launch_relmax(const float* r, const float* x, int N, double* partial, double* out, hipStream_t s);
// w -= sum_i coef[i] basis_i, i < k <= kMaxBasis; with nrm_out (device, one
// double; partial: kStreamBlocks * kDotGroup doubles) also |w|^2 of the result
hipError_t launch_axpys(float* w, const float* basis, int k, size_t ld, const double* coef, int N, hipStream_t s,
                       double* partial = nullptr, double* nrm_out = nullptr);
// dst = s * src
hipError_t launch_scale(const float* src, double s, float* dst, int N, hipStream_t st);
// dst = (*sc) * src, the factor read from device memory
hipError_t launch_scale_dev(const float* src, const double* sc, float* dst, int N, hipStream_t s);
// column k of the Arnoldi process and its Givens rotation, on the device (see k_arnoldi_col)
hipError_t launch_arnoldi_col(int k, int m, const double* d, const double* nrm2, double* H, double* cs, double* sn,
                              double* g, double* inv_hn, double* status, hipStream_t s);
// dst[j] = src[j] at the free nodes j
hipError_t launch_free_copy(const SweepArgs& a, const float* src, float* dst, hipStream_t s);
// dst[j] = 0 at the free nodes j
hipError_t launch_free_zero(const SweepArgs& a, float* dst, hipStream_t s);

}  // namespace dpo
