// Device-side wavelet/prox helpers and the pass launchers used by the solver.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace expenc {

// Analysis filters (low-pass h, high-pass g[k] = (-1)^k h[M-1-k]) kept in
// FP64: rounding the irrational db4 taps to FP32 makes the transform
// slightly non-orthonormal, and FISTA's momentum accumulates that bias
// (about 1e-5 relative after 50 iterations), so the passes filter in FP64.
struct FilterSet {
  int taps;
  double h[8];
  double g[8];
};

// Soft-threshold of one complex coefficient: w * max(0, 1 - tau/|w|)
// (evaluated in FP64 so that the threshold carries no FP32 rounding bias).
// 1/|w| is the hardware reciprocal square root of |w|^2 refined by one
// Newton step, y (1 + (1 - |w|^2 y^2) / 2), which is accurate to a few FP64
// ulps, far below the FP32 rounding of the result; |w| > tau is tested as
// |w|^2 > tau^2.  NaN input stays NaN (0 * NaN).  |w|^2 of FP32 components
// is zero or above 1e-90, so the reciprocal square root never sees an FP64
// subnormal.
__device__ inline float2 soft(float2 v, double t) {
  const double m2 = (double)v.x * v.x + (double)v.y * v.y;
  const double y0 = __builtin_amdgcn_rsq(m2);
  const double y = fma(0.5 * y0, fma(-m2 * y0, y0, 1.0), y0);
  const double sc = m2 > t * t ? 1.0 - t * y : 0.0;
  return make_float2((float)(v.x * sc), (float)(v.y * sc));
}

int make_filter_set(int32_t wavelet, FilterSet *f);

// Multi-level analysis of src into w ([B][ny][nx]); w may equal src.  When
// tau (device, [B]) is given the detail coefficients are soft-thresholded as
// they are produced, and when l1_part is given the per-block sums of the
// thresholded detail moduli go to l1_part[level][b][block] (l1_stride blocks).
int dwt_forward_levels(const FilterSet &f, int nx, int ny, int levels, int batch, const float2 *src,
                       float2 *w, const double *tau, double *l1_part, int l1_stride, hipStream_t s);
// Multi-level synthesis, in place on w except the last row pass, which writes
// dst; if zout is given it also writes zout = dst + beta*(dst - xprev).
int dwt_inverse_levels(const FilterSet &f, int nx, int ny, int levels, int batch, float2 *w, float2 *dst,
                       const float2 *xprev, float2 *zout, double beta, hipStream_t s);

// One FISTA proximal step with its momentum, on the fused-level kernels
// (each level's row and column passes in one launch over 2D tiles staged in
// LDS): w = S_tau(W v) (thresholded detail bands), x_k = W^H w and
// z = x_k + beta (x_k - x_prev), for nimg images of nx x ny ([nimg][ny][nx],
// row stride nx).  The intermediate low-pass blocks ping-pong between v and
// x_k, both of which are overwritten (x_k with the result); x_prev and z must
// be other buffers.  l1_part (optional) receives per-tile FP64 sums of the
// thresholded detail moduli at [level][image][tile] (l1_stride tiles, see
// dwt2_tiles).  status (optional): flagged if x_k holds NaN or Inf.
int dwt2_prox(const FilterSet &f, int nx, int ny, int levels, int nimg, float2 *v, float2 *w, float2 *xk,
              const float2 *xprev, float2 *z, double beta, const double *tau, double *l1_part, int l1_stride,
              hipStream_t s, unsigned *status = nullptr);
// Number of analysis tiles of level j (its l1 partial sums).
int dwt2_tiles(int nx, int ny, int level);

}  // namespace expenc
