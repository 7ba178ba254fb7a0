// Wavelet transform W of eq. 1 and the soft-threshold proximal step.
//
// Periodised, orthonormal, separable 2D transform with the Mallat layout.
// One level on a periodic line v of even length n:
//   a[m] = sum_k h[k] v[(2m+k) mod n],  d[m] = sum_k g[k] v[(2m+k) mod n],
//   g[k] = (-1)^k h[M-1-k];
// rows first, then columns, on the current top-left low-pass block.  The
// inverse is the transpose: v[m] = sum over taps k with k = m (mod 2) of
// h[k] a[i] + g[k] d[i], i = ((m-k) mod n)/2.
//
// Each pass is one launch that stages whole lines in LDS and writes them back
// in place, so a multi-level transform needs no scratch buffer.  Row passes
// use one workgroup per image row (a coalesced line of n complex values);
// column passes stage a strip of 16 columns x n rows (128-byte coalesced
// row segments); taps and sums are FP64, data FP32.  The column pass of the analysis can apply the
// soft-threshold to every detail coefficient it produces, because a level's
// detail bands are final once its column pass is done.  These are HBM /
// launch-bound kernels: no MFMA.
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"
#include "wavelet_dev.h"

namespace expenc {

// ---------------------------------------------------------------------------
// Filters (host): Haar, and Daubechies with p = 4 vanishing moments by
// spectral factorisation of P(y) = sum_{k<p} C(p-1+k, k) y^k, where
// |m0(w)|^2 = cos^{2p}(w/2) P(sin^2(w/2)) and y = (2 - z - 1/z)/4.  Each root
// y_k of P gives z^2 - (2 - 4 y_k) z + 1 = 0; the root with |z| < 1 is kept,
// so H(z) = sum h[n] z^-n has its non-trivial zeros inside the unit circle.
// ---------------------------------------------------------------------------

static std::vector<std::complex<double>> poly_roots(const std::vector<double> &asc) {
  // Durand-Kerner iteration on the monic polynomial with ascending coefficients asc.
  const int n = (int)asc.size() - 1;
  std::vector<std::complex<double>> c(n + 1);
  for (int i = 0; i <= n; ++i) c[i] = asc[i] / asc[n];
  std::vector<std::complex<double>> z(n);
  const std::complex<double> seed(0.4, 0.9);
  for (int i = 0; i < n; ++i) z[i] = std::pow(seed, i);
  for (int it = 0; it < 500; ++it) {
    double delta = 0;
    for (int i = 0; i < n; ++i) {
      std::complex<double> num = c[n];
      for (int k = n - 1; k >= 0; --k) num = num * z[i] + c[k];
      std::complex<double> den = 1.0;
      for (int j = 0; j < n; ++j)
        if (j != i) den *= (z[i] - z[j]);
      std::complex<double> step = num / den;
      z[i] -= step;
      delta = std::max(delta, std::abs(step));
    }
    if (delta < 1e-17) break;
  }
  return z;
}

int wavelet_filter(int32_t wavelet, double *h, int *taps) {
  if (wavelet == EXPENC_HAAR) {
    h[0] = h[1] = 1.0 / std::sqrt(2.0);
    *taps = 2;
    return EXPENC_OK;
  }
  if (wavelet != EXPENC_DB4) return fail(EXPENC_EINVAL, "unknown wavelet %d", wavelet);
  const int p = 4;
  std::vector<double> pasc(p);
  for (int k = 0; k < p; ++k) {
    double binom = 1;  // C(p-1+k, k)
    for (int i = 1; i <= k; ++i) binom = binom * (p - 1 + i) / i;
    pasc[k] = binom;
  }
  auto yr = poly_roots(pasc);
  // descending-power polynomial (1+z)^p prod (z - z_k)
  std::vector<std::complex<double>> poly{1.0};
  auto mul = [&](std::complex<double> a0, std::complex<double> a1) {  // times (a0*z + a1)
    std::vector<std::complex<double>> out(poly.size() + 1, 0.0);
    for (size_t i = 0; i < poly.size(); ++i) {
      out[i] += poly[i] * a0;
      out[i + 1] += poly[i] * a1;
    }
    poly.swap(out);
  };
  for (int i = 0; i < p; ++i) mul(1.0, 1.0);
  for (auto yk : yr) {
    std::complex<double> b = 2.0 - 4.0 * yk;
    std::complex<double> disc = std::sqrt(b * b - 4.0);
    std::complex<double> z1 = (b + disc) / 2.0, z2 = (b - disc) / 2.0;
    mul(1.0, -(std::abs(z1) < 1.0 ? z1 : z2));
  }
  double sum = 0;
  for (auto &c : poly) sum += c.real();
  for (int i = 0; i < 2 * p; ++i) h[i] = poly[i].real() / sum * std::sqrt(2.0);
  *taps = 2 * p;
  return EXPENC_OK;
}

int make_filter_set(int32_t wavelet, FilterSet *f) {
  double h[16];
  int taps = 0;
  EX_TRY(wavelet_filter(wavelet, h, &taps));
  f->taps = taps;
  for (int k = 0; k < taps; ++k) {
    f->h[k] = h[k];
    f->g[k] = ((k & 1) ? -1.0 : 1.0) * h[taps - 1 - k];
  }
  return EXPENC_OK;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Analysis along rows of the top-left my x mx block.  src/dst: [B][ny][nx]
// with row stride nx (elements); src may equal dst (the line is staged in
// LDS before any store).  One workgroup per (row, image).
__global__ __launch_bounds__(256) void k_dwt_rows(const float2 *src, float2 *dst,
                                                  int nx, int ny, int mx, FilterSet f) {
  extern __shared__ float2 line[];
  const int row = blockIdx.x, b = blockIdx.y;
  const float2 *s = src + ((int64_t)b * ny + row) * nx;
  float2 *d = dst + ((int64_t)b * ny + row) * nx;
  for (int i = threadIdx.x; i < mx; i += blockDim.x) line[i] = s[i];
  __syncthreads();
  const int half = mx >> 1;
  for (int m = threadIdx.x; m < half; m += blockDim.x) {
    double ax = 0.0, ay = 0.0, dx = 0.0, dy = 0.0;
    for (int k = 0; k < f.taps; ++k) {
      int j = 2 * m + k;
      if (j >= mx) j -= mx;
      if (j >= mx) j %= mx;
      const float2 v = line[j];
      ax = fma(f.h[k], (double)v.x, ax);
      ay = fma(f.h[k], (double)v.y, ay);
      dx = fma(f.g[k], (double)v.x, dx);
      dy = fma(f.g[k], (double)v.y, dy);
    }
    d[m] = make_float2((float)ax, (float)ay);
    d[half + m] = make_float2((float)dx, (float)dy);
  }
}

// Synthesis along rows (inverse of k_dwt_rows).  Optionally fused FISTA
// momentum: out = x_k; z = x_k + beta*(x_k - x_prev).
__global__ __launch_bounds__(256) void k_idwt_rows(const float2 *src, float2 *dst,
                                                   int nx, int ny, int mx, FilterSet f,
                                                   const float2 *__restrict__ xprev,
                                                   float2 *__restrict__ zout, double beta) {
  extern __shared__ float2 line[];
  const int row = blockIdx.x, b = blockIdx.y;
  const int64_t base = ((int64_t)b * ny + row) * nx;
  for (int i = threadIdx.x; i < mx; i += blockDim.x) line[i] = src[base + i];
  __syncthreads();
  const int half = mx >> 1;
  for (int m = threadIdx.x; m < mx; m += blockDim.x) {
    double vx = 0.0, vy = 0.0;
    for (int k = (m & 1); k < f.taps; k += 2) {
      int q = m - k;
      q %= mx;
      if (q < 0) q += mx;
      const int i = q >> 1;
      const float2 a = line[i], d = line[half + i];
      vx = fma(f.g[k], (double)d.x, fma(f.h[k], (double)a.x, vx));
      vy = fma(f.g[k], (double)d.y, fma(f.h[k], (double)a.y, vy));
    }
    const float2 v = make_float2((float)vx, (float)vy);
    dst[base + m] = v;
    if (zout) {
      const float2 p = xprev[base + m];
      zout[base + m] = make_float2((float)(v.x + beta * ((double)v.x - p.x)), (float)(v.y + beta * ((double)v.y - p.y)));
    }
  }
}

// Analysis along columns of the top-left my x mx block, in place, 16
// columns per workgroup.  If tau != nullptr, every detail coefficient of
// this level (outputs outside the next LL block) is soft-thresholded with
// tau[b], and if l1 != nullptr the sum of their moduli after thresholding is
// added (FP64) into l1_part[b][blockIdx.x] (for the objective).
__global__ __launch_bounds__(256) void k_dwt_cols(float2 *__restrict__ w, int nx, int ny, int mx, int my,
                                                  FilterSet f, const double *__restrict__ tau,
                                                  double *__restrict__ l1_part, int l1_stride) {
  extern __shared__ float2 strip[];  // [my][16]
  const int b = blockIdx.y;
  const int x0 = blockIdx.x * 16;
  const int cx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int ncols = min(16, mx - x0);
  float2 *img = w + (int64_t)b * ny * nx;
  for (int i = ty; i < my; i += 16)
    if (cx < ncols) strip[i * 16 + cx] = img[(int64_t)i * nx + x0 + cx];
  __syncthreads();
  const int half = my >> 1;
  const double t = tau ? tau[b] : 0.0;
  double l1 = 0.0;
  if (cx < ncols) {
    const bool detail_col = (x0 + cx) >= (mx >> 1);
    for (int m = ty; m < half; m += 16) {
      double ax = 0.0, ay = 0.0, dx = 0.0, dy = 0.0;
      for (int k = 0; k < f.taps; ++k) {
        int j = 2 * m + k;
        if (j >= my) j %= my;
        const float2 v = strip[j * 16 + cx];
        ax = fma(f.h[k], (double)v.x, ax);
        ay = fma(f.h[k], (double)v.y, ay);
        dx = fma(f.g[k], (double)v.x, dx);
        dy = fma(f.g[k], (double)v.y, dy);
      }
      float2 a = make_float2((float)ax, (float)ay), dd = make_float2((float)dx, (float)dy);
      if (tau) {
        if (detail_col) {
          a = soft(a, t);
          l1 += sqrt((double)a.x * a.x + (double)a.y * a.y);
        }
        dd = soft(dd, t);
        l1 += sqrt((double)dd.x * dd.x + (double)dd.y * dd.y);
      }
      img[(int64_t)m * nx + x0 + cx] = a;
      img[(int64_t)(half + m) * nx + x0 + cx] = dd;
    }
  }
  if (l1_part) {
    // block reduction in fixed order
    __shared__ double red[256];
    red[threadIdx.x] = l1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) l1_part[(int64_t)b * l1_stride + blockIdx.x] = red[0];
  }
}

// Synthesis along columns, in place.
__global__ __launch_bounds__(256) void k_idwt_cols(float2 *__restrict__ w, int nx, int ny, int mx, int my,
                                                   FilterSet f) {
  extern __shared__ float2 strip[];
  const int b = blockIdx.y;
  const int x0 = blockIdx.x * 16;
  const int cx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int ncols = min(16, mx - x0);
  float2 *img = w + (int64_t)b * ny * nx;
  for (int i = ty; i < my; i += 16)
    if (cx < ncols) strip[i * 16 + cx] = img[(int64_t)i * nx + x0 + cx];
  __syncthreads();
  const int half = my >> 1;
  if (cx < ncols) {
    for (int m = ty; m < my; m += 16) {
      double vx = 0.0, vy = 0.0;
      for (int k = (m & 1); k < f.taps; k += 2) {
        int q = (m - k) % my;
        if (q < 0) q += my;
        const int i = q >> 1;
        const float2 a = strip[i * 16 + cx], d = strip[(half + i) * 16 + cx];
        vx = fma(f.g[k], (double)d.x, fma(f.h[k], (double)a.x, vx));
        vy = fma(f.g[k], (double)d.y, fma(f.h[k], (double)a.y, vy));
      }
      img[(int64_t)m * nx + x0 + cx] = make_float2((float)vx, (float)vy);
    }
  }
}

// ---------------------------------------------------------------------------
// Fused-level kernels of the solver's proximal step.  A level's row and
// column passes run in one launch over 2D tiles: the periodic input region
// of a tile (its outputs' footprint plus taps - 2 rows and columns) is staged
// in LDS, the row pass writes its FP32 results to LDS, and the column pass
// produces the tile's outputs.  The arithmetic (FP64 sums over the taps in
// the same order, FP32 between the passes) is that of the per-pass kernels
// above.  Levels read and write different buffers, so tiles never race.
// ---------------------------------------------------------------------------

constexpr int kTapsMax = 8;
constexpr int kFwdTX = 16, kFwdTY = 8;  // analysis tile: coefficient positions per band
constexpr int kInvTX = 32, kInvTY = 16;  // synthesis tile: output pixels (x, y)

// i mod n for i in [-n, 2n) with two compares; other i (a level narrower
// than a tile's footprint) take the general remainder.
__device__ inline int wrap(int i, int n) {
  if (i < 0) i += n;
  if (i >= n) i -= n;
  if (i < 0 || i >= n) {
    i %= n;
    if (i < 0) i += n;
  }
  return i;
}

// wrap for an index known to lie in [-n, 2n) (FAST: two selects, no
// branch), else the general form
template <bool FAST>
__device__ inline int wrap_in(int i, int n) {
  if constexpr (FAST) {
    i += i < 0 ? n : 0;
    i -= i >= n ? n : 0;
    return i;
  } else {
    return wrap(i, n);
  }
}

__device__ inline double2 widen(float2 v) { return make_double2(v.x, v.y); }

// Staging of a level's input footprint (RY x RX from row 2 ty0, column
// 2 tx0, periodic) into LDS: every load is issued before the first LDS store
// and none sits under a branch, so a thread waits for memory once.  The tail
// index is clamped (a repeated load, not stored).
template <int RY, int RX, bool FAST>
__device__ inline void stage_analysis(const float2 *__restrict__ in, int istride, int tx0, int ty0, int mx, int my,
                                      float2 (*dst)[RX]) {
  constexpr int NIN = RY * RX, NLD = (NIN + 255) / 256;
  float2 ld[NLD];
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int i = min((int)threadIdx.x + 256 * k, NIN - 1);
    const int r = i / RX, c = i - r * RX;
    ld[k] = in[(int64_t)wrap_in<FAST>(2 * ty0 + r, my) * istride + wrap_in<FAST>(2 * tx0 + c, mx)];
  }
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i < NIN) dst[i / RX][i % RX] = ld[k];
  }
}

// Staging of a synthesis tile's coefficients: NY x NX of each quarter (LL
// from ll, the detail bands from w's level block) into sc [2 NY][2 NX] in
// FP64, loads first as above.
template <int NY, int NX, bool FAST>
__device__ inline void stage_synthesis(const float2 *__restrict__ llb, int lstride, const float2 *__restrict__ wb,
                                       int nx, int i0, int j0, int hx, int hy, double2 (*sc)[2 * NX]) {
  constexpr int NIN = 4 * NY * NX, NLD = (NIN + 255) / 256;
  float2 ld[NLD];
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int i = min((int)threadIdx.x + 256 * k, NIN - 1);
    const int r = i / (2 * NX), c = i - r * (2 * NX);
    const bool rh = r >= NY, ch = c >= NX;
    const int gy = wrap_in<FAST>(i0 + (rh ? r - NY : r), hy), gx = wrap_in<FAST>(j0 + (ch ? c - NX : c), hx);
    const float2 *src = (!rh && !ch) ? llb + (int64_t)gy * lstride + gx
                                     : wb + (int64_t)(rh ? hy + gy : gy) * nx + (ch ? hx + gx : gx);
    ld[k] = *src;
  }
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i < NIN) {
      const int r = i / (2 * NX), c = i - r * (2 * NX);
      sc[r][c] = widen(ld[k]);
    }
  }
}
// FP32 rounding of an intermediate pass result, kept in FP64 form
__device__ inline double2 round32(double x, double y) { return make_double2((float)x, (float)y); }

// Analysis of one level: in (mx x my, row stride istride, image pitch
// ipitch) -> LL to ll (hx x hy, row stride lstride, pitch lpitch) and the
// three detail bands into w's level block (row stride nx, pitch wpitch),
// soft-thresholded with tau[image] when tau is given; l1_part[image][tile]
// receives the FP64 sum of the thresholded detail moduli when given.
// Block: 256 threads; grid (ceil(hx/16), ceil(hy/8), images).  TAPS (2 or 8)
// fixes the tile's footprint at compile time.
template <int TAPS>
__global__ __launch_bounds__(256) void k_dwt2_level(const float2 *__restrict__ in, int istride, int64_t ipitch,
                                                    float2 *__restrict__ ll, int lstride, int64_t lpitch,
                                                    float2 *__restrict__ w, int nx, int64_t wpitch, int mx, int my,
                                                    FilterSet f, const double *__restrict__ tau,
                                                    double *__restrict__ l1_part, int l1_stride) {
  constexpr int RY = 2 * kFwdTY + TAPS - 2, RX = 2 * kFwdTX + TAPS - 2;
  __shared__ float2 sin_[RY][RX];
  __shared__ float2 slo[RY][kFwdTX], shi[RY][kFwdTX];
  __shared__ double red[256];
  const int b = blockIdx.z;
  const int hx = mx >> 1, hy = my >> 1;
  const int tx0 = blockIdx.x * kFwdTX, ty0 = blockIdx.y * kFwdTY;
  in += b * ipitch;
  // footprint rows 2 ty0 .. 2 ty0 + RY - 1 < 2 my (and columns) when the
  // level is at least as large as the footprint
  if (RY <= my && RX <= mx)
    stage_analysis<RY, RX, true>(in, istride, tx0, ty0, mx, my, sin_);
  else
    stage_analysis<RY, RX, false>(in, istride, tx0, ty0, mx, my, sin_);
  __syncthreads();
  // rows: low and high outputs at tile column x for every staged row
  for (int i = threadIdx.x; i < RY * kFwdTX; i += blockDim.x) {
    const int r = i / kFwdTX, x = i % kFwdTX;
    double ax = 0.0, ay = 0.0, dx = 0.0, dy = 0.0;
#pragma unroll
    for (int k = 0; k < TAPS; ++k) {
      const float2 v = sin_[r][2 * x + k];
      ax = fma(f.h[k], (double)v.x, ax);
      ay = fma(f.h[k], (double)v.y, ay);
      dx = fma(f.g[k], (double)v.x, dx);
      dy = fma(f.g[k], (double)v.y, dy);
    }
    slo[r][x] = make_float2((float)ax, (float)ay);
    shi[r][x] = make_float2((float)dx, (float)dy);
  }
  __syncthreads();
  // columns: thread = (x part: low/high, row y, column x) of the tile
  const int part = threadIdx.x >> 7, y = (threadIdx.x >> 4) & 7, x = threadIdx.x & 15;
  const int oy = ty0 + y, ox = tx0 + x;
  double l1 = 0.0;
  if (oy < hy && ox < hx) {
    double ax = 0.0, ay = 0.0, dx = 0.0, dy = 0.0;
#pragma unroll
    for (int k = 0; k < TAPS; ++k) {
      const float2 v = part ? shi[2 * y + k][x] : slo[2 * y + k][x];
      ax = fma(f.h[k], (double)v.x, ax);
      ay = fma(f.h[k], (double)v.y, ay);
      dx = fma(f.g[k], (double)v.x, dx);
      dy = fma(f.g[k], (double)v.y, dy);
    }
    float2 a = make_float2((float)ax, (float)ay), dd = make_float2((float)dx, (float)dy);
    if (tau) {
      const double t = tau[b];
      if (part) {
        a = soft(a, t);
        l1 += sqrt((double)a.x * a.x + (double)a.y * a.y);
      }
      dd = soft(dd, t);
      l1 += sqrt((double)dd.x * dd.x + (double)dd.y * dd.y);
    }
    float2 *wb = w + b * wpitch;
    if (part)
      wb[(int64_t)oy * nx + hx + ox] = a;                  // x high, y low
    else
      ll[b * lpitch + (int64_t)oy * lstride + ox] = a;     // low / low
    wb[(int64_t)(hy + oy) * nx + (part ? hx : 0) + ox] = dd;  // y high
  }
  if (l1_part) {
    red[threadIdx.x] = l1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) l1_part[(int64_t)b * l1_stride + blockIdx.y * gridDim.x + blockIdx.x] = red[0];
  }
}

// Synthesis of one level (columns, then rows): LL from ll (hx x hy, row
// stride lstride, pitch lpitch) and the detail bands from w's level block
// (row stride nx, pitch wpitch) -> out (mx x my, row stride ostride, pitch
// opitch); with zout, also zout = out + beta (out - xprev) (out's layout).
// Output pixels 2i and 2i + 1 (along either axis) are sums over the same
// TAPS/2 coefficients i - TAPS/2 + 1 .. i of each half, with the even and
// the odd taps respectively, so one thread forms both members of such a
// pair: a 32 x 16 output tile needs 16 + TAPS/2 - 1 coefficient columns
// and 8 + TAPS/2 - 1 coefficient rows of each half, staged in FP64.
// Block: 256 threads (16 rows x 16 pairs in the row pass); grid
// (ceil(mx/32), ceil(my/16), images).
template <int TAPS>
__global__ __launch_bounds__(256) void k_idwt2_level(const float2 *__restrict__ ll, int lstride, int64_t lpitch,
                                                     const float2 *__restrict__ w, int nx, int64_t wpitch,
                                                     float2 *__restrict__ out, int ostride, int64_t opitch, int mx,
                                                     int my, FilterSet f, const float2 *__restrict__ xprev,
                                                     float2 *__restrict__ zout, double beta, unsigned *status) {
  constexpr int H = TAPS / 2;
  constexpr int NY = kInvTY / 2 + H - 1, NX = kInvTX / 2 + H - 1;
  __shared__ double2 sc[2 * NY][2 * NX];  // [low | high rows][low | high columns]
  __shared__ double2 cp[kInvTY][2 * NX];  // column-pass output rows (FP32 values)
  const int b = blockIdx.z;
  const int hx = mx >> 1, hy = my >> 1;
  const int m0 = blockIdx.y * kInvTY, n0 = blockIdx.x * kInvTX;
  const int i0 = m0 / 2 - H + 1, j0 = n0 / 2 - H + 1;
  const float2 *wb = w + b * wpitch;
  // coefficient rows i0 .. i0 + NY - 1 lie in [-hy, 2 hy) (and columns)
  // when the level is at least as large as the footprint (i0 >= 1 - H)
  if (NY <= hy && NX <= hx)
    stage_synthesis<NY, NX, true>(ll + b * lpitch, lstride, wb, nx, i0, j0, hx, hy, sc);
  else
    stage_synthesis<NY, NX, false>(ll + b * lpitch, lstride, wb, nx, i0, j0, hx, hy, sc);
  __syncthreads();
  // columns: output rows 2p, 2p + 1 at every staged column
  for (int i = threadIdx.x; i < (kInvTY / 2) * 2 * NX; i += blockDim.x) {
    const int p = i / (2 * NX), c = i - p * (2 * NX);
    double ex = 0.0, ey = 0.0, ox = 0.0, oy = 0.0;
#pragma unroll
    for (int kk = 0; kk < H; ++kk) {
      const double2 a = sc[p + H - 1 - kk][c], d = sc[NY + p + H - 1 - kk][c];
      ex = fma(f.g[2 * kk], d.x, fma(f.h[2 * kk], a.x, ex));
      ey = fma(f.g[2 * kk], d.y, fma(f.h[2 * kk], a.y, ey));
      ox = fma(f.g[2 * kk + 1], d.x, fma(f.h[2 * kk + 1], a.x, ox));
      oy = fma(f.g[2 * kk + 1], d.y, fma(f.h[2 * kk + 1], a.y, oy));
    }
    cp[2 * p][c] = round32(ex, ey);
    cp[2 * p + 1][c] = round32(ox, oy);
  }
  __syncthreads();
  // rows: output pixels 2q, 2q + 1 of row ml (one pair per thread)
  const int ml = threadIdx.x >> 4, q = threadIdx.x & 15;
  const int m = m0 + ml, n = n0 + 2 * q;
  if (m < my && n < mx) {
    double ex = 0.0, ey = 0.0, ox = 0.0, oy = 0.0;
#pragma unroll
    for (int kk = 0; kk < H; ++kk) {
      const double2 a = cp[ml][q + H - 1 - kk], d = cp[ml][NX + q + H - 1 - kk];
      ex = fma(f.g[2 * kk], d.x, fma(f.h[2 * kk], a.x, ex));
      ey = fma(f.g[2 * kk], d.y, fma(f.h[2 * kk], a.y, ey));
      ox = fma(f.g[2 * kk + 1], d.x, fma(f.h[2 * kk + 1], a.x, ox));
      oy = fma(f.g[2 * kk + 1], d.y, fma(f.h[2 * kk + 1], a.y, oy));
    }
    const float2 v0 = make_float2((float)ex, (float)ey), v1 = make_float2((float)ox, (float)oy);
    const int64_t o = b * opitch + (int64_t)m * ostride + n;
    out[o] = v0;
    out[o + 1] = v1;
    flag_nonfinite(status, v0);
    flag_nonfinite(status, v1);
    if (zout) {
      const float2 p0 = xprev[o], p1 = xprev[o + 1];
      zout[o] = make_float2((float)(v0.x + beta * ((double)v0.x - p0.x)),
                            (float)(v0.y + beta * ((double)v0.y - p0.y)));
      zout[o + 1] = make_float2((float)(v1.x + beta * ((double)v1.x - p1.x)),
                                (float)(v1.y + beta * ((double)v1.y - p1.y)));
    }
  }
}

__global__ void k_soft(const float2 *__restrict__ in, float2 *__restrict__ out, int nx, int ny, int llx,
                       int lly, int64_t total, float tau) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t p = i % ((int64_t)nx * ny);
  const int yy = (int)(p / nx), xx = (int)(p % nx);
  float2 v = in[i];
  if (!(yy < lly && xx < llx)) v = soft(v, (double)tau);
  out[i] = v;
}

// grad_in = a g + b u Re(conj(u) g) on detail coefficients with |w| > tau,
// 0 where |w| <= tau, g on the coarsest LL block.
__global__ void k_soft_vjp(const float2 *__restrict__ w, const float2 *__restrict__ g, float2 *__restrict__ out,
                           int nx, int ny, int llx, int lly, int64_t total, float tau) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t p = i % ((int64_t)nx * ny);
  const int yy = (int)(p / nx), xx = (int)(p % nx);
  const float2 gv = g[i];
  if (yy < lly && xx < llx) {
    out[i] = gv;
    return;
  }
  const float2 v = w[i];
  const float m = sqrtf(v.x * v.x + v.y * v.y);
  if (!(m > tau)) {
    out[i] = make_float2(0.f, 0.f);
    return;
  }
  const float a = 1.f - tau / m, b = tau / m;
  const float ux = v.x / m, uy = v.y / m;
  const float re = ux * gv.x + uy * gv.y;  // Re(conj(u) g)
  out[i] = make_float2(a * gv.x + b * ux * re, a * gv.y + b * uy * re);
}

__global__ void k_copy2(const float2 *__restrict__ in, float2 *__restrict__ out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static int check_grid(int32_t nx, int32_t ny, int32_t levels, int32_t batch) {
  if (nx < 2 || ny < 2 || levels < 1 || levels > 12 || batch < 1)
    return fail(EXPENC_EINVAL, "bad wavelet grid %dx%d levels %d batch %d", nx, ny, levels, batch);
  if ((nx % (1 << levels)) || (ny % (1 << levels)))
    return fail(EXPENC_EINVAL, "grid %dx%d is not a multiple of 2^%d", nx, ny, levels);
  if (nx > 4096 || ny > 512) return fail(EXPENC_EUNSUPPORTED, "wavelet grid larger than 4096 x 512");
  return EXPENC_OK;
}

int dwt_forward_levels(const FilterSet &f, int nx, int ny, int levels, int batch, const float2 *src,
                       float2 *w, const double *tau, double *l1_part, int l1_stride, hipStream_t s) {
  for (int j = 0; j < levels; ++j) {
    const int mx = nx >> j, my = ny >> j;
    k_dwt_rows<<<dim3(my, batch), 256, mx * sizeof(float2), s>>>(j == 0 ? src : w, w, nx, ny, mx, f);
    EX_LAUNCHED("dwt rows");
    const int nb = (int)ceil_div(mx, 16);
    double *lp = l1_part ? l1_part + (int64_t)j * batch * l1_stride : nullptr;
    k_dwt_cols<<<dim3(nb, batch), 256, my * 16 * sizeof(float2), s>>>(w, nx, ny, mx, my, f, tau, lp, l1_stride);
    EX_LAUNCHED("dwt cols");
  }
  return EXPENC_OK;
}

int dwt_inverse_levels(const FilterSet &f, int nx, int ny, int levels, int batch, float2 *w, float2 *dst,
                       const float2 *xprev, float2 *zout, double beta, hipStream_t s) {
  for (int j = levels - 1; j >= 0; --j) {
    const int mx = nx >> j, my = ny >> j;
    const int nb = (int)ceil_div(mx, 16);
    k_idwt_cols<<<dim3(nb, batch), 256, my * 16 * sizeof(float2), s>>>(w, nx, ny, mx, my, f);
    EX_LAUNCHED("idwt cols");
    const bool last = (j == 0);
    k_idwt_rows<<<dim3(my, batch), 256, mx * sizeof(float2), s>>>(w, last ? dst : w, nx, ny, mx, f,
                                                                   last ? xprev : nullptr,
                                                                   last ? zout : nullptr, beta);
    EX_LAUNCHED("idwt rows");
  }
  return EXPENC_OK;
}

int dwt2_tiles(int nx, int ny, int level) {
  const int hx = (nx >> level) >> 1, hy = (ny >> level) >> 1;
  return (int)(ceil_div(hx, kFwdTX) * ceil_div(hy, kFwdTY));
}

// Buffer roles: analysis level j reads LL_j (v for j = 0, else x_k for odd j
// and v for even j) and writes LL_{j+1} to the other one (w's top-left block
// for the last level); synthesis level j reads LL_{j+1} (w for the last
// level, else v for odd j+1 and x_k for even j+1) and writes LL_j to the
// other one, x_k itself for j = 0.  Every launch therefore reads and writes
// different buffers.
int dwt2_prox(const FilterSet &f, int nx, int ny, int levels, int nimg, float2 *v, float2 *w, float2 *xk,
              const float2 *xprev, float2 *z, double beta, const double *tau, double *l1_part, int l1_stride,
              hipStream_t s, unsigned *status) {
  if (f.taps != 2 && f.taps != kTapsMax) return fail(EXPENC_EUNSUPPORTED, "filters of %d taps", f.taps);
  if (nx % (1 << levels) || ny % (1 << levels)) return fail(EXPENC_EINVAL, "grid not a multiple of 2^levels");
  const int64_t pitch = (int64_t)nx * ny;
  auto fwd_buf = [&](int j) { return (j & 1) ? xk : v; };  // LL_j of the analysis, j >= 1
  auto inv_buf = [&](int j) { return (j & 1) ? v : xk; };  // LL_j of the synthesis, j >= 1
  for (int j = 0; j < levels; ++j) {
    const int mx = nx >> j, my = ny >> j;
    const float2 *in = j == 0 ? v : fwd_buf(j);
    const int istride = j == 0 ? nx : mx;
    const bool last = j + 1 == levels;
    float2 *ll = last ? w : fwd_buf(j + 1);
    const int lstride = last ? nx : mx >> 1;
    dim3 grid((unsigned)ceil_div(mx >> 1, kFwdTX), (unsigned)ceil_div(my >> 1, kFwdTY), (unsigned)nimg);
    double *lp = l1_part ? l1_part + (int64_t)j * nimg * l1_stride : nullptr;
    if (f.taps == 2)
      k_dwt2_level<2><<<grid, 256, 0, s>>>(in, istride, pitch, ll, lstride, pitch, w, nx, pitch, mx, my, f, tau, lp,
                                           l1_stride);
    else
      k_dwt2_level<8><<<grid, 256, 0, s>>>(in, istride, pitch, ll, lstride, pitch, w, nx, pitch, mx, my, f, tau, lp,
                                           l1_stride);
    EX_LAUNCHED("dwt level");
  }
  for (int j = levels - 1; j >= 0; --j) {
    const int mx = nx >> j, my = ny >> j;
    const bool top = j + 1 == levels;
    const float2 *ll = top ? w : inv_buf(j + 1);
    const int lstride = top ? nx : mx >> 1;
    float2 *out = j == 0 ? xk : inv_buf(j);
    const int ostride = j == 0 ? nx : mx;
    dim3 grid((unsigned)ceil_div(mx, kInvTX), (unsigned)ceil_div(my, kInvTY), (unsigned)nimg);
    const float2 *xp = j == 0 ? xprev : nullptr;
    float2 *zo = j == 0 ? z : nullptr;
    unsigned *st = j == 0 ? status : nullptr;
    if (f.taps == 2)
      k_idwt2_level<2><<<grid, 256, 0, s>>>(ll, lstride, pitch, w, nx, pitch, out, ostride, pitch, mx, my, f, xp, zo,
                                            beta, st);
    else
      k_idwt2_level<8><<<grid, 256, 0, s>>>(ll, lstride, pitch, w, nx, pitch, out, ostride, pitch, mx, my, f, xp, zo,
                                            beta, st);
    EX_LAUNCHED("idwt level");
  }
  return EXPENC_OK;
}

}  // namespace expenc

using namespace expenc;

extern "C" int wavelet_fwd(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch,
                           const float *x, float *w, void *stream) {
  EX_TRY(check_grid(nx, ny, levels, batch));
  if (!x || !w) return fail(EXPENC_EINVAL, "NULL array");
  FilterSet f;
  EX_TRY(make_filter_set(wavelet, &f));
  return dwt_forward_levels(f, nx, ny, levels, batch, reinterpret_cast<const float2 *>(x),
                            reinterpret_cast<float2 *>(w), nullptr, nullptr, 0, (hipStream_t)stream);
}

extern "C" int wavelet_inv(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch,
                           const float *w, float *x, void *stream) {
  EX_TRY(check_grid(nx, ny, levels, batch));
  if (!x || !w) return fail(EXPENC_EINVAL, "NULL array");
  FilterSet f;
  EX_TRY(make_filter_set(wavelet, &f));
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = (int64_t)nx * ny * batch;
  if (x != w) {
    k_copy2<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(reinterpret_cast<const float2 *>(w),
                                                      reinterpret_cast<float2 *>(x), n);
    EX_LAUNCHED("copy");
  }
  float2 *xx = reinterpret_cast<float2 *>(x);
  return dwt_inverse_levels(f, nx, ny, levels, batch, xx, xx, nullptr, nullptr, 0.0, s);
}

extern "C" int wavelet_prox(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch, float *v,
                            float *w, float *x, const float *x_prev, float *z, double beta, const double *tau,
                            void *stream) {
  EX_TRY(check_grid(nx, ny, levels, batch));
  if (batch > 65535) return fail(EXPENC_EINVAL, "batch %d > 65535", batch);
  if (!v || !w || !x || !x_prev || !z || !tau) return fail(EXPENC_EINVAL, "NULL array");
  if (v == w || v == x || w == x || x_prev == v || x_prev == w || x_prev == x || z == v || z == w || z == x ||
      z == x_prev)
    return fail(EXPENC_EINVAL, "v, w, x, x_prev and z must be distinct buffers");
  FilterSet f;
  EX_TRY(make_filter_set(wavelet, &f));
  return dwt2_prox(f, nx, ny, levels, batch, reinterpret_cast<float2 *>(v), reinterpret_cast<float2 *>(w),
                   reinterpret_cast<float2 *>(x), reinterpret_cast<const float2 *>(x_prev),
                   reinterpret_cast<float2 *>(z), beta, tau, nullptr, 0, (hipStream_t)stream);
}

extern "C" int soft_threshold(int32_t nx, int32_t ny, int32_t levels, int32_t batch, const float *w_in,
                              float *w_out, float tau, void *stream) {
  if (nx < 1 || ny < 1 || levels < 0 || batch < 1 || !w_in || !w_out || !(tau >= 0.f))
    return fail(EXPENC_EINVAL, "bad soft_threshold arguments");
  const int64_t total = (int64_t)nx * ny * batch;
  k_soft<<<(unsigned)ceil_div(total, 256), 256, 0, (hipStream_t)stream>>>(
      reinterpret_cast<const float2 *>(w_in), reinterpret_cast<float2 *>(w_out), nx, ny, nx >> levels,
      ny >> levels, total, tau);
  EX_LAUNCHED("soft_threshold");
  return EXPENC_OK;
}

extern "C" int soft_threshold_vjp(int32_t nx, int32_t ny, int32_t levels, int32_t batch, const float *w_in,
                                  const float *g, float *grad_in, float tau, void *stream) {
  if (nx < 1 || ny < 1 || levels < 0 || batch < 1 || !w_in || !g || !grad_in || !(tau >= 0.f))
    return fail(EXPENC_EINVAL, "bad soft_threshold_vjp arguments");
  const int64_t total = (int64_t)nx * ny * batch;
  k_soft_vjp<<<(unsigned)ceil_div(total, 256), 256, 0, (hipStream_t)stream>>>(
      reinterpret_cast<const float2 *>(w_in), reinterpret_cast<const float2 *>(g), reinterpret_cast<float2 *>(grad_in),
      nx, ny, nx >> levels, ny >> levels, total, tau);
  EX_LAUNCHED("soft_threshold_vjp");
  return EXPENC_OK;
}
