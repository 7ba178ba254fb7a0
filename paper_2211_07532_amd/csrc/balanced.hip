// The paper's regulariser (Methods 2.1, Supporting Information S1): the
// undecimated wavelet transform, one weight per level set to sigma/2 from
// the histogram of the level's high-pass coefficients of W A^H y, and
// balanced FISTA.
//
// Undecimated ("a trous") periodised separable transform, J levels, any
// image size: level j (step d = 2^j) produces from u the bands
//   b0 = lo_y hi_x u,  b1 = hi_y lo_x u,  b2 = hi_y hi_x u,  LL = lo_y lo_x u
// with 1D filters f(u)[i] = 2^-1/2 sum_k f[k] u[(i + d k) mod n]; the last
// LL is kept.  Coefficients are laid out [B][3J+1][ny][nx] (level j in
// bands 3j .. 3j+2, the low pass last).  With orthonormal filters W is a
// tight frame: W^H W = I.  Each level is one pass in which every thread
// forms one pixel's four outputs from its (taps x taps) neighbourhood with
// FP64 accumulation; W^H is the gather-form adjoint.
//
// Balanced model on the coefficients alpha:
//   F = ||A W^H alpha - y||^2 + kappa/2 ||(I - W W^H) alpha||^2 + sum_b lambda_b ||alpha_b||_1,
// FISTA with step 1/L, L = L_A + kappa, L_A = 2 lambda_max(A^H A); per
// iteration x_b = W^H beta, r = A^H (A x_b - y), c = 2 r - kappa x_b and
//   alpha = S_tau(beta - (W c + kappa beta) / L),
// so each iteration costs one A, one A^H, one W and one W^H.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "reduce.h"
#include "wavelet_dev.h"

namespace expenc {

namespace {

constexpr int kBins = 256;

// i mod n for i within one period of [0, n) with two compares; others (taps
// spanning more than the image) take the general remainder
__device__ inline int wrap_i(int i, int n) {
  if (i >= n) i -= n;
  if (i < 0) i += n;
  if (i < 0 || i >= n) {
    i %= n;
    if (i < 0) i += n;
  }
  return i;
}

// One analysis level at tap spacing d: the four bands of pixel i from its
// TAPS x TAPS neighbourhood (FP64 sums in the same order for every band).
// The wrapped row and column indices are formed once per pixel.
template <int TAPS>
__global__ __launch_bounds__(256) void k_swt_level(const float2 *__restrict__ u, int64_t ustride, float2 *__restrict__ bands,
                            int64_t bstride, float2 *__restrict__ llout, int64_t lstride, int nx, int ny, int d,
                            FilterSet f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny;
  if (i >= N) return;
  const int b = blockIdx.y;
  u += b * ustride;
  bands += b * bstride;
  llout += b * lstride;
  const int yy = (int)(i / nx), xx = (int)(i % nx);
  int cols[TAPS];
#pragma unroll
  for (int k = 0; k < TAPS; ++k) cols[k] = wrap_i(xx + d * k, nx);
  double s0x = 0, s0y = 0, s1x = 0, s1y = 0, s2x = 0, s2y = 0, slx = 0, sly = 0;
#pragma unroll 1
  for (int ky = 0; ky < TAPS; ++ky) {
    const float2 *urow = u + (int64_t)wrap_i(yy + d * ky, ny) * nx;
    const double hy = f.h[ky], gy = f.g[ky];
#pragma unroll
    for (int kx = 0; kx < TAPS; ++kx) {
      const float2 v = urow[cols[kx]];
      const double hx = f.h[kx], gx = f.g[kx];
      const double w0 = gx * hy, w1 = hx * gy, w2 = gx * gy, wl = hx * hy;
      s0x += w0 * v.x, s0y += w0 * v.y;
      s1x += w1 * v.x, s1y += w1 * v.y;
      s2x += w2 * v.x, s2y += w2 * v.y;
      slx += wl * v.x, sly += wl * v.y;
    }
  }
  bands[i] = make_float2((float)(0.5 * s0x), (float)(0.5 * s0y));
  bands[N + i] = make_float2((float)(0.5 * s1x), (float)(0.5 * s1y));
  bands[2 * N + i] = make_float2((float)(0.5 * s2x), (float)(0.5 * s2y));
  llout[i] = make_float2((float)(0.5 * slx), (float)(0.5 * sly));
}

// The adjoint of one level: pixel i from the four bands at the TAPS x TAPS
// neighbours i - d k.
template <int TAPS>
__global__ __launch_bounds__(256) void k_iswt_level(const float2 *__restrict__ bands, int64_t bstride, const float2 *__restrict__ ll,
                             int64_t lstride, float2 *__restrict__ u, int64_t ustride, int nx, int ny, int d,
                             FilterSet f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)nx * ny;
  if (i >= N) return;
  const int b = blockIdx.y;
  bands += b * bstride;
  ll += b * lstride;
  u += b * ustride;
  const int yy = (int)(i / nx), xx = (int)(i % nx);
  int cols[TAPS];
#pragma unroll
  for (int k = 0; k < TAPS; ++k) cols[k] = wrap_i(xx - d * k, nx);
  double sx = 0.0, sy = 0.0;
#pragma unroll 1
  for (int ky = 0; ky < TAPS; ++ky) {
    const int64_t row = (int64_t)wrap_i(yy - d * ky, ny) * nx;
    const double hy = f.h[ky], gy = f.g[ky];
#pragma unroll
    for (int kx = 0; kx < TAPS; ++kx) {
      const int64_t o = row + cols[kx];
      const double hx = f.h[kx], gx = f.g[kx];
      const float2 a0 = bands[o], a1 = bands[N + o], a2 = bands[2 * N + o], al = ll[o];
      const double w0 = gx * hy, w1 = hx * gy, w2 = gx * gy, wl = hx * hy;
      sx += w0 * a0.x + w1 * a1.x + w2 * a2.x + wl * al.x;
      sy += w0 * a0.y + w1 * a1.y + w2 * a2.y + wl * al.y;
    }
  }
  u[i] = make_float2((float)(0.5 * sx), (float)(0.5 * sy));
}

// part[(b*J + j) * nblk + blk] = partial sums of |w| over level j's 3 bands
__global__ __launch_bounds__(256) void k_level_abs_part(const float2 *__restrict__ w, int64_t N, int nb, int J,
                                                        double *__restrict__ part) {
  __shared__ double red[256];
  const int j = blockIdx.y, b = blockIdx.z;
  const float2 *p = w + ((int64_t)b * nb + 3 * j) * N;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * N; i += (int64_t)gridDim.x * blockDim.x)
    s += sqrt((double)p[i].x * p[i].x + (double)p[i].y * p[i].y);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[((int64_t)b * J + j) * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_zero_u32(unsigned *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// counts[(b*J + j)][k] += #{ |w| in [k, k+1) * width },  width = 4 mean / 256
__global__ __launch_bounds__(256) void k_level_hist(const float2 *__restrict__ w, int64_t N, int nb, int J,
                                                    const double *__restrict__ mean, unsigned *__restrict__ counts) {
  __shared__ unsigned h[kBins];
  const int j = blockIdx.y, b = blockIdx.z;
  h[threadIdx.x] = 0u;
  __syncthreads();
  const double width = 4.0 * mean[b * J + j] / kBins;
  if (width > 0.0) {
    const float2 *p = w + ((int64_t)b * nb + 3 * j) * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * N;
         i += (int64_t)gridDim.x * blockDim.x) {
      const double m = sqrt((double)p[i].x * p[i].x + (double)p[i].y * p[i].y);
      const double q = floor(m / width);
      if (q < kBins) atomicAdd(&h[(int)q], 1u);
    }
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&counts[((int64_t)b * J + j) * kBins + threadIdx.x], h[threadIdx.x]);
}

// lam[b][3j..3j+2] = scale * sigma/2, sigma = centre of the fullest bin
// (lowest index on ties); lam[b][3J] = 0
__global__ void k_level_mode(const unsigned *__restrict__ counts, const double *__restrict__ mean, int J, int nb,
                             double scale, double *__restrict__ lam) {
  const int bj = blockIdx.x;
  const int b = bj / J, j = bj % J;
  if (threadIdx.x != 0) return;
  const unsigned *c = counts + (int64_t)bj * kBins;
  int best = 0;
  for (int k = 1; k < kBins; ++k)
    if (c[k] > c[best]) best = k;
  const double width = 4.0 * mean[bj] / kBins;
  const double sigma = (best + 0.5) * width;
  for (int q = 0; q < 3; ++q) lam[(int64_t)b * nb + 3 * j + q] = scale * 0.5 * sigma;
  if (j == 0) lam[(int64_t)b * nb + 3 * J] = 0.0;
}

__global__ void k_set_scalar(double *p, double v) {
  if (threadIdx.x == 0) p[0] = v;
}

// sc[1] = kappa (or L_A when kappa < 0), sc[2] = L = L_A + kappa
__global__ void k_bal_scalars(double *sc, double kappa) {
  if (threadIdx.x == 0) {
    sc[1] = kappa >= 0.0 ? kappa : sc[0];
    sc[2] = sc[0] + sc[1];
  }
}

__global__ void k_bal_tau(const double *__restrict__ sc, const double *__restrict__ lam, double *__restrict__ tau,
                          int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) tau[i] = sc[2] > 0.0 ? lam[i] / sc[2] : 0.0;
}

__global__ void k_copy_lam(const double *__restrict__ in, double *__restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

__global__ void k_zero_c(float2 *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_float2(0.f, 0.f);
}

// c = 2 r - kappa x
__global__ void k_bal_combine(const float2 *__restrict__ r, const float2 *__restrict__ x,
                              const double *__restrict__ sc, float2 *__restrict__ c, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double k = sc[1];
  c[i] = make_float2((float)(2.0 * r[i].x - k * x[i].x), (float)(2.0 * r[i].y - k * x[i].y));
}

// alpha = S_tau(beta - (gw + kappa beta)/L) per band (no threshold where tau = 0),
// beta <- alpha + m (alpha - alpha_prev)
__global__ void k_bal_update(float2 *__restrict__ beta, const float2 *__restrict__ gw,
                             const float2 *__restrict__ alpha_prev, float2 *__restrict__ alpha,
                             const double *__restrict__ sc, const double *__restrict__ tau, int nb, int64_t N,
                             int64_t total, double m, unsigned *status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t bb = i / N;  // (image, band)
  const double t = tau[bb];
  const double k = sc[1], invL = sc[2] > 0.0 ? 1.0 / sc[2] : 0.0;
  const float2 be = beta[i], g = gw[i];
  const double vx = be.x - (g.x + k * be.x) * invL, vy = be.y - (g.y + k * be.y) * invL;
  double ax = vx, ay = vy;
  if (t > 0.0) {
    const double mag = sqrt(vx * vx + vy * vy);
    const double scl = mag > t ? 1.0 - t / mag : 0.0;
    ax *= scl;
    ay *= scl;
  }
  const float2 na = make_float2((float)ax, (float)ay);
  alpha[i] = na;
  flag_nonfinite(status, na);
  const float2 ap = alpha_prev[i];
  beta[i] = make_float2((float)(na.x + m * ((double)na.x - ap.x)), (float)(na.y + m * ((double)na.y - ap.y)));
}

int check_swt(int nx, int ny, int levels, int batch) {
  if (nx < 1 || ny < 1 || batch < 1 || levels < 1 || levels > 8)
    return fail(EXPENC_EINVAL, "bad undecimated transform shape %dx%d, levels %d, batch %d", nx, ny, levels, batch);
  if ((int64_t)nx * ny > (1 << 26)) return fail(EXPENC_EINVAL, "image too large");
  if (batch > 65535) return fail(EXPENC_EINVAL, "batch too large");
  return EXPENC_OK;
}

}  // namespace

// x [B][ny][nx] -> w [B][3J+1][ny][nx]; tmp: 2 x B x N scratch (J > 1)
int swt_forward(const FilterSet &f, int nx, int ny, int J, int B, const float2 *x, float2 *w, float2 *tmp,
                hipStream_t s) {
  const int64_t N = (int64_t)nx * ny;
  const int nb = 3 * J + 1;
  const dim3 grid((unsigned)ceil_div(N, 256), (unsigned)B);
  const float2 *u = x;
  int64_t us = N;
  for (int j = 0; j < J; ++j) {
    float2 *ll = (j == J - 1) ? w + (int64_t)3 * J * N : tmp + (int64_t)(j % 2) * B * N;
    const int64_t ls = (j == J - 1) ? nb * N : N;
    if (f.taps == 2)
      k_swt_level<2><<<grid, 256, 0, s>>>(u, us, w + (int64_t)3 * j * N, nb * N, ll, ls, nx, ny, 1 << j, f);
    else
      k_swt_level<8><<<grid, 256, 0, s>>>(u, us, w + (int64_t)3 * j * N, nb * N, ll, ls, nx, ny, 1 << j, f);
    EX_LAUNCHED("undecimated analysis");
    u = ll;
    us = ls;
  }
  return EXPENC_OK;
}

// w [B][3J+1][ny][nx] -> x [B][ny][nx] (W^H)
int swt_adjoint(const FilterSet &f, int nx, int ny, int J, int B, const float2 *w, float2 *x, float2 *tmp,
                hipStream_t s) {
  const int64_t N = (int64_t)nx * ny;
  const int nb = 3 * J + 1;
  const dim3 grid((unsigned)ceil_div(N, 256), (unsigned)B);
  const float2 *ll = w + (int64_t)3 * J * N;
  int64_t ls = nb * N;
  for (int j = J - 1; j >= 0; --j) {
    float2 *u = (j == 0) ? x : tmp + (int64_t)(j % 2) * B * N;
    if (f.taps == 2)
      k_iswt_level<2><<<grid, 256, 0, s>>>(w + (int64_t)3 * j * N, nb * N, ll, ls, u, N, nx, ny, 1 << j, f);
    else
      k_iswt_level<8><<<grid, 256, 0, s>>>(w + (int64_t)3 * j * N, nb * N, ll, ls, u, N, nx, ny, 1 << j, f);
    EX_LAUNCHED("undecimated synthesis");
    ll = u;
    ls = N;
  }
  return EXPENC_OK;
}

// lam [B][3J+1] from the coefficients w; part >= B*J*kRedBlocks doubles,
// mean >= B*J doubles, counts >= B*J*256
int sigma_weights(const float2 *w, int nx, int ny, int J, int B, double scale, double *part, double *mean,
                  unsigned *counts, double *lam, hipStream_t s) {
  const int64_t N = (int64_t)nx * ny;
  const int nb = 3 * J + 1;
  k_level_abs_part<<<dim3(kRedBlocks, J, B), 256, 0, s>>>(w, N, nb, J, part);
  EX_LAUNCHED("level magnitudes");
  EX_TRY(reduce_sum_parts(part, kRedBlocks, B * J, 1.0 / (3.0 * (double)N), mean, s));
  k_zero_u32<<<(unsigned)ceil_div((int64_t)B * J * kBins, 256), 256, 0, s>>>(counts, (int64_t)B * J * kBins);
  EX_LAUNCHED("histogram clear");
  const unsigned hb = (unsigned)std::min<int64_t>(256, ceil_div(3 * N, 256));
  k_level_hist<<<dim3(hb, J, B), kBins, 0, s>>>(w, N, nb, J, mean, counts);
  EX_LAUNCHED("histogram");
  k_level_mode<<<B * J, 64, 0, s>>>(counts, mean, J, nb, scale, lam);
  EX_LAUNCHED("histogram mode");
  return EXPENC_OK;
}

namespace {

struct BalLayout {
  EncPlan p, pf, p1;
  EncBuffers eb;
  int J = 1, nb = 4, B = 1;
  int64_t N = 0;
  float2 *a0 = nullptr, *a1 = nullptr, *beta = nullptr, *gw = nullptr;  // [B][nb][N]
  float2 *xb = nullptr, *r = nullptr, *c = nullptr, *xref = nullptr, *rref = nullptr, *tmp = nullptr;
  float2 *pvec = nullptr, *ptmp = nullptr;
  double *dpart = nullptr, *sc = nullptr;  // sc: L_A, kappa, L, pad, lam[B nb], tau[B nb], mean[B J], 3 scratch
  unsigned *counts = nullptr;
  unsigned *status = nullptr;  // the call's status word (start of the workspace)
  double *lam() const { return sc + 4; }
  double *tau() const { return sc + 4 + B * nb; }
  double *mean() const { return sc + 4 + 2 * B * nb; }
  double *scratch() const { return sc + 4 + 2 * B * nb + B * J; }
};

int layout_bal(const expenc_op *op, int32_t batch, const expenc_balanced_opts *o, Arena &a, BalLayout *L) {
  if (!o) return fail(EXPENC_EINVAL, "options are NULL");
  if (o->levels < 1 || o->levels > 8) return fail(EXPENC_EINVAL, "levels must be in [1, 8]");
  L->status = take_status(a);
  EX_TRY(make_plan(op, batch, o->precision, &L->p));
  EX_TRY(make_plan(op, batch, EXPENC_FP32, &L->pf));
  // power iteration in the solve's precision when there is one image (p1 and
  // p then share geometry and tables)
  EX_TRY(make_plan(op, 1, batch == 1 ? o->precision : EXPENC_FP32, &L->p1));
  L->J = o->levels;
  L->nb = 3 * o->levels + 1;
  L->B = batch;
  L->N = (int64_t)op->nx * op->ny;
  carve_enc(L->p, a, &L->eb, std::max(enc_part_elems(L->p1), enc_part_elems(L->pf)));
  const size_t coef = (size_t)batch * L->nb * L->N, img = (size_t)batch * L->N;
  L->a0 = a.take<float2>(coef);
  L->a1 = a.take<float2>(coef);
  L->beta = a.take<float2>(coef);
  L->gw = a.take<float2>(coef);
  L->xb = a.take<float2>(img);
  L->r = a.take<float2>(img);
  L->c = a.take<float2>(img);
  L->tmp = a.take<float2>(2 * img);
  if (o->precision != EXPENC_FP32) {
    L->xref = a.take<float2>(img);
    L->rref = a.take<float2>(img);
  }
  L->pvec = a.take<float2>((size_t)L->p.R);
  L->ptmp = a.take<float2>((size_t)L->p.R);
  L->dpart = a.take<double>((size_t)std::max(batch * L->J, batch) * kRedBlocks);
  L->sc = a.take<double>((size_t)4 + 2 * batch * L->nb + batch * L->J + 3);
  L->counts = a.take<unsigned>((size_t)batch * L->J * kBins);
  return a.ok() ? EXPENC_OK : EXPENC_EWORKSPACE;
}

int check_bal(const expenc_balanced_opts *o, int *refine) {
  if (!o) return fail(EXPENC_EINVAL, "options are NULL");
  if (o->n_iter < 0) return fail(EXPENC_EINVAL, "n_iter must be >= 0");
  if (o->wavelet != EXPENC_HAAR && o->wavelet != EXPENC_DB4) return fail(EXPENC_EINVAL, "unknown wavelet");
  if (o->lipschitz <= 0 && (!o->power_v0 || o->n_power < 1))
    return fail(EXPENC_EINVAL, "lipschitz <= 0 requires power_v0 and n_power >= 1");
  if (!o->lambda && !(o->lambda_scale > 0)) return fail(EXPENC_EINVAL, "lambda_scale must be > 0");
  if (o->anchor != EXPENC_ANCHOR_ENDS && o->anchor != EXPENC_ANCHOR_FP32 && o->anchor != EXPENC_ANCHOR_SPLIT)
    return fail(EXPENC_EINVAL, "unknown anchor mode %d", o->anchor);
  *refine = o->refine_every > 0 ? o->refine_every : default_refine(o->precision, o->anchor);
  return EXPENC_OK;
}

}  // namespace
}  // namespace expenc

using namespace expenc;

extern "C" size_t expenc_swt_workspace_size(int32_t nx, int32_t ny, int32_t levels, int32_t batch) {
  if (check_swt(nx, ny, levels, batch) != EXPENC_OK) return 0;
  return (size_t)2 * batch * nx * ny * sizeof(float2) + 256;
}

extern "C" int swt_fwd(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch, const float *x,
                       float *w, void *ws, size_t ws_bytes, void *stream) {
  EX_TRY(check_swt(nx, ny, levels, batch));
  if (!x || !w) return fail(EXPENC_EINVAL, "NULL array");
  if ((levels > 1) && (!ws || ws_bytes < expenc_swt_workspace_size(nx, ny, levels, batch)))
    return fail(EXPENC_EWORKSPACE, "workspace too small");
  FilterSet f;
  EX_TRY(make_filter_set(wavelet, &f));
  return swt_forward(f, nx, ny, levels, batch, reinterpret_cast<const float2 *>(x), reinterpret_cast<float2 *>(w),
                     static_cast<float2 *>(ws), (hipStream_t)stream);
}

extern "C" int swt_inv(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch, const float *w,
                       float *x, void *ws, size_t ws_bytes, void *stream) {
  EX_TRY(check_swt(nx, ny, levels, batch));
  if (!x || !w) return fail(EXPENC_EINVAL, "NULL array");
  if ((levels > 1) && (!ws || ws_bytes < expenc_swt_workspace_size(nx, ny, levels, batch)))
    return fail(EXPENC_EWORKSPACE, "workspace too small");
  FilterSet f;
  EX_TRY(make_filter_set(wavelet, &f));
  return swt_adjoint(f, nx, ny, levels, batch, reinterpret_cast<const float2 *>(w), reinterpret_cast<float2 *>(x),
                     static_cast<float2 *>(ws), (hipStream_t)stream);
}

extern "C" size_t expenc_sigma_workspace_size(int32_t nx, int32_t ny, int32_t levels, int32_t batch) {
  if (check_swt(nx, ny, levels, batch) != EXPENC_OK) return 0;
  Arena a;
  a.take<double>((size_t)batch * levels * kRedBlocks);
  a.take<double>((size_t)batch * levels);
  a.take<unsigned>((size_t)batch * levels * kBins);
  return a.used + 256;
}

extern "C" int expenc_sigma_weights(int32_t nx, int32_t ny, int32_t levels, int32_t batch, const float *w,
                                    double scale, double *lam, unsigned *counts, void *ws, size_t ws_bytes,
                                    void *stream) {
  EX_TRY(check_swt(nx, ny, levels, batch));
  if (!w || !lam) return fail(EXPENC_EINVAL, "NULL array");
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  double *part = a.take<double>((size_t)batch * levels * kRedBlocks);
  double *mean = a.take<double>((size_t)batch * levels);
  unsigned *cnt = a.take<unsigned>((size_t)batch * levels * kBins);
  if (!ws || !a.ok()) return fail(EXPENC_EWORKSPACE, "workspace too small");
  return sigma_weights(reinterpret_cast<const float2 *>(w), nx, ny, levels, batch, scale, part, mean,
                       counts ? counts : cnt, lam, (hipStream_t)stream);
}

extern "C" size_t fista_balanced_workspace_size(const expenc_op *op, int32_t batch, const expenc_balanced_opts *opts) {
  Arena a;
  BalLayout L;
  const int st = layout_bal(op, batch, opts, a, &L);
  if (st != EXPENC_OK && st != EXPENC_EWORKSPACE) return 0;
  return a.used + 256;
}

extern "C" int fista_balanced_solve(const expenc_op *op, int32_t batch, const float *y, float *x,
                                    const expenc_balanced_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  int refine = 0;
  EX_TRY(check_bal(opts, &refine));
  if (!y || !x) return fail(EXPENC_EINVAL, "y or x is NULL");
  BalLayout L;
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  const int st = layout_bal(op, batch, opts, a, &L);
  if (st == EXPENC_EWORKSPACE || !ws)
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                fista_balanced_workspace_size(op, batch, opts));
  EX_TRY(st);
  FilterSet f;
  EX_TRY(make_filter_set(opts->wavelet, &f));
  hipStream_t s = (hipStream_t)stream;
  const EncPlan &p = L.p, &pf = L.pf;
  const int B = batch, J = L.J, nb = L.nb;
  const int64_t N = L.N, img = (int64_t)B * N, coef = img * nb;
  const float2 *y2 = reinterpret_cast<const float2 *>(y);
  const bool split = opts->precision != EXPENC_FP32;
  // prologue: tables, L_A, kappa, L, weights, thresholds, zero state
  EX_TRY(clear_status(L.status, s));
  EX_TRY(enc_prepare(pf, op, L.eb, s));
  if (split) EX_TRY(enc_prepare(p, op, L.eb, s));
  if (opts->lipschitz > 0) {
    k_set_scalar<<<1, 64, 0, s>>>(L.sc, opts->lipschitz);
    EX_LAUNCHED("lipschitz");
  } else {
    EX_TRY(lipschitz_run(L.p1, op, L.eb, opts->n_power, opts->power_v0, L.pvec, L.ptmp, L.dpart, L.scratch(), L.sc,
                         s));
  }
  k_bal_scalars<<<1, 64, 0, s>>>(L.sc, opts->kappa);
  EX_LAUNCHED("balanced scalars");
  if (opts->lambda) {
    k_copy_lam<<<(unsigned)ceil_div(B * nb, 256), 256, 0, s>>>(opts->lambda, L.lam(), B * nb);
    EX_LAUNCHED("weights");
  } else {
    // sigma/2 weights from W A^H y (FP32 operators)
    EX_TRY(enc_pack_y(pf, y2, L.eb, s));
    EX_TRY(enc_adjoint_partials(pf, L.eb, s));
    EX_TRY(enc_adjoint_reduce_out(pf, L.eb, op->smaps, L.xb, N, op->nx, nullptr, nullptr, s));
    EX_TRY(swt_forward(f, op->nx, op->ny, J, B, L.xb, L.gw, L.tmp, s));
    EX_TRY(sigma_weights(L.gw, op->nx, op->ny, J, B, opts->lambda_scale, L.dpart, L.mean(), L.counts, L.lam(), s));
  }
  k_bal_tau<<<(unsigned)ceil_div(B * nb, 256), 256, 0, s>>>(L.sc, L.lam(), L.tau(), B * nb);
  EX_LAUNCHED("thresholds");
  k_zero_c<<<(unsigned)ceil_div(coef, 256), 256, 0, s>>>(L.a0, coef);
  k_zero_c<<<(unsigned)ceil_div(coef, 256), 256, 0, s>>>(L.beta, coef);
  EX_LAUNCHED("zero state");
  const int K = opts->n_iter;
  std::vector<double> mom(K, 0.0);
  {
    double t = 1.0;
    for (int k = 0; k < K; ++k) {
      const double tn = opts->ista ? 1.0 : (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      mom[k] = (t - 1.0) / tn;
      t = tn;
    }
  }
  auto body = [&](hipStream_t cs) -> int {
    for (int k = 0; k < K; ++k) {
      float2 *aprev = (k % 2 == 0) ? L.a0 : L.a1;
      float2 *anew = (k % 2 == 0) ? L.a1 : L.a0;
      EX_TRY(swt_adjoint(f, op->nx, op->ny, J, B, L.beta, L.xb, L.tmp, cs));
      // beta_0 = 0, so the first residual A W^H beta - y is -y without a
      // forward product
      auto residual_fp32 = [&](const EncPlan &q) -> int {
        if (k == 0) return enc_pack_y(q, y2, L.eb, cs, -1.f);
        EX_TRY(enc_build_z(q, op->smaps, L.xb, N, op->nx, L.eb, cs));
        EX_TRY(enc_forward_partials(q, L.eb, cs));
        return enc_forward_residual(q, L.eb, y2, cs);
      };
      if (!split) {
        EX_TRY(residual_fp32(p));
        EX_TRY(enc_adjoint_partials(p, L.eb, cs));
        EX_TRY(enc_adjoint_reduce_out(p, L.eb, op->smaps, L.r, N, op->nx, nullptr, nullptr, cs));
      } else if (k % refine == 0 || k == K - 1) {
        const EncPlan &pa = anchor_in_fp32(opts->anchor, k, K) ? pf : p;
        EX_TRY(residual_fp32(pa));
        EX_TRY(enc_adjoint_partials(pa, L.eb, cs));
        EX_TRY(enc_adjoint_reduce_out(pa, L.eb, op->smaps, L.rref, N, op->nx, nullptr, nullptr, cs));
        EX_TRY(copy_f2(L.rref, L.r, img, cs));
        EX_TRY(copy_f2(L.xb, L.xref, img, cs));
      } else {
        EX_TRY(enc_build_z(p, op->smaps, L.xb, N, op->nx, L.eb, cs, L.xref));
        EX_TRY(enc_forward_partials(p, L.eb, cs));
        EX_TRY(enc_forward_residual(p, L.eb, nullptr, cs));
        EX_TRY(enc_adjoint_partials(p, L.eb, cs));
        EX_TRY(enc_adjoint_reduce_out(p, L.eb, op->smaps, L.r, N, op->nx, nullptr, nullptr, cs, L.rref));
      }
      k_bal_combine<<<(unsigned)ceil_div(img, 256), 256, 0, cs>>>(L.r, L.xb, L.sc, L.c, img);
      EX_LAUNCHED("combine");
      EX_TRY(swt_forward(f, op->nx, op->ny, J, B, L.c, L.gw, L.tmp, cs));
      k_bal_update<<<(unsigned)ceil_div(coef, 256), 256, 0, cs>>>(L.beta, L.gw, aprev, anew, L.sc, L.tau(), nb, N,
                                                                   coef, mom[k], L.status);
      EX_LAUNCHED("balanced update");
    }
    return EXPENC_OK;
  };
  uint64_t key = 0x5bd1e9955bd1e995ull;
  key = hash_bytes(key, op, sizeof(*op));
  key = hash_bytes(key, &batch, sizeof(batch));
  key = hash_bytes(key, &y, sizeof(y));
  key = hash_bytes(key, &ws, sizeof(ws));
  key = hash_bytes(key, &ws_bytes, sizeof(ws_bytes));
  key = hash_bytes(key, opts, sizeof(*opts));
  const uint64_t gen = tuning_generation();
  key = hash_bytes(key, &gen, sizeof(gen));
  if (K > 0) EX_TRY(run_captured(key, s, body));
  const float2 *aK = (K == 0) ? L.a0 : ((K - 1) % 2 == 0 ? L.a1 : L.a0);
  EX_TRY(swt_adjoint(f, op->nx, op->ny, J, B, aK, reinterpret_cast<float2 *>(x), L.tmp, s));
  if (opts->scalars) {
    k_copy_lam<<<(unsigned)ceil_div(3 + 2 * B * nb, 256), 256, 0, s>>>(L.sc, opts->scalars, 3);
    k_copy_lam<<<(unsigned)ceil_div(2 * B * nb, 256), 256, 0, s>>>(L.lam(), opts->scalars + 3, 2 * B * nb);
    EX_LAUNCHED("scalars out");
  }
  return EXPENC_OK;
}
