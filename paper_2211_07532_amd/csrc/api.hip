// C-ABI entry points for the encoding operators, the field basis and the
// Lipschitz estimate, plus the FP64 reduction kernels the solvers share.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.h"
#include "reduce.h"

namespace expenc {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

int fail(int status, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

// ---------------------------------------------------------------------------
// Field basis: real solid harmonics up to 3rd order on the pixel grid.
// ---------------------------------------------------------------------------

__global__ void k_sh_basis(int nx, int ny, double dx, double dy, double z, int L, double *__restrict__ out) {
  const int64_t R = (int64_t)nx * ny;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int i = (int)(r % nx), j = (int)(r / nx);
  const double x = (i - 0.5 * nx) * dx;
  const double y = (j - 0.5 * ny) * dy;
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  double v[16];
  v[0] = 1.0;
  v[1] = x;
  v[2] = y;
  v[3] = z;
  v[4] = x * y;
  v[5] = y * z;
  v[6] = 2.0 * z2 - x2 - y2;
  v[7] = x * z;
  v[8] = x2 - y2;
  v[9] = y * (3.0 * x2 - y2);
  v[10] = x * y * z;
  v[11] = y * (4.0 * z2 - x2 - y2);
  v[12] = z * (2.0 * z2 - 3.0 * x2 - 3.0 * y2);
  v[13] = x * (4.0 * z2 - x2 - y2);
  v[14] = z * (x2 - y2);
  v[15] = x * (x2 - 3.0 * y2);
  for (int l = 0; l < L; ++l) out[l * R + r] = v[l];
}

// ---------------------------------------------------------------------------
// FP64 reductions with a fixed summation order (bitwise reproducible).
// part[b * nblk + blk] holds block sums; k_finish_* adds them in order.
// ---------------------------------------------------------------------------

__device__ inline double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  return red[0];
}

__device__ inline double block_max(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  return red[0];
}

// Re sum conj(a) b over problem slice b (n elements each, stride `stride`).
__global__ __launch_bounds__(256) void k_dot_part(const float2 *__restrict__ a, const float2 *__restrict__ b,
                                                  int64_t n, int64_t stride, double *__restrict__ part) {
  __shared__ double red[256];
  const int prob = blockIdx.y;
  const float2 *pa = a + prob * stride;
  const float2 *pb = b + prob * stride;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float2 u = pa[i], v = pb[i];
    s += (double)u.x * v.x + (double)u.y * v.y;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[prob * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_maxabs_part(const float2 *__restrict__ a, int64_t n, int64_t stride,
                                                     double *__restrict__ part) {
  __shared__ double red[256];
  const int prob = blockIdx.y;
  const float2 *pa = a + prob * stride;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float2 u = pa[i];
    s = fmax(s, sqrt((double)u.x * u.x + (double)u.y * u.y));
  }
  s = block_max(s, red);
  if (threadIdx.x == 0) part[prob * gridDim.x + blockIdx.x] = s;
}

// out[b] = scale * sum_k part[b*nblk + k]  (mode 0)  or max (mode 1)
__global__ __launch_bounds__(256) void k_finish(const double *__restrict__ part, int nblk, double scale, int mode,
                                                double *__restrict__ out) {
  __shared__ double red[256];
  const int prob = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    const double v = part[prob * nblk + k];
    s = mode ? fmax(s, v) : s + v;
  }
  s = mode ? block_max(s, red) : block_sum(s, red);
  if (threadIdx.x == 0) out[prob] = scale * s;
}

int reduce_dot(const float2 *a, const float2 *b, int64_t n, int64_t stride, int B, double scale, double *part,
               double *out, hipStream_t s) {
  k_dot_part<<<dim3(kRedBlocks, B), 256, 0, s>>>(a, b, n, stride, part);
  EX_LAUNCHED("dot");
  k_finish<<<B, 256, 0, s>>>(part, kRedBlocks, scale, 0, out);
  EX_LAUNCHED("dot finish");
  return EXPENC_OK;
}

int reduce_maxabs(const float2 *a, int64_t n, int64_t stride, int B, double scale, double *part, double *out,
                  hipStream_t s) {
  k_maxabs_part<<<dim3(kRedBlocks, B), 256, 0, s>>>(a, n, stride, part);
  EX_LAUNCHED("maxabs");
  k_finish<<<B, 256, 0, s>>>(part, kRedBlocks, scale, 1, out);
  EX_LAUNCHED("maxabs finish");
  return EXPENC_OK;
}

int reduce_sum_parts(const double *part, int nblk, int B, double scale, double *out, hipStream_t s) {
  k_finish<<<B, 256, 0, s>>>(part, nblk, scale, 0, out);
  EX_LAUNCHED("sum finish");
  return EXPENC_OK;
}

// v[b][i] *= 1/sqrt(nrm2[b])   (power-iteration normalisation)
__global__ void k_scale_rsqrt(float2 *__restrict__ v, int64_t n, int64_t stride, const double *__restrict__ nrm2) {
  const int prob = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double nv = nrm2[prob];
  const float sc = nv > 0.0 ? (float)(1.0 / sqrt(nv)) : 0.f;
  float2 u = v[prob * stride + i];
  v[prob * stride + i] = make_float2(u.x * sc, u.y * sc);
}

__global__ void k_copy_f2(const float2 *__restrict__ in, float2 *__restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

// out = a x + b y over n complex values (real a, b)
__global__ void k_axpby(int64_t n, float a, const float2 *__restrict__ x, float b, const float2 *__restrict__ y,
                        float2 *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 u = x[i], v = y[i];
  out[i] = make_float2(fmaf(a, u.x, b * v.x), fmaf(a, u.y, b * v.y));
}

// L[p] = 2 * num[p]/den[p] for each problem
__global__ void k_lipschitz_final(const double *__restrict__ num, const double *__restrict__ den, double *out, int P) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) out[p] = den[p] > 0.0 ? 2.0 * num[p] / den[p] : 0.0;
}

int scale_rsqrt(float2 *v, int64_t n, int64_t stride, int B, const double *nrm2, hipStream_t s) {
  k_scale_rsqrt<<<dim3((unsigned)ceil_div(n, 256), B), 256, 0, s>>>(v, n, stride, nrm2);
  EX_LAUNCHED("scale");
  return EXPENC_OK;
}

int copy_f2(const float2 *in, float2 *out, int64_t n, hipStream_t s) {
  k_copy_f2<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(in, out, n);
  EX_LAUNCHED("copy");
  return EXPENC_OK;
}

// u = A^H A v for the batch-1 plan of each of p.P problems: v, u [P][R] (row stride nx).
int normal_apply(const EncPlan &p, const expenc_op *op, const EncBuffers &eb, const float2 *v, float2 *u,
                 hipStream_t s) {
  EX_TRY(enc_build_z(p, op->smaps, v, p.R, p.nx, eb, s, nullptr, p.R));
  EX_TRY(enc_forward_partials(p, eb, s));
  EX_TRY(enc_forward_residual(p, eb, nullptr, s));
  EX_TRY(enc_adjoint_partials(p, eb, s));
  return enc_adjoint_reduce_out(p, eb, op->smaps, u, p.R, p.nx, nullptr, nullptr, s, nullptr, p.R);
}

size_t lipschitz_bytes(const EncPlan &p1) {
  Arena a;
  EncBuffers eb;
  carve_enc(p1, a, &eb);
  a.take<float2>((size_t)p1.R * p1.P);
  a.take<float2>((size_t)p1.R * p1.P);
  a.take<double>((size_t)kRedBlocks * p1.P + 8 * p1.P);
  return a.used + 256;
}

// Power iteration for each of p1.P problems (batch-1 plan, kap/bet prepared
// in eb), all from the same start vector v0 [R].  Scratch: vec, tmp [P][R],
// dpart [P * kRedBlocks], dsc [3P].  Writes L[p] to L_out[p].
int lipschitz_run(const EncPlan &p1, const expenc_op *op, const EncBuffers &eb, int n_iter, const float *v0,
                  float2 *vec, float2 *tmp, double *dpart, double *dsc, double *L_out, hipStream_t s) {
  const int64_t R = p1.R;
  const int P = p1.P;
  for (int q = 0; q < P; ++q) EX_TRY(copy_f2(reinterpret_cast<const float2 *>(v0), vec + q * R, R, s));
  EX_TRY(reduce_dot(vec, vec, R, R, P, 1.0, dpart, dsc, s));
  EX_TRY(scale_rsqrt(vec, R, R, P, dsc, s));
  for (int it = 0; it < n_iter; ++it) {
    EX_TRY(normal_apply(p1, op, eb, vec, tmp, s));
    EX_TRY(reduce_dot(tmp, tmp, R, R, P, 1.0, dpart, dsc, s));
    EX_TRY(scale_rsqrt(tmp, R, R, P, dsc, s));
    std::swap(vec, tmp);
  }
  // Rayleigh quotient <v, A^H A v>/<v, v>: the FP32 form takes ||A v||^2 from
  // its residual operand; the split forms pack their residual into MFMA
  // records, so they apply A^H A once more
  if (p1.prec == EXPENC_FP32) {
    EX_TRY(enc_build_z(p1, op->smaps, vec, R, p1.nx, eb, s, nullptr, R));
    EX_TRY(enc_forward_partials(p1, eb, s));
    EX_TRY(enc_forward_residual(p1, eb, nullptr, s));
    EX_TRY(reduce_dot(eb.yop, eb.yop, p1.Tp * p1.NCP, p1.Tp * p1.NCP, P, 1.0, dpart, dsc + P, s));
  } else {
    EX_TRY(normal_apply(p1, op, eb, vec, tmp, s));
    EX_TRY(reduce_dot(vec, tmp, R, R, P, 1.0, dpart, dsc + P, s));
  }
  EX_TRY(reduce_dot(vec, vec, R, R, P, 1.0, dpart, dsc + 2 * P, s));
  k_lipschitz_final<<<(unsigned)ceil_div(P, 256), 256, 0, s>>>(dsc + P, dsc + 2 * P, L_out, P);
  EX_LAUNCHED("lipschitz final");
  return EXPENC_OK;
}

}  // namespace expenc

using namespace expenc;

extern "C" const char *expenc_last_error(void) { return g_last_error.c_str(); }

extern "C" int expenc_sh_basis(int32_t nx, int32_t ny, double fov_x, double fov_y, double z0, int32_t nbasis,
                               double *basis, void *stream) {
  if (nx < 1 || ny < 1 || nbasis < 0 || nbasis > 16 || !(fov_x > 0) || !(fov_y > 0))
    return fail(EXPENC_EINVAL, "bad sh_basis arguments (nx=%d ny=%d nbasis=%d)", nx, ny, nbasis);
  if (nbasis == 0) return EXPENC_OK;
  if (!basis) return fail(EXPENC_EINVAL, "basis output is NULL");
  const int64_t R = (int64_t)nx * ny;
  k_sh_basis<<<(unsigned)ceil_div(R, 256), 256, 0, (hipStream_t)stream>>>(nx, ny, fov_x / nx, fov_y / ny, z0,
                                                                          nbasis, basis);
  EX_LAUNCHED("sh_basis");
  return EXPENC_OK;
}

extern "C" size_t expenc_workspace_size(const expenc_op *op, int32_t batch, int32_t precision, int32_t what,
                                        int32_t nx_pad, int32_t ny_pad) {
  EncPlan p;
  if (make_plan(op, batch, precision, &p) != EXPENC_OK) return 0;
  switch (what) {
    case EXPENC_WS_FORWARD:
    case EXPENC_WS_ADJOINT:
      return enc_operand_bytes(p);
    case EXPENC_WS_LIPSCHITZ: {
      EncPlan p1;
      if (make_plan(op, 1, precision, &p1) != EXPENC_OK) return 0;
      return lipschitz_bytes(p1);
    }
    case EXPENC_WS_FISTA:
      return fista_bytes(op, batch, precision, nx_pad, ny_pad);
    case EXPENC_WS_CG:
      return cg_bytes(op, batch, precision);
    case EXPENC_WS_FIELD_GRAD:
      return grad_bytes(op, precision);
    default:
      return 0;
  }
}

extern "C" int expenc_forward(const expenc_op *op, int32_t batch, int32_t precision, const float *x, float *y,
                              void *ws, size_t ws_bytes, void *stream) {
  EncPlan p;
  EX_TRY(make_plan(op, batch, precision, &p));
  if (!x || !y) return fail(EXPENC_EINVAL, "x or y is NULL");
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  EncBuffers eb;
  if (carve_enc(p, a, &eb) != EXPENC_OK || !ws)
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                enc_operand_bytes(p));
  hipStream_t s = (hipStream_t)stream;
  EX_TRY(enc_prepare(p, op, eb, s));
  EX_TRY(enc_build_z(p, op->smaps, reinterpret_cast<const float2 *>(x), p.R, p.nx, eb, s));
  EX_TRY(enc_forward_partials(p, eb, s));
  return enc_forward_reduce_out(p, eb, reinterpret_cast<float2 *>(y), s);
}

extern "C" int expenc_adjoint(const expenc_op *op, int32_t batch, int32_t precision, const float *y, float *x,
                              void *ws, size_t ws_bytes, void *stream) {
  EncPlan p;
  EX_TRY(make_plan(op, batch, precision, &p));
  if (!x || !y) return fail(EXPENC_EINVAL, "x or y is NULL");
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  EncBuffers eb;
  if (carve_enc(p, a, &eb) != EXPENC_OK || !ws)
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                enc_operand_bytes(p));
  hipStream_t s = (hipStream_t)stream;
  EX_TRY(enc_prepare(p, op, eb, s));
  EX_TRY(enc_pack_y(p, reinterpret_cast<const float2 *>(y), eb, s));
  EX_TRY(enc_adjoint_partials(p, eb, s));
  return enc_adjoint_reduce_out(p, eb, op->smaps, reinterpret_cast<float2 *>(x), p.R, p.nx, nullptr, nullptr, s);
}

extern "C" int expenc_lipschitz(const expenc_op *op, int32_t precision, int32_t n_iter, const float *v0,
                                double *lipschitz_out, void *ws, size_t ws_bytes, void *stream) {
  EncPlan p1;
  EX_TRY(make_plan(op, 1, precision, &p1));
  if (n_iter < 0 || !v0 || !lipschitz_out) return fail(EXPENC_EINVAL, "bad lipschitz arguments");
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  EncBuffers eb;
  carve_enc(p1, a, &eb);
  float2 *vec = a.take<float2>((size_t)p1.R);
  float2 *tmp = a.take<float2>((size_t)p1.R);
  double *dpart = a.take<double>(kRedBlocks + 8);
  if (!a.ok() || !ws)
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                lipschitz_bytes(p1));
  hipStream_t s = (hipStream_t)stream;
  EX_TRY(enc_prepare(p1, op, eb, s));
  return lipschitz_run(p1, op, eb, n_iter, v0, vec, tmp, dpart, dpart + kRedBlocks, lipschitz_out, s);
}

extern "C" int expenc_axpby(int64_t n, double a, const float *x, double b, const float *y, float *out,
                            void *stream) {
  if (n < 0) return fail(EXPENC_EINVAL, "n must be >= 0");
  if (n == 0) return EXPENC_OK;
  if (!x || !y || !out) return fail(EXPENC_EINVAL, "NULL array");
  k_axpby<<<(unsigned)ceil_div(n, 256), 256, 0, (hipStream_t)stream>>>(
      n, (float)a, reinterpret_cast<const float2 *>(x), (float)b, reinterpret_cast<const float2 *>(y),
      reinterpret_cast<float2 *>(out));
  EX_LAUNCHED("axpby");
  return EXPENC_OK;
}

extern "C" int expenc_kernel_timing(int32_t mode, double *out) { return kernel_timing(mode, out); }

extern "C" int expenc_solve_status(const void *ws, void *stream) {
  if (!ws) return fail(EXPENC_EINVAL, "workspace is NULL");
  hipStream_t s = (hipStream_t)stream;
  unsigned flags = 0u;
  EX_HIP(hipMemcpyAsync(&flags, ws, sizeof(flags), hipMemcpyDeviceToHost, s));
  EX_HIP(hipStreamSynchronize(s));
  if (flags & kStatusNonFinite) return fail(EXPENC_ENONFINITE, "the call produced NaN or Inf values");
  if (flags & kStatusDiverged)
    return fail(EXPENC_EDIVERGED, "the objective rose above its value at the zero image (step 1/L too large?)");
  return EXPENC_OK;
}

extern "C" int expenc_set_tuning(const expenc_op *op, int32_t batch, int32_t precision, int32_t fwd_target,
                                 int32_t adj_target) {
  EncPlan chk;
  EX_TRY(make_plan(op, batch, precision, &chk));
  return set_tuning(op, batch, precision, fwd_target, adj_target, 0);
}

extern "C" int expenc_set_launch_shape(const expenc_op *op, int32_t batch, int32_t precision, int32_t fwd_target,
                                       int32_t adj_target, int32_t col_groups) {
  return set_tuning(op, batch, precision, fwd_target, adj_target, col_groups);
}

extern "C" int expenc_plan_info_ex(const expenc_op *op, int32_t batch, int32_t precision, int32_t nprob,
                                   int64_t *out, int32_t n_out) {
  if (!out) return fail(EXPENC_EINVAL, "out is NULL");
  if (n_out < 0) return fail(EXPENC_EINVAL, "n_out must be >= 0");
  EncPlan p;
  EX_TRY(make_plan(op, batch, precision, &p, nprob));
  const int64_t v[7] = {p.fwd_split,
                        p.adj_split,
                        (int64_t)p.Tp / 256 * p.fwd_split * p.NGY * p.P,  // forward workgroups per launch
                        (int64_t)p.Rp / 256 * p.adj_split * p.NGY * p.P,  // adjoint workgroups per launch
                        p.Rp / 16,                                        // largest forward split
                        p.Tp / 16,                                        // largest adjoint split
                        p.GW};                                            // 16-column groups per wave
  for (int i = 0; i < n_out && i < 7; ++i) out[i] = v[i];
  return EXPENC_OK;
}

extern "C" int expenc_plan_info(const expenc_op *op, int32_t batch, int32_t precision, int32_t nprob,
                                int64_t *out) {
  return expenc_plan_info_ex(op, batch, precision, nprob, out, 6);
}
