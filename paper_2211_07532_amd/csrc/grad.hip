// Gradients of the encoding operators with respect to the field parameters
// k_l(t) and dw0(r) (the differentiable form of eq. 1's operator).
//
// With E(t,r) = exp(i phi), phi = sum_l k_l(t) b_l(r) + dw0(r) t, one has
// dA/dk_l(t) = i b_l(r) A and dA/d dw0(r) = i t A.  For a real loss with
// upstream gradients in the convention grad = dL/dRe + i dL/dIm:
//   y = A x,    upstream g:   grad_k[t,l]  = -Im sum_c conj(g[t,c]) [A(b_l x)](t,c)
//                             grad_dw[r]   = -Im( x(r) conj([A^H (t g)](r)) )
//   x = A^H y,  upstream gx:  grad_k[t,l]  = -Im sum_c conj(y[t,c]) [A(b_l gx)](t,c)
//                             grad_dw[r]   = -Im( gx(r) conj([A^H (t y)](r)) )
// i.e. one form with (w, kk) = (x, g) or (gx, y).  The L products A(b_l w)
// run as ONE batched forward contraction with L*C columns, so every phase
// tile is generated once and shared by all basis terms; grad_dw needs one
// adjoint.  Sums over coils are accumulated in FP64.
#include "internal.h"
#include "reduce.h"

namespace expenc {

// xb[l][r] = b_l(r) * w(r): b_l from the FP64 phase table bet[r][l] (basis
// given as maps), or, with bet NULL, the solid harmonics at the pixel centre
// ((x - nx/2) dx, (y - ny/2) dy, z0)
__global__ void k_basis_weight(const double *__restrict__ bet, int NT, int L, const float2 *__restrict__ w, int R,
                               float2 *__restrict__ xb, int nx, int ny, double dx, double dy, double z0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)L * R) return;
  const int l = (int)(i / R), r = (int)(i % R);
  float b;
  if (bet) {
    b = (float)bet[(int64_t)r * NT + l];
  } else {
    double v[16];
    sh_eval((r % nx - 0.5 * nx) * dx, (r / nx - 0.5 * ny) * dy, z0, v);
    b = (float)v[l];
  }
  const float2 v = w[r];
  xb[i] = make_float2(b * v.x, b * v.y);
}

// tk[t][c] = time[t] * kk[t][c]
__global__ void k_time_weight(const double *__restrict__ time, const float2 *__restrict__ kk, int64_t T, int C,
                              float2 *__restrict__ tk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T * C) return;
  const float t = (float)time[i / C];
  const float2 v = kk[i];
  tk[i] = make_float2(t * v.x, t * v.y);
}

// grad_k[t][l] = -Im sum_c conj(kk[t][c]) yb[l][t][c]   (FP64)
__global__ void k_grad_coef(const float2 *__restrict__ yb, const float2 *__restrict__ kk, int64_t T, int C, int L,
                            double *__restrict__ grad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T * L) return;
  const int64_t t = i / L;
  const int l = (int)(i % L);
  double s = 0.0;
  for (int c = 0; c < C; ++c) {
    const float2 a = kk[t * C + c];
    const float2 b = yb[((int64_t)l * T + t) * C + c];
    s += (double)a.x * b.y - (double)a.y * b.x;  // Im(conj(a) b)
  }
  grad[i] = -s;
}

// grad_dw[r] = -Im( w(r) conj(a(r)) )
__global__ void k_grad_dw(const float2 *__restrict__ w, const float2 *__restrict__ a, int R,
                          double *__restrict__ grad) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const float2 u = w[r], v = a[r];
  grad[r] = -((double)u.y * v.x - (double)u.x * v.y);
}

struct GradLayout {
  EncPlan pL;   // batch L (the basis-weighted forward products)
  EncPlan p1;   // batch 1 (the time-weighted adjoint)
  EncBuffers eb;
  float2 *xb = nullptr, *yb = nullptr, *tk = nullptr, *ax = nullptr;
};

static int layout_grad(const expenc_op *op, int32_t precision, Arena &a, GradLayout *G) {
  const int L = op ? op->nbasis : 0;
  EX_TRY(make_plan(op, L > 0 ? L : 1, precision, &G->pL));
  EX_TRY(make_plan(op, 1, precision, &G->p1));
  carve_enc(G->pL, a, &G->eb, enc_part_elems(G->p1));
  const size_t R = (size_t)op->nx * op->ny;
  G->xb = a.take<float2>((size_t)(L > 0 ? L : 1) * R);
  G->yb = a.take<float2>((size_t)(L > 0 ? L : 1) * op->nsamples * op->ncoils);
  G->tk = a.take<float2>((size_t)op->nsamples * op->ncoils);
  G->ax = a.take<float2>(R);
  return a.ok() ? EXPENC_OK : EXPENC_EWORKSPACE;
}

size_t grad_bytes(const expenc_op *op, int32_t precision) {
  Arena a;
  GradLayout G;
  if (layout_grad(op, precision, a, &G) != EXPENC_OK && !G.pL.R) return 0;
  return a.used + 256;
}

}  // namespace expenc

using namespace expenc;

extern "C" int expenc_field_grad(const expenc_op *op, int32_t precision, const float *w, const float *kk,
                                 double *grad_coef, double *grad_dw0, void *ws, size_t ws_bytes, void *stream) {
  if (!w || !kk) return fail(EXPENC_EINVAL, "w or kk is NULL");
  if (precision != EXPENC_FP32) return fail(EXPENC_EUNSUPPORTED, "field gradients are computed in the FP32 form");
  GradLayout G;
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  const int st = layout_grad(op, precision, a, &G);
  if (st == EXPENC_EWORKSPACE || !ws)
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                grad_bytes(op, precision));
  EX_TRY(st);
  hipStream_t s = (hipStream_t)stream;
  const float2 *w2 = reinterpret_cast<const float2 *>(w);
  const float2 *k2 = reinterpret_cast<const float2 *>(kk);
  const EncPlan &pL = G.pL, &p1 = G.p1;
  const int L = op->nbasis;
  const int R = p1.R;
  const int64_t T = p1.T;
  const int C = p1.C;
  EX_TRY(enc_prepare(pL, op, G.eb, s));
  if (grad_coef && L > 0) {
    k_basis_weight<<<(unsigned)ceil_div((int64_t)L * R, 256), 256, 0, s>>>(pL.sh ? nullptr : G.eb.bet, pL.NT, L, w2,
                                                                          R, G.xb, p1.nx, p1.ny, pL.dx, pL.dy, pL.z0);
    EX_LAUNCHED("basis weighting");
    EX_TRY(enc_build_z(pL, op->smaps, G.xb, R, p1.nx, G.eb, s));
    EX_TRY(enc_forward_partials(pL, G.eb, s));
    EX_TRY(enc_forward_reduce_out(pL, G.eb, G.yb, s));
    k_grad_coef<<<(unsigned)ceil_div(T * L, 256), 256, 0, s>>>(G.yb, k2, T, C, L, grad_coef);
    EX_LAUNCHED("coefficient gradient");
  }
  if (grad_dw0) {
    k_time_weight<<<(unsigned)ceil_div(T * C, 256), 256, 0, s>>>(op->time, k2, T, C, G.tk);
    EX_LAUNCHED("time weighting");
    EX_TRY(enc_pack_y(p1, G.tk, G.eb, s));
    EX_TRY(enc_adjoint_partials(p1, G.eb, s));
    EX_TRY(enc_adjoint_reduce_out(p1, G.eb, op->smaps, G.ax, R, p1.nx, nullptr, nullptr, s));
    k_grad_dw<<<(unsigned)ceil_div(R, 256), 256, 0, s>>>(w2, G.ax, R, grad_dw0);
    EX_LAUNCHED("off-resonance gradient");
  }
  return EXPENC_OK;
}
