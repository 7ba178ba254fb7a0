// Solvers of eq. 1 on the GPU: FISTA for the l1-wavelet (CS) problem and
// conjugate gradients with early stopping for least squares (Methods 2.1).
//
// FISTA iteration (eq. 1 as written, f(x) = ||A crop(x) - y||^2):
//   r   = A crop(z_k) - y                     (forward contraction + residual)
//   v   = z_k - (2/L) pad(A^H r)              (adjoint contraction + fused step)
//   w   = S_tau(W v)                          (analysis passes, threshold fused)
//   x_k = W^H w,  z_{k+1} = x_k + beta_k (x_k - x_{k-1})   (synthesis, momentum fused)
// with beta_k = (t_k - 1)/t_{k+1}, t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2,
// which do not depend on the data and are baked into the launch arguments.
// L, lambda and tau live in device memory, so the whole prologue (power
// iteration, lambda from A^H y) and the loop run without a host round trip.
// The loop is captured once per argument set into a HIP graph and replayed.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"
#include "reduce.h"
#include "wavelet_dev.h"

namespace expenc {

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------

__global__ void k_fill_d(double *out, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

__global__ void k_zero_f2(float2 *out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2(0.f, 0.f);
}

// sc[0] = L; sc[1] = -2/L; tau[b] = lambda[b]/L
__global__ void k_fista_scalars(double *sc, int B) {
  const int b = threadIdx.x;
  const double L = sc[0];
  if (b == 0) sc[1] = L > 0.0 ? -2.0 / L : 0.0;
  if (b < B) sc[2 + B + b] = L > 0.0 ? sc[2 + b] / L : 0.0;
}

// out[b][y][x] = src[b][y][x] for the nx x ny crop of an nxp x nyp grid
__global__ void k_crop(const float2 *__restrict__ src, int nxp, int nyp, int nx, int ny, int B,
                       float2 *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)nx * ny;
  if (i >= n * B) return;
  const int b = (int)(i / n);
  const int64_t r = i % n;
  const int yy = (int)(r / nx), xx = (int)(r % nx);
  out[i] = src[((int64_t)b * nyp + yy) * nxp + xx];
}

// Per-problem |r|^2 over the adjoint operand's columns b*C .. b*C+C-1.
__global__ __launch_bounds__(256) void k_resid_norm_part(const float2 *__restrict__ yop, int64_t Tp, int NCP,
                                                         int C, double *__restrict__ part) {
  __shared__ double red[256];
  const int b = blockIdx.y;
  const int64_t n = Tp * C;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = i / C;
    const int c = (int)(i % C);
    const float2 v = yop[t * NCP + b * C + c];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[b * gridDim.x + blockIdx.x] = red[0];
}

// objective[b*K + k] = data[b] + lambda[b] * sum_{level, blk} l1[level][b][blk]
// (level j wrote ceil((nxp >> j)/16) block sums out of nblk slots)
__global__ __launch_bounds__(256) void k_objective(const double *__restrict__ data, const double *__restrict__ l1,
                                                   int levels, int B, int nblk, int nxp,
                                                   const double *__restrict__ lam, double *__restrict__ obj, int K,
                                                   int k) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < levels * nblk; i += blockDim.x) {
    const int lev = i / nblk, blk = i % nblk;
    if (blk < (((nxp >> lev) + 15) >> 4)) s += l1[((int64_t)lev * B + b) * nblk + blk];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) obj[(int64_t)b * K + k] = data[b] + lam[b] * red[0];
}

// CG: alpha = rs/pq; x += alpha p; r -= alpha q
__global__ void k_cg_step(float2 *__restrict__ x, float2 *__restrict__ r, const float2 *__restrict__ p,
                          const float2 *__restrict__ q, int64_t n, const double *__restrict__ rs,
                          const double *__restrict__ pq) {
  const int b = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double den = pq[b];
  const float a = den != 0.0 ? (float)(rs[b] / den) : 0.f;
  const int64_t o = (int64_t)b * n + i;
  const float2 pv = p[o], qv = q[o];
  float2 xv = x[o], rv = r[o];
  xv.x += a * pv.x;
  xv.y += a * pv.y;
  rv.x -= a * qv.x;
  rv.y -= a * qv.y;
  x[o] = xv;
  r[o] = rv;
}

// CG: beta = rs_new/rs; p = r + beta p   (rs updated by the caller afterwards)
__global__ void k_cg_dir(float2 *__restrict__ p, const float2 *__restrict__ r, int64_t n,
                         const double *__restrict__ rs, const double *__restrict__ rs_new) {
  const int b = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double den = rs[b];
  const float be = den != 0.0 ? (float)(rs_new[b] / den) : 0.f;
  const int64_t o = (int64_t)b * n + i;
  const float2 rv = r[o];
  float2 pv = p[o];
  p[o] = make_float2(rv.x + be * pv.x, rv.y + be * pv.y);
}

// v = z + alpha * g on the nx x ny crop of each nxp x nyp image, v = z elsewhere
__global__ void k_grad_step(float2 *__restrict__ v, const float2 *__restrict__ z, const float2 *__restrict__ g,
                            const double *__restrict__ alpha_dev, int nxp, int nyp, int nx, int ny, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = i % ((int64_t)nxp * nyp);
  const int yy = (int)(p / nxp), xx = (int)(p % nxp);
  float2 o = z[i];
  if (yy < ny && xx < nx) {
    const float a = (float)*alpha_dev;
    o.x += a * g[i].x;
    o.y += a * g[i].y;
  }
  v[i] = o;
}

__global__ void k_copy_d(const double *in, double *out, int n) {
  const int i = threadIdx.x;
  if (i < n) out[i] = in[i];
}

// ---------------------------------------------------------------------------
// Graph cache: one instantiated graph per distinct argument set.
// ---------------------------------------------------------------------------

struct GraphEntry {
  uint64_t key;
  int device;
  hipGraphExec_t exec;
  hipStream_t last_stream;
};
static std::mutex g_graph_mu;
static std::vector<GraphEntry> g_graphs;
static constexpr size_t kGraphCacheMax = 16;

static uint64_t fnv(uint64_t h, const void *p, size_t n) {
  const unsigned char *c = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

static bool graphs_enabled() {
  static bool on = [] {
    const char *e = getenv("EXPENC_NO_GRAPH");
    return !(e && atoi(e) != 0);
  }();
  return on;
}

static hipStream_t capture_stream(int device) {
  static std::mutex mu;
  static std::vector<hipStream_t> streams;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)streams.size() <= device) streams.resize(device + 1, nullptr);
  if (!streams[device]) hipStreamCreateWithFlags(&streams[device], hipStreamNonBlocking);
  return streams[device];
}

// Runs `body(stream)` either eagerly on s, or captured into a cached graph
// that is then launched on s.
template <class Body>
static int run_graph(uint64_t key, hipStream_t s, Body body) {
  if (!graphs_enabled()) return body(s);
  int dev = 0;
  EX_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto &e : g_graphs)
      if (e.key == key && e.device == dev) {
        e.last_stream = s;
        EX_HIP(hipGraphLaunch(e.exec, s));
        return EXPENC_OK;
      }
  }
  hipStream_t cs = capture_stream(dev);
  if (!cs) return fail(EXPENC_EHIP, "could not create the capture stream");
  EX_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  const int st = body(cs);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &graph);
  if (st != EXPENC_OK) {
    if (graph) hipGraphDestroy(graph);
    return st;
  }
  if (ec != hipSuccess) return fail(EXPENC_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (ei != hipSuccess) return fail(EXPENC_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
  EX_HIP(hipGraphLaunch(exec, s));
  std::lock_guard<std::mutex> lk(g_graph_mu);
  if (g_graphs.size() >= kGraphCacheMax) {
    // the oldest entry may still run on its stream: wait for that stream first
    hipStreamSynchronize(g_graphs.front().last_stream);
    hipGraphExecDestroy(g_graphs.front().exec);
    g_graphs.erase(g_graphs.begin());
  }
  g_graphs.push_back({key, dev, exec, s});
  return EXPENC_OK;
}

// ---------------------------------------------------------------------------
// FISTA
// ---------------------------------------------------------------------------

struct FistaLayout {
  EncPlan p, p1, pf;  // p: iteration precision (batch B); p1: FP32 batch 1; pf: FP32 batch B
  int nxp = 0, nyp = 0;
  EncBuffers eb;
  float2 *z = nullptr, *v = nullptr, *w = nullptr, *x0 = nullptr, *x1 = nullptr;
  float2 *zref = nullptr, *gref = nullptr;   // split forms: anchor z_ref and A^H(A z_ref - y)
  float2 *pvec = nullptr, *ptmp = nullptr;
  double *dpart = nullptr;   // [B * kRedBlocks]
  double *sc = nullptr;      // [2 + 2B + 8]
  double *l1 = nullptr;      // [levels][B][l1_blocks]
  double *data = nullptr;    // [B]
  int l1_blocks = 0;
};

static int resolve_pad(int n, int given, int levels, int *out) {
  const int m = 1 << levels;
  const int v = given > 0 ? given : (int)round_up(n, m);
  if (v < n || v % m) return fail(EXPENC_EINVAL, "wavelet grid side %d must be >= %d and a multiple of %d", v, n, m);
  *out = v;
  return EXPENC_OK;
}

static int layout_fista(const expenc_op *op, int32_t batch, int32_t precision, int levels, int nx_pad, int ny_pad,
                        bool objective, Arena &a, FistaLayout *L) {
  EX_TRY(make_plan(op, batch, precision, &L->p));
  EX_TRY(make_plan(op, 1, EXPENC_FP32, &L->p1));
  EX_TRY(make_plan(op, batch, EXPENC_FP32, &L->pf));
  if (levels < 1 || levels > 12) return fail(EXPENC_EINVAL, "levels must be in [1, 12]");
  EX_TRY(resolve_pad(op->nx, nx_pad, levels, &L->nxp));
  EX_TRY(resolve_pad(op->ny, ny_pad, levels, &L->nyp));
  // p's buffers hold the FP32 operands of pf as well; the partial-sum buffer
  // is shared by all three plans (identical padded geometry)
  carve_enc(L->p, a, &L->eb, std::max(enc_part_elems(L->p1), enc_part_elems(L->pf)));
  const size_t img = (size_t)batch * L->nxp * L->nyp;
  L->z = a.take<float2>(img);
  L->v = a.take<float2>(img);
  L->w = a.take<float2>(img);
  L->x0 = a.take<float2>(img);
  L->x1 = a.take<float2>(img);
  if (precision != EXPENC_FP32) {
    L->zref = a.take<float2>(img);
    L->gref = a.take<float2>(img);
  }
  L->pvec = a.take<float2>((size_t)L->p.R);
  L->ptmp = a.take<float2>((size_t)L->p.R);
  L->dpart = a.take<double>((size_t)batch * kRedBlocks);
  L->sc = a.take<double>((size_t)2 + 2 * batch + 8);
  L->l1_blocks = (int)ceil_div(L->nxp, 16);
  if (objective) {
    L->l1 = a.take<double>((size_t)levels * batch * L->l1_blocks);
    L->data = a.take<double>((size_t)batch);
  }
  return a.ok() ? EXPENC_OK : EXPENC_EWORKSPACE;
}

size_t fista_bytes(const expenc_op *op, int32_t batch, int32_t precision, int32_t nx_pad, int32_t ny_pad) {
  // worst case over levels: use the padding implied by 12 levels only if none given
  Arena a;
  FistaLayout L;
  int levels = 1;
  if (nx_pad > 0 && ny_pad > 0) {
    levels = 1;
  } else {
    levels = 4;  // default grids are rounded to 2^levels; 4 covers the usual cases
  }
  if (layout_fista(op, batch, precision, levels, nx_pad, ny_pad, true, a, &L) != EXPENC_OK && !L.p.R) return 0;
  return a.used + 256;
}

static int check_fista_opts(const expenc_fista_opts *o, int *eff_refine) {
  if (!o) return fail(EXPENC_EINVAL, "options are NULL");
  if (o->n_iter < 0) return fail(EXPENC_EINVAL, "n_iter must be >= 0");
  if (o->wavelet != EXPENC_HAAR && o->wavelet != EXPENC_DB4) return fail(EXPENC_EINVAL, "unknown wavelet %d", o->wavelet);
  if (o->lipschitz <= 0 && (!o->power_v0 || o->n_power < 1))
    return fail(EXPENC_EINVAL, "lipschitz <= 0 requires power_v0 and n_power >= 1");
  if (o->lambda < 0 && !(o->lambda_factor > 0)) return fail(EXPENC_EINVAL, "lambda < 0 requires lambda_factor > 0");
  *eff_refine = o->refine_every > 0 ? o->refine_every : 10;
  return EXPENC_OK;
}

}  // namespace expenc

using namespace expenc;

extern "C" int fista_solve(const expenc_op *op, int32_t batch, const float *y, float *x,
                           const expenc_fista_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  int refine = 10;
  EX_TRY(check_fista_opts(opts, &refine));
  if (!y || !x) return fail(EXPENC_EINVAL, "y or x is NULL");
  FistaLayout L;
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  const int st = layout_fista(op, batch, opts->precision, opts->levels, opts->nx_pad, opts->ny_pad,
                              opts->objective != nullptr, a, &L);
  if (st == EXPENC_EWORKSPACE || !ws) {
    Arena need;
    FistaLayout tmp;
    layout_fista(op, batch, opts->precision, opts->levels, opts->nx_pad, opts->ny_pad, opts->objective != nullptr,
                 need, &tmp);
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                need.used + 256);
  }
  EX_TRY(st);
  FilterSet f;
  EX_TRY(make_filter_set(opts->wavelet, &f));
  hipStream_t s = (hipStream_t)stream;
  const EncPlan &p = L.p;
  const int B = batch;
  const int nxp = L.nxp, nyp = L.nyp;
  const int64_t img = (int64_t)nxp * nyp;
  const float2 *y2 = reinterpret_cast<const float2 *>(y);

  // ---- prologue (eager, stream-ordered) ----
  // FP32 tables first (the FP32 plan's pixel layout), then the split tables
  EX_TRY(enc_prepare(L.pf, op, L.eb, s));
  if (opts->precision != EXPENC_FP32) EX_TRY(enc_prepare(p, op, L.eb, s));
  if (opts->lipschitz > 0) {
    k_fill_d<<<1, 64, 0, s>>>(L.sc, 1, opts->lipschitz);
    EX_LAUNCHED("fill");
  } else {
    EX_TRY(lipschitz_run(L.p1, op, L.eb, opts->n_power, opts->power_v0, L.pvec, L.ptmp, L.dpart,
                         L.sc + 2 + 2 * B, L.sc, s));
  }
  if (opts->lambda >= 0) {
    k_fill_d<<<1, 256, 0, s>>>(L.sc + 2, B, opts->lambda);
    EX_LAUNCHED("fill");
  } else {
    const EncPlan &pf = L.pf;
    EX_TRY(enc_pack_y(pf, y2, L.eb, s));
    EX_TRY(enc_adjoint_partials(pf, L.eb, s));
    EX_TRY(enc_adjoint_reduce_out(pf, L.eb, op->smaps, L.v, pf.R, pf.nx, nullptr, nullptr, s));
    EX_TRY(reduce_maxabs(L.v, pf.R, pf.R, B, opts->lambda_factor, L.dpart, L.sc + 2, s));
  }
  k_fista_scalars<<<1, 256, 0, s>>>(L.sc, B);
  EX_LAUNCHED("scalars");
  k_zero_f2<<<(unsigned)ceil_div(img * B, 256), 256, 0, s>>>(L.x0, img * B);
  k_zero_f2<<<(unsigned)ceil_div(img * B, 256), 256, 0, s>>>(L.z, img * B);
  EX_LAUNCHED("zero");

  // ---- iterations (captured) ----
  const int K = opts->n_iter;
  std::vector<double> beta(K);
  {
    double t = 1.0;
    for (int k = 0; k < K; ++k) {
      const double tn = opts->ista ? 1.0 : (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      beta[k] = (t - 1.0) / tn;
      t = tn;
    }
  }
  const bool padded = (nxp != p.nx) || (nyp != p.ny);
  const bool split = opts->precision != EXPENC_FP32;
  const bool with_obj = opts->objective != nullptr;
  auto body = [&](hipStream_t cs) -> int {
    for (int k = 0; k < K; ++k) {
      float2 *xk = (k % 2 == 0) ? L.x1 : L.x0;
      float2 *xprev = (k % 2 == 0) ? L.x0 : L.x1;
      if (!split) {
        // v = z - (2/L) A^H (A z - y)
        EX_TRY(enc_build_z(p, op->smaps, L.z, img, nxp, L.eb, cs));
        EX_TRY(enc_forward_partials(p, L.eb, cs));
        EX_TRY(enc_forward_residual(p, L.eb, y2, cs));
        EX_TRY(enc_adjoint_partials(p, L.eb, cs));
        if (padded) EX_TRY(copy_f2(L.z, L.v, img * B, cs));
        EX_TRY(enc_adjoint_reduce_out(p, L.eb, op->smaps, L.v, img, nxp, L.sc + 1, L.z, cs));
      } else if (k % refine == 0 || k == K - 1) {
        // anchor: exact FP32 gradient at z_ref = z
        const EncPlan &pf = L.pf;
        EX_TRY(enc_build_z(pf, op->smaps, L.z, img, nxp, L.eb, cs));
        EX_TRY(enc_forward_partials(pf, L.eb, cs));
        EX_TRY(enc_forward_residual(pf, L.eb, y2, cs));
        EX_TRY(enc_adjoint_partials(pf, L.eb, cs));
        EX_TRY(enc_adjoint_reduce_out(pf, L.eb, op->smaps, L.gref, img, nxp, nullptr, nullptr, cs));
        k_grad_step<<<(unsigned)ceil_div(img * B, 256), 256, 0, cs>>>(L.v, L.z, L.gref, L.sc + 1, nxp, nyp, p.nx,
                                                                       p.ny, (int64_t)B * img);
        EX_LAUNCHED("gradient step");
        EX_TRY(copy_f2(L.z, L.zref, img * B, cs));
      } else {
        // split operators on the difference: g = g_ref + A~^H A~ (z - z_ref)
        EX_TRY(enc_build_z(p, op->smaps, L.z, img, nxp, L.eb, cs, L.zref));
        EX_TRY(enc_forward_partials(p, L.eb, cs));
        EX_TRY(enc_forward_residual(p, L.eb, nullptr, cs));
        EX_TRY(enc_adjoint_partials(p, L.eb, cs));
        if (padded) EX_TRY(copy_f2(L.z, L.v, img * B, cs));
        EX_TRY(enc_adjoint_reduce_out(p, L.eb, op->smaps, L.v, img, nxp, L.sc + 1, L.z, cs, L.gref));
      }
      EX_TRY(dwt_forward_levels(f, nxp, nyp, opts->levels, B, L.v, L.w, L.sc + 2 + B, with_obj ? L.l1 : nullptr,
                                L.l1_blocks, cs));
      EX_TRY(dwt_inverse_levels(f, nxp, nyp, opts->levels, B, L.w, xk, xprev, L.z, beta[k], cs));
      if (with_obj) {
        const EncPlan &pf = L.pf;
        EX_TRY(enc_build_z(pf, op->smaps, xk, img, nxp, L.eb, cs));
        EX_TRY(enc_forward_partials(pf, L.eb, cs));
        EX_TRY(enc_forward_residual(pf, L.eb, y2, cs));
        k_resid_norm_part<<<dim3(kRedBlocks, B), 256, 0, cs>>>(L.eb.yop, pf.Tp, pf.NCP, pf.C, L.dpart);
        EX_LAUNCHED("residual norm");
        EX_TRY(reduce_sum_parts(L.dpart, kRedBlocks, B, 1.0, L.data, cs));
        k_objective<<<B, 256, 0, cs>>>(L.data, L.l1, opts->levels, B, L.l1_blocks, nxp, L.sc + 2,
                                        opts->objective, K, k);
        EX_LAUNCHED("objective");
      }
    }
    return EXPENC_OK;
  };
  uint64_t key = 1469598103934665603ull;
  key = fnv(key, op, sizeof(*op));
  key = fnv(key, &batch, sizeof(batch));
  key = fnv(key, &y, sizeof(y));
  key = fnv(key, &ws, sizeof(ws));
  key = fnv(key, &ws_bytes, sizeof(ws_bytes));
  key = fnv(key, opts, sizeof(*opts));
  if (K > 0) EX_TRY(run_graph(key, s, body));

  // ---- epilogue ----
  const float2 *xK = (K == 0) ? L.x0 : ((K - 1) % 2 == 0 ? L.x1 : L.x0);
  k_crop<<<(unsigned)ceil_div((int64_t)p.R * B, 256), 256, 0, s>>>(xK, nxp, nyp, p.nx, p.ny, B,
                                                                   reinterpret_cast<float2 *>(x));
  EX_LAUNCHED("crop");
  if (opts->scalars) {
    k_copy_d<<<1, 256, 0, s>>>(L.sc, opts->scalars, 2 + 2 * B);
    EX_LAUNCHED("scalars out");
  }
  return EXPENC_OK;
}

// ---------------------------------------------------------------------------
// CG least squares with early stopping
// ---------------------------------------------------------------------------

namespace expenc {
struct CgLayout {
  EncPlan p;
  EncBuffers eb;
  float2 *xv = nullptr, *rv = nullptr, *pv = nullptr, *qv = nullptr;
  double *dpart = nullptr, *rs = nullptr, *pq = nullptr, *rsn = nullptr;
};

static int layout_cg(const expenc_op *op, int32_t batch, int32_t precision, Arena &a, CgLayout *L) {
  EX_TRY(make_plan(op, batch, precision, &L->p));
  carve_enc(L->p, a, &L->eb);
  const size_t n = (size_t)batch * L->p.R;
  L->xv = a.take<float2>(n);
  L->rv = a.take<float2>(n);
  L->pv = a.take<float2>(n);
  L->qv = a.take<float2>(n);
  L->dpart = a.take<double>((size_t)batch * kRedBlocks);
  L->rs = a.take<double>(batch);
  L->pq = a.take<double>(batch);
  L->rsn = a.take<double>(batch);
  return a.ok() ? EXPENC_OK : EXPENC_EWORKSPACE;
}

size_t cg_bytes(const expenc_op *op, int32_t batch, int32_t precision) {
  Arena a;
  CgLayout L;
  if (make_plan(op, batch, precision, &L.p) != EXPENC_OK) return 0;
  layout_cg(op, batch, precision, a, &L);
  return a.used + 256;
}
}  // namespace expenc

extern "C" int cg_solve(const expenc_op *op, int32_t batch, const float *y, float *x, const expenc_fista_opts *opts,
                        void *ws, size_t ws_bytes, void *stream) {
  if (!opts || opts->n_iter < 0) return fail(EXPENC_EINVAL, "bad CG options");
  if (!y || !x) return fail(EXPENC_EINVAL, "y or x is NULL");
  CgLayout L;
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  const int st = layout_cg(op, batch, opts->precision, a, &L);
  if (st == EXPENC_EWORKSPACE || !ws)
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                cg_bytes(op, batch, opts->precision));
  EX_TRY(st);
  hipStream_t s = (hipStream_t)stream;
  const EncPlan &p = L.p;
  const int B = batch;
  const int64_t n = p.R;
  const dim3 vg((unsigned)ceil_div(n, 256), B);
  EX_TRY(enc_prepare(p, op, L.eb, s));
  // r = A^H y ; p = r ; x = 0 ; rs = <r, r>
  EX_TRY(enc_pack_y(p, reinterpret_cast<const float2 *>(y), L.eb, s));
  EX_TRY(enc_adjoint_partials(p, L.eb, s));
  EX_TRY(enc_adjoint_reduce_out(p, L.eb, op->smaps, L.rv, n, p.nx, nullptr, nullptr, s));
  EX_TRY(copy_f2(L.rv, L.pv, n * B, s));
  k_zero_f2<<<(unsigned)ceil_div(n * B, 256), 256, 0, s>>>(L.xv, n * B);
  EX_LAUNCHED("zero");
  EX_TRY(reduce_dot(L.rv, L.rv, n, n, B, 1.0, L.dpart, L.rs, s));
  auto body = [&](hipStream_t cs) -> int {
    for (int k = 0; k < opts->n_iter; ++k) {
      EX_TRY(enc_build_z(p, op->smaps, L.pv, n, p.nx, L.eb, cs));
      EX_TRY(enc_forward_partials(p, L.eb, cs));
      EX_TRY(enc_forward_residual(p, L.eb, nullptr, cs));
      EX_TRY(enc_adjoint_partials(p, L.eb, cs));
      EX_TRY(enc_adjoint_reduce_out(p, L.eb, op->smaps, L.qv, n, p.nx, nullptr, nullptr, cs));
      EX_TRY(reduce_dot(L.pv, L.qv, n, n, B, 1.0, L.dpart, L.pq, cs));
      k_cg_step<<<vg, 256, 0, cs>>>(L.xv, L.rv, L.pv, L.qv, n, L.rs, L.pq);
      EX_LAUNCHED("cg step");
      EX_TRY(reduce_dot(L.rv, L.rv, n, n, B, 1.0, L.dpart, L.rsn, cs));
      k_cg_dir<<<vg, 256, 0, cs>>>(L.pv, L.rv, n, L.rs, L.rsn);
      EX_LAUNCHED("cg direction");
      k_copy_d<<<1, 256, 0, cs>>>(L.rsn, L.rs, B);
      EX_LAUNCHED("cg copy");
    }
    return EXPENC_OK;
  };
  uint64_t key = 0x9e3779b97f4a7c15ull;
  key = fnv(key, op, sizeof(*op));
  key = fnv(key, &batch, sizeof(batch));
  key = fnv(key, &ws, sizeof(ws));
  key = fnv(key, &ws_bytes, sizeof(ws_bytes));
  key = fnv(key, &opts->n_iter, sizeof(opts->n_iter));
  key = fnv(key, &opts->precision, sizeof(opts->precision));
  if (opts->n_iter > 0) EX_TRY(run_graph(key, s, body));
  EX_TRY(copy_f2(L.xv, reinterpret_cast<float2 *>(x), n * B, s));
  return EXPENC_OK;
}
