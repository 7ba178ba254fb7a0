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
#include <functional>
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

// per problem p: sc[P + p] = -2/L_p; per column: tau = lambda/L_p
__global__ void k_fista_scalars(double *sc, int P, int B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * B) return;
  const int p = i / B;
  const double L = sc[p];
  if (i % B == 0) sc[P + p] = L > 0.0 ? -2.0 / L : 0.0;
  sc[2 * P + P * B + i] = L > 0.0 ? sc[2 * P + i] / L : 0.0;
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

// objective[b*K + k] = data[b] + lambda[b] * sum_{level, tile} l1[level][b][tile]
// (level j wrote ceil(hx_j/16) * ceil(hy_j/8) tile sums out of nblk slots,
// hx_j = (nxp >> j)/2, hy_j = (nyp >> j)/2)
// With status: F(x_k) above f0[b] = F(0) = ||y_b||^2 flags divergence, a
// non-finite F flags a non-finite iterate.
__global__ __launch_bounds__(256) void k_objective(const double *__restrict__ data, const double *__restrict__ l1,
                                                   int levels, int B, int nblk, int nxp, int nyp,
                                                   const double *__restrict__ lam, double *__restrict__ obj, int K,
                                                   int k, const double *__restrict__ f0, unsigned *status) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < levels * nblk; i += blockDim.x) {
    const int lev = i / nblk, blk = i % nblk;
    const int tiles = (((nxp >> lev) / 2 + 15) / 16) * (((nyp >> lev) / 2 + 7) / 8);
    if (blk < tiles) s += l1[((int64_t)lev * B + b) * nblk + blk];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double F = data[b] + lam[b] * red[0];
    obj[(int64_t)b * K + k] = F;
    if (status) {
      if (!isfinite(F)) atomicOr(status, kStatusNonFinite);
      else if (F > f0[b]) atomicOr(status, kStatusDiverged);
    }
  }
}

// CG: alpha = rs/pq; x += alpha p; r -= alpha q
__global__ void k_cg_step(float2 *__restrict__ x, float2 *__restrict__ r, const float2 *__restrict__ p,
                          const float2 *__restrict__ q, int64_t n, const double *__restrict__ rs,
                          const double *__restrict__ pq, unsigned *status) {
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
  flag_nonfinite(status, xv);
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
// (alpha_dev holds one value per problem of B images)
__global__ void k_grad_step(float2 *__restrict__ v, const float2 *__restrict__ z, const float2 *__restrict__ g,
                            const double *__restrict__ alpha_dev, int nxp, int nyp, int nx, int ny, int64_t n,
                            int B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t img = (int64_t)nxp * nyp;
  const int64_t p = i % img;
  const int yy = (int)(p / nxp), xx = (int)(p % nxp);
  float2 o = z[i];
  if (yy < ny && xx < nx) {
    const float a = (float)alpha_dev[(i / img) / B];
    o.x += a * g[i].x;
    o.y += a * g[i].y;
  }
  v[i] = o;
}

__global__ void k_copy_d(const double *in, double *out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

__global__ void k_clear_status(unsigned *status) {
  if (threadIdx.x == 0) status[0] = 0u;
}

int clear_status(unsigned *status, hipStream_t s) {
  k_clear_status<<<1, 64, 0, s>>>(status);
  EX_LAUNCHED("status clear");
  return EXPENC_OK;
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
// Held from the start of a capture to its end: the per-device capture stream
// (and the batched solver's fork streams) serve one capture at a time.
static std::mutex g_capture_mu;
static constexpr size_t kGraphCacheMax = 64;

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
// Launches the cached graph of (key, device) on s; false when there is none.
static bool launch_cached(uint64_t key, int dev, hipStream_t s, int *rc) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto &e : g_graphs)
    if (e.key == key && e.device == dev) {
      e.last_stream = s;
      const hipError_t err = hipGraphLaunch(e.exec, s);
      *rc = err == hipSuccess ? EXPENC_OK : fail(EXPENC_EHIP, "graph launch failed: %s", hipGetErrorString(err));
      return true;
    }
  return false;
}

template <class Body>
static int run_graph(uint64_t key, hipStream_t s, Body body) {
  if (!graphs_enabled()) return body(s);
  int dev = 0;
  EX_HIP(hipGetDevice(&dev));
  int rc = EXPENC_OK;
  if (launch_cached(key, dev, s, &rc)) return rc;
  // one capture at a time; a thread that waited here may find the graph
  // another thread has just captured for the same key
  std::lock_guard<std::mutex> cap(g_capture_mu);
  if (launch_cached(key, dev, s, &rc)) return rc;
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

// Shared with the other graph-captured solvers.
int run_captured(uint64_t key, hipStream_t s, const std::function<int(hipStream_t)> &body) {
  return run_graph(key, s, body);
}
uint64_t hash_bytes(uint64_t h, const void *p, size_t n) { return fnv(h, p, n); }

// ---------------------------------------------------------------------------
// FISTA for a group of P problems of identical shape (P = 1 for
// fista_solve), each with B columns sharing its operator.  Scalars in sc:
// L[p] at sc[p], alpha = -2/L at sc[P + p], lambda at sc[2P + p*B + b],
// tau = lambda/L at sc[2P + PB + p*B + b], then scratch.
// ---------------------------------------------------------------------------

struct FistaLayout {
  EncPlan p, p1, pf;  // p: iteration precision (batch B); p1: batch 1 (power iteration); pf: FP32 batch B
  int P = 1, B = 1;
  int nxp = 0, nyp = 0;
  EncBuffers eb;
  float2 *z = nullptr, *v = nullptr, *w = nullptr, *x0 = nullptr, *x1 = nullptr;
  // zref (split forms): the anchor z_ref; gref: A^H(A z_ref - y) (split
  // forms), and the lambda rule's -A^H y, the gradient at z_0 = 0 (all forms)
  float2 *zref = nullptr, *gref = nullptr;
  float2 *pvec = nullptr, *ptmp = nullptr;
  double *dpart = nullptr;   // [P * B * kRedBlocks]
  double *sc = nullptr;      // [2P + 2PB + 3P]
  double *l1 = nullptr;      // [levels][B][l1_blocks]   (P == 1 only)
  double *data = nullptr;    // [B]
  double *f0 = nullptr;      // [B] F(0) = ||y_b||^2   (P == 1, objective only)
  unsigned *status = nullptr;  // the call's status word (start of the workspace)
  int l1_blocks = 0;
  double *lam_of(int) const { return sc + 2 * P; }
  double *tau() const { return sc + 2 * P + P * B; }
  double *scratch() const { return sc + 2 * P + 2 * P * B; }
};

static int resolve_pad(int n, int given, int levels, int *out) {
  const int m = 1 << levels;
  const int v = given > 0 ? given : (int)round_up(n, m);
  if (v < n || v % m) return fail(EXPENC_EINVAL, "wavelet grid side %d must be >= %d and a multiple of %d", v, n, m);
  *out = v;
  return EXPENC_OK;
}

static int layout_fista(const expenc_op *op, int32_t nprob, int32_t batch, int32_t precision, int levels, int nx_pad,
                        int ny_pad, bool objective, Arena &a, FistaLayout *L) {
  EX_TRY(make_plan(op, batch, precision, &L->p, nprob));
  // the power iteration runs in the solve's precision when each problem has
  // one image (then p1 and p share geometry, tables and coil table)
  EX_TRY(make_plan(op, 1, batch == 1 ? precision : EXPENC_FP32, &L->p1, nprob));
  EX_TRY(make_plan(op, batch, EXPENC_FP32, &L->pf, nprob));
  if (levels < 1 || levels > 12) return fail(EXPENC_EINVAL, "levels must be in [1, 12]");
  if (objective && nprob != 1) return fail(EXPENC_EUNSUPPORTED, "objective traces are per single problem");
  EX_TRY(resolve_pad(op->nx, nx_pad, levels, &L->nxp));
  EX_TRY(resolve_pad(op->ny, ny_pad, levels, &L->nyp));
  L->P = nprob;
  L->B = batch;
  // p's buffers hold the FP32 operands of pf as well; the partial-sum buffer
  // is shared by all three plans (identical padded geometry)
  carve_enc(L->p, a, &L->eb, std::max(enc_part_elems(L->p1), enc_part_elems(L->pf)));
  const size_t img = (size_t)nprob * batch * L->nxp * L->nyp;
  L->z = a.take<float2>(img);
  L->v = a.take<float2>(img);
  L->w = a.take<float2>(img);
  L->x0 = a.take<float2>(img);
  L->x1 = a.take<float2>(img);
  if (precision != EXPENC_FP32) L->zref = a.take<float2>(img);
  L->gref = a.take<float2>(img);
  L->pvec = a.take<float2>((size_t)L->p.R * nprob);
  L->ptmp = a.take<float2>((size_t)L->p.R * nprob);
  L->dpart = a.take<double>((size_t)nprob * batch * kRedBlocks);
  L->sc = a.take<double>((size_t)2 * nprob + 2 * nprob * batch + 3 * nprob + 8);
  L->l1_blocks = dwt2_tiles(L->nxp, L->nyp, 0);
  if (objective) {
    L->l1 = a.take<double>((size_t)levels * batch * L->l1_blocks);
    L->data = a.take<double>((size_t)batch);
    L->f0 = a.take<double>((size_t)batch);
  }
  return a.ok() ? EXPENC_OK : EXPENC_EWORKSPACE;
}

size_t fista_bytes(const expenc_op *op, int32_t batch, int32_t precision, int32_t nx_pad, int32_t ny_pad) {
  // default grids are rounded to 2^levels; 4 levels covers the usual cases
  Arena a;
  FistaLayout L;
  take_status(a);
  const int levels = (nx_pad > 0 && ny_pad > 0) ? 1 : 4;
  if (layout_fista(op, 1, batch, precision, levels, nx_pad, ny_pad, true, a, &L) != EXPENC_OK && !L.p.R) return 0;
  return a.used + 256;
}

static int check_fista_opts(const expenc_fista_opts *o, int *eff_refine) {
  if (!o) return fail(EXPENC_EINVAL, "options are NULL");
  if (o->n_iter < 0) return fail(EXPENC_EINVAL, "n_iter must be >= 0");
  if (o->batch_launch != EXPENC_BATCH_FORKED && o->batch_launch != EXPENC_BATCH_GROUPED)
    return fail(EXPENC_EINVAL, "unknown batch_launch %d", o->batch_launch);
  if (o->wavelet != EXPENC_HAAR && o->wavelet != EXPENC_DB4) return fail(EXPENC_EINVAL, "unknown wavelet %d", o->wavelet);
  if (o->lipschitz <= 0 && (!o->power_v0 || o->n_power < 1))
    return fail(EXPENC_EINVAL, "lipschitz <= 0 requires power_v0 and n_power >= 1");
  if (o->lambda < 0 && !(o->lambda_factor > 0)) return fail(EXPENC_EINVAL, "lambda < 0 requires lambda_factor > 0");
  if (o->anchor != EXPENC_ANCHOR_ENDS && o->anchor != EXPENC_ANCHOR_FP32 && o->anchor != EXPENC_ANCHOR_SPLIT)
    return fail(EXPENC_EINVAL, "unknown anchor mode %d", o->anchor);
  if (o->reserved != 0) return fail(EXPENC_EINVAL, "reserved option field must be 0");
  *eff_refine = o->refine_every > 0 ? o->refine_every : default_refine(o->precision, o->anchor);
  return EXPENC_OK;
}

// One group's solve, split into stream-ordered phases so that several groups
// can share one captured graph.
struct FistaGroup {
  const expenc_op *op = nullptr;  // packed operator of the group
  FistaLayout L;
  FilterSet f;
  const expenc_fista_opts *opts = nullptr;
  const float2 *y = nullptr;      // [P][B][T][C]
  int refine = 0;
  std::vector<double> beta;
  bool gref_at_zero = false;  // gref holds -A^H y (FP32) from the lambda rule

  int prologue(hipStream_t s) {
    const EncPlan &p = L.p, &pf = L.pf;
    const int P = L.P, B = L.B;
    const int64_t img = (int64_t)L.nxp * L.nyp;
    // FP32 tables first (the FP32 plan's pixel layout), then the split tables
    EX_TRY(enc_prepare(pf, op, L.eb, s));
    if (opts->precision != EXPENC_FP32) EX_TRY(enc_prepare(p, op, L.eb, s));
    if (opts->lipschitz > 0) {
      k_fill_d<<<(unsigned)ceil_div(P, 256), 256, 0, s>>>(L.sc, P, opts->lipschitz);
      EX_LAUNCHED("fill");
    } else {
      EX_TRY(lipschitz_run(L.p1, op, L.eb, opts->n_power, opts->power_v0, L.pvec, L.ptmp, L.dpart, L.scratch(),
                           L.sc, s));
    }
    if (opts->lambda >= 0) {
      k_fill_d<<<(unsigned)ceil_div(P * B, 256), 256, 0, s>>>(L.lam_of(0), P * B, opts->lambda);
      EX_LAUNCHED("fill");
    } else {
      // -A^H y in FP32 on the wavelet grid (zero padding): lambda =
      // factor * max|A^H y|, and the first iteration's gradient at z_0 = 0
      // (2/L times it), so that iteration needs no contraction of its own
      k_zero_f2<<<(unsigned)ceil_div(img * P * B, 256), 256, 0, s>>>(L.gref, img * P * B);
      EX_LAUNCHED("zero");
      EX_TRY(enc_pack_y(pf, y, L.eb, s, -1.f));
      EX_TRY(enc_adjoint_partials(pf, L.eb, s));
      EX_TRY(enc_adjoint_reduce_out(pf, L.eb, op->smaps, L.gref, img, L.nxp, nullptr, nullptr, s, nullptr,
                                    img * B));
      EX_TRY(reduce_maxabs(L.gref, img, img, P * B, opts->lambda_factor, L.dpart, L.lam_of(0), s));
      gref_at_zero = true;
    }
    k_fista_scalars<<<(unsigned)ceil_div(P * B, 256), 256, 0, s>>>(L.sc, P, B);
    EX_LAUNCHED("scalars");
    if (opts->objective) {
      // F(0) = ||y||^2, the divergence bar of the objective trace
      const int64_t ty = p.T * p.C;
      EX_TRY(reduce_dot(y, y, ty, ty, B, 1.0, L.dpart, L.f0, s));
    }
    k_zero_f2<<<(unsigned)ceil_div(img * P * B, 256), 256, 0, s>>>(L.x0, img * P * B);
    k_zero_f2<<<(unsigned)ceil_div(img * P * B, 256), 256, 0, s>>>(L.z, img * P * B);
    EX_LAUNCHED("zero");
    const int K = opts->n_iter;
    beta.assign(K, 0.0);
    double t = 1.0;
    for (int k = 0; k < K; ++k) {
      const double tn = opts->ista ? 1.0 : (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      beta[k] = (t - 1.0) / tn;
      t = tn;
    }
    return EXPENC_OK;
  }

  int body(hipStream_t cs) {
    for (int k = 0; k < opts->n_iter; ++k) EX_TRY(iteration(cs, k, kStageAll));
    return EXPENC_OK;
  }

  // Whether iteration k applies the split operators to z - z_ref (the
  // iterations whose contractions a grouped batched launch takes over).
  bool split_difference(int k) const {
    const int K = opts->n_iter;
    return opts->precision != EXPENC_FP32 && !(k == 0 && gref_at_zero) && !(k % refine == 0 || k == K - 1);
  }

  // Stages of one iteration: kStagePre ends before the forward contraction,
  // kStageMid lies between the two contractions, kStagePost follows the
  // adjoint.  The contractions themselves run only with kStageAll; a caller
  // that runs the stages one at a time issues them in between (only for the
  // iterations of split_difference; the others run with kStageAll).
  static constexpr int kStagePre = 1, kStageMid = 2, kStagePost = 4, kStageAll = 7;

  int iteration(hipStream_t cs, int k, int stage) {
    const EncPlan &p = L.p, &pf = L.pf;
    const int P = L.P, B = L.B;
    const int nxp = L.nxp, nyp = L.nyp;
    const int64_t img = (int64_t)nxp * nyp;
    const int64_t pimg = img * B;  // elements between problems
    const int64_t all = pimg * P;
    const bool padded = (nxp != p.nx) || (nyp != p.ny);
    const bool split = opts->precision != EXPENC_FP32;
    const bool with_obj = opts->objective != nullptr;
    const double *alpha = L.sc + P;
    const int K = opts->n_iter;
    const bool whole = stage == kStageAll;
    {
      float2 *xk = (k % 2 == 0) ? L.x1 : L.x0;
      float2 *xprev = (k % 2 == 0) ? L.x0 : L.x1;
      // z_0 = 0, so the first residual A z - y is -y without a forward product
      auto residual_fp32 = [&](const EncPlan &q) -> int {
        if (k == 0) return enc_pack_y(q, y, L.eb, cs, -1.f);
        EX_TRY(enc_build_z(q, op->smaps, L.z, img, nxp, L.eb, cs, nullptr, pimg));
        EX_TRY(enc_forward_partials(q, L.eb, cs));
        return enc_forward_residual(q, L.eb, y, cs);
      };
      const int pnx = padded ? nxp : 0, pny = padded ? nyp : 0;
      if (!split_difference(k) && !whole) return fail(EXPENC_EINVAL, "iteration %d runs whole", k);
      if (k == 0 && gref_at_zero) {
        // v = z_0 - (2/L) A^H y from the prologue's FP32 -A^H y (also the
        // split forms' first anchor: z_ref = z_0)
        k_grad_step<<<(unsigned)ceil_div(all, 256), 256, 0, cs>>>(L.v, L.z, L.gref, alpha, nxp, nyp, p.nx, p.ny, all, B);
        EX_LAUNCHED("gradient step");
        if (split) EX_TRY(copy_f2(L.z, L.zref, all, cs));
      } else if (!split) {
        // v = z - (2/L) A^H (A z - y)
        EX_TRY(residual_fp32(p));
        EX_TRY(enc_adjoint_partials(p, L.eb, cs));
        EX_TRY(enc_adjoint_reduce_out(p, L.eb, op->smaps, L.v, img, nxp, alpha, L.z, cs, nullptr, pimg, pnx, pny));
      } else if (k % refine == 0 || k == K - 1) {
        // anchor: the gradient at z_ref = z, in FP32 or in the split form
        const EncPlan &pa = anchor_in_fp32(opts->anchor, k, K) ? pf : p;
        EX_TRY(residual_fp32(pa));
        EX_TRY(enc_adjoint_partials(pa, L.eb, cs));
        EX_TRY(enc_adjoint_reduce_out(pa, L.eb, op->smaps, L.gref, img, nxp, nullptr, nullptr, cs, nullptr, pimg));
        k_grad_step<<<(unsigned)ceil_div(all, 256), 256, 0, cs>>>(L.v, L.z, L.gref, alpha, nxp, nyp, p.nx, p.ny, all, B);
        EX_LAUNCHED("gradient step");
        EX_TRY(copy_f2(L.z, L.zref, all, cs));
      } else {
        // split operators on the difference: g = g_ref + A~^H A~ (z - z_ref)
        if (stage & kStagePre) EX_TRY(enc_build_z(p, op->smaps, L.z, img, nxp, L.eb, cs, L.zref, pimg));
        if (whole) EX_TRY(enc_forward_partials(p, L.eb, cs));
        if (stage & kStageMid) EX_TRY(enc_forward_residual(p, L.eb, nullptr, cs));
        if (whole) EX_TRY(enc_adjoint_partials(p, L.eb, cs));
        if (stage & kStagePost)
          EX_TRY(enc_adjoint_reduce_out(p, L.eb, op->smaps, L.v, img, nxp, alpha, L.z, cs, L.gref, pimg, pnx, pny));
      }
      if (!(stage & kStagePost)) return EXPENC_OK;
      // x_k = W^H S_tau(W v), z = x_k + beta_k (x_k - x_{k-1}); v and x_k serve
      // as the transform's ping-pong buffers
      EX_TRY(dwt2_prox(f, nxp, nyp, opts->levels, P * B, L.v, L.w, xk, xprev, L.z, beta[k], L.tau(),
                       with_obj ? L.l1 : nullptr, L.l1_blocks, cs, L.status));
      if (with_obj) {
        EX_TRY(enc_build_z(pf, op->smaps, xk, img, nxp, L.eb, cs));
        EX_TRY(enc_forward_partials(pf, L.eb, cs));
        EX_TRY(enc_forward_residual(pf, L.eb, y, cs));
        k_resid_norm_part<<<dim3(kRedBlocks, B), 256, 0, cs>>>(L.eb.yop, pf.Tp, pf.NCP, pf.C, L.dpart);
        EX_LAUNCHED("residual norm");
        EX_TRY(reduce_sum_parts(L.dpart, kRedBlocks, B, 1.0, L.data, cs));
        k_objective<<<B, 256, 0, cs>>>(L.data, L.l1, opts->levels, B, L.l1_blocks, nxp, nyp, L.lam_of(0),
                                        opts->objective, K, k, L.f0, L.status);
        EX_LAUNCHED("objective");
      }
    }
    return EXPENC_OK;
  }

  // crop of x_K into out [P][B][ny][nx]
  int epilogue(float2 *out, hipStream_t s) {
    const int K = opts->n_iter;
    const float2 *xK = (K == 0) ? L.x0 : ((K - 1) % 2 == 0 ? L.x1 : L.x0);
    const int PB = L.P * L.B;
    k_crop<<<(unsigned)ceil_div((int64_t)L.p.R * PB, 256), 256, 0, s>>>(xK, L.nxp, L.nyp, L.p.nx, L.p.ny, PB, out);
    EX_LAUNCHED("crop");
    return EXPENC_OK;
  }
};

}  // namespace expenc

using namespace expenc;

extern "C" int fista_solve(const expenc_op *op, int32_t batch, const float *y, float *x,
                           const expenc_fista_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  int refine = 0;
  EX_TRY(check_fista_opts(opts, &refine));
  if (!y || !x) return fail(EXPENC_EINVAL, "y or x is NULL");
  FistaGroup G;
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  unsigned *status = take_status(a);
  const int st = layout_fista(op, 1, batch, opts->precision, opts->levels, opts->nx_pad, opts->ny_pad,
                              opts->objective != nullptr, a, &G.L);
  if (st == EXPENC_EWORKSPACE || !ws) {
    Arena need;
    FistaLayout tmp;
    take_status(need);
    layout_fista(op, 1, batch, opts->precision, opts->levels, opts->nx_pad, opts->ny_pad, opts->objective != nullptr,
                 need, &tmp);
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                need.used + 256);
  }
  EX_TRY(st);
  EX_TRY(make_filter_set(opts->wavelet, &G.f));
  G.op = op;
  G.opts = opts;
  G.y = reinterpret_cast<const float2 *>(y);
  G.refine = refine;
  G.L.status = status;
  hipStream_t s = (hipStream_t)stream;
  EX_TRY(clear_status(status, s));
  EX_TRY(G.prologue(s));
  uint64_t key = 1469598103934665603ull;
  key = fnv(key, op, sizeof(*op));
  key = fnv(key, &batch, sizeof(batch));
  key = fnv(key, &y, sizeof(y));
  key = fnv(key, &ws, sizeof(ws));
  key = fnv(key, &ws_bytes, sizeof(ws_bytes));
  key = fnv(key, opts, sizeof(*opts));
  const uint64_t gen = tuning_generation();
  key = fnv(key, &gen, sizeof(gen));
  if (opts->n_iter > 0) EX_TRY(run_graph(key, s, [&](hipStream_t cs) { return G.body(cs); }));
  EX_TRY(G.epilogue(reinterpret_cast<float2 *>(x), s));
  if (opts->scalars) {
    k_copy_d<<<(unsigned)ceil_div(2 + 2 * batch, 256), 256, 0, s>>>(G.L.sc, opts->scalars, 2 + 2 * batch);
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
  unsigned *status = nullptr;
  float2 *xv = nullptr, *rv = nullptr, *pv = nullptr, *qv = nullptr;
  double *dpart = nullptr, *rs = nullptr, *pq = nullptr, *rsn = nullptr;
};

static int layout_cg(const expenc_op *op, int32_t batch, int32_t precision, Arena &a, CgLayout *L) {
  EX_TRY(make_plan(op, batch, precision, &L->p));
  L->status = take_status(a);
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
  EX_TRY(clear_status(L.status, s));
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
      k_cg_step<<<vg, 256, 0, cs>>>(L.xv, L.rv, L.pv, L.qv, n, L.rs, L.pq, L.status);
      EX_LAUNCHED("cg step");
      EX_TRY(reduce_dot(L.rv, L.rv, n, n, B, 1.0, L.dpart, L.rsn, cs));
      k_cg_dir<<<vg, 256, 0, cs>>>(L.pv, L.rv, n, L.rs, L.rsn);
      EX_LAUNCHED("cg direction");
      k_copy_d<<<(unsigned)ceil_div(B, 256), 256, 0, cs>>>(L.rsn, L.rs, B);
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
  const uint64_t gen = tuning_generation();
  key = fnv(key, &gen, sizeof(gen));
  if (opts->n_iter > 0) EX_TRY(run_graph(key, s, body));
  EX_TRY(copy_f2(L.xv, reinterpret_cast<float2 *>(x), n * B, s));
  return EXPENC_OK;
}

// ---------------------------------------------------------------------------
// Batched FISTA over independent problems of mixed shapes.  Problems with the
// same geometry form a group whose operands are packed contiguously
// ([P][...] per array), so that every contraction, table and wavelet pass of
// the group is ONE launch with the problem index in the grid.  All groups'
// iteration loops are captured into one graph, each group on its own forked
// capture stream, so small passes of different groups overlap.
// ---------------------------------------------------------------------------

namespace expenc {

struct Vals64 {
  double v[64];
};

__global__ void k_set_vals(double *out, Vals64 vals, int n) {
  const int i = threadIdx.x;
  if (i < n) out[i] = vals.v[i];
}

static bool same_geometry(const expenc_op &a, const expenc_op &b) {
  return a.nx == b.nx && a.ny == b.ny && a.ncoils == b.ncoils && a.nbasis == b.nbasis && a.nsamples == b.nsamples &&
         a.basis_kind == b.basis_kind && (a.dw0 != nullptr) == (b.dw0 != nullptr) && a.fov_x == b.fov_x &&
         a.fov_y == b.fov_y;
}

struct BatchPlan {
  std::vector<std::vector<int>> members;  // problem indices per group, in input order
  std::vector<FistaGroup> groups;
  std::vector<expenc_op> packed;          // one packed operator per group
  std::vector<double *> z0s;
  unsigned *status = nullptr;             // the call's status word (start of the workspace)
};

static int layout_batched(int32_t nprob, const expenc_op *ops, int32_t batch, const expenc_fista_opts *o, Arena &a,
                          BatchPlan *bp) {
  if (nprob < 1 || nprob > 65535) return fail(EXPENC_EINVAL, "problem count %d out of range", nprob);
  if (!ops) return fail(EXPENC_EINVAL, "ops is NULL");
  if (o->objective || o->scalars) return fail(EXPENC_EUNSUPPORTED, "objective/scalars outputs are per single solve");
  if (o->nx_pad > 0 || o->ny_pad > 0)
    return fail(EXPENC_EINVAL, "batched solves pad each problem to 2^levels (nx_pad, ny_pad must be 0)");
  bp->status = take_status(a);
  for (int i = 0; i < nprob; ++i) {
    int g = 0;
    for (; g < (int)bp->members.size(); ++g)
      if (same_geometry(ops[bp->members[g][0]], ops[i])) break;
    if (g == (int)bp->members.size()) bp->members.emplace_back();
    bp->members[g].push_back(i);
  }
  const int NG = (int)bp->members.size();
  bp->groups.resize(NG);
  bp->packed.resize(NG);
  bp->z0s.resize(NG);
  for (int g = 0; g < NG; ++g) {
    const std::vector<int> &m = bp->members[g];
    const int P = (int)m.size();
    const expenc_op &o0 = ops[m[0]];
    expenc_op &q = bp->packed[g];
    q = o0;
    const size_t R = (size_t)o0.nx * o0.ny, T = (size_t)o0.nsamples, Lb = (size_t)std::max(o0.nbasis, 0);
    // packed inputs (each member's arrays copied in, input order)
    q.coef = Lb ? a.take<double>(P * T * Lb) : nullptr;
    q.time = a.take<double>(P * T);
    q.basis = (Lb && o0.basis_kind == EXPENC_BASIS_MAPS) ? a.take<double>(P * Lb * R) : nullptr;
    q.dw0 = o0.dw0 ? a.take<double>(P * R) : nullptr;
    q.smaps = reinterpret_cast<const float *>(a.take<float2>(P * (size_t)o0.ncoils * R));
    bp->z0s[g] = a.take<double>(P);
    bp->groups[g].y = a.take<float2>((size_t)P * batch * T * o0.ncoils);
    // the plans take geometry from the first member (make_plan also checks
    // its pointers, which the packed copies may not have yet when sizing)
    const expenc_op &chk = o0;
    // (a short arena is only known at the end: keep carving to learn the total)
    const int st = layout_fista(&chk, P, batch, o->precision, o->levels, 0, 0, false, a, &bp->groups[g].L);
    if (st != EXPENC_OK && st != EXPENC_EWORKSPACE) return st;
    bp->groups[g].L.p.z0s = bp->groups[g].L.p1.z0s = bp->groups[g].L.pf.z0s = bp->z0s[g];
  }
  return a.ok() ? EXPENC_OK : EXPENC_EWORKSPACE;
}

// Fork/join resources of the batched capture: up to kForkStreams streams
// (group g is captured on stream g % kForkStreams) and one event per group
// plus the fork event, per device.  They are created before a capture
// begins and kept until the process ends, so that no stream or event is
// created or destroyed while a stream is being captured (an event recorded
// into a capture stays referenced by the capture until it ends).  The pool
// serves one solve at a time: the caller holds *hold while it forks.
constexpr int kForkStreams = 8;
struct ForkPool {
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
};

static int fork_resources(int device, int ngroups, std::vector<hipStream_t> *streams,
                          std::vector<hipEvent_t> *events, std::unique_lock<std::mutex> *hold) {
  static std::mutex mu;
  static std::vector<ForkPool> pools;
  *hold = std::unique_lock<std::mutex>(mu);
  if ((int)pools.size() <= device) pools.resize(device + 1);
  ForkPool &fp = pools[device];
  const int ns = std::min(ngroups, kForkStreams);
  while ((int)fp.streams.size() < ns) {
    hipStream_t st = nullptr;
    EX_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    fp.streams.push_back(st);
  }
  while ((int)fp.events.size() < ngroups + 1) {
    hipEvent_t e = nullptr;
    EX_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    fp.events.push_back(e);
  }
  streams->assign(fp.streams.begin(), fp.streams.begin() + ns);
  events->assign(fp.events.begin(), fp.events.begin() + ngroups + 1);
  return EXPENC_OK;
}

}  // namespace expenc

extern "C" size_t fista_batched_workspace_size(int32_t nprob, const expenc_op *ops, int32_t batch,
                                               const expenc_fista_opts *opts) {
  int refine = 0;
  if (check_fista_opts(opts, &refine) != EXPENC_OK) return 0;
  Arena a;
  BatchPlan bp;
  if (layout_batched(nprob, ops, batch, opts, a, &bp) != EXPENC_OK && a.used == 0) return 0;
  return a.used + 256;
}

extern "C" int fista_solve_batched(int32_t nprob, const expenc_op *ops, int32_t batch, const float *const *y,
                                   float *const *x, const expenc_fista_opts *opts, void *ws, size_t ws_bytes,
                                   void *stream) {
  int refine = 0;
  EX_TRY(check_fista_opts(opts, &refine));
  if (!y || !x) return fail(EXPENC_EINVAL, "y or x pointer array is NULL");
  for (int i = 0; i < nprob; ++i)
    if (!y[i] || !x[i]) return fail(EXPENC_EINVAL, "problem %d: y or x is NULL", i);
  for (int i = 0; i < nprob; ++i) {
    EncPlan chk;
    EX_TRY(make_plan(&ops[i], batch, opts->precision, &chk));
  }
  BatchPlan bp;
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  const int st = layout_batched(nprob, ops, batch, opts, a, &bp);
  if (st == EXPENC_EWORKSPACE || !ws)
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                fista_batched_workspace_size(nprob, ops, batch, opts));
  EX_TRY(st);
  FilterSet f;
  EX_TRY(make_filter_set(opts->wavelet, &f));
  hipStream_t s = (hipStream_t)stream;
  const int NG = (int)bp.members.size();
  // the grouped launch pattern needs one shape class for every group
  bool grouped = opts->batch_launch == EXPENC_BATCH_GROUPED && opts->precision != EXPENC_FP32;
  for (int g = 0; g < NG && grouped; ++g) grouped = split_groupable(bp.groups[0].L.p, bp.groups[g].L.p);
  if (opts->batch_launch == EXPENC_BATCH_GROUPED && !grouped)
    return fail(EXPENC_EUNSUPPORTED, "grouped batch launches need split precision and the solid-harmonic kind "
                                     "with one column width for every group");
  EX_TRY(clear_status(bp.status, s));
  // gather the members' inputs into the packed group arrays
  for (int g = 0; g < NG; ++g) {
    const std::vector<int> &m = bp.members[g];
    const expenc_op &q = bp.packed[g];
    const size_t R = (size_t)q.nx * q.ny, T = (size_t)q.nsamples, Lb = (size_t)std::max(q.nbasis, 0);
    const size_t ny = (size_t)batch * T * q.ncoils;
    Vals64 z0v{};
    for (size_t j = 0; j < m.size(); ++j) {
      const expenc_op &o = ops[m[j]];
      auto cp = [&](const void *dst, const void *src, size_t bytes) {
        return hipMemcpyAsync(const_cast<void *>(dst), src, bytes, hipMemcpyDeviceToDevice, s);
      };
      if (Lb) EX_HIP(cp(q.coef + j * T * Lb, o.coef, T * Lb * sizeof(double)));
      EX_HIP(cp(q.time + j * T, o.time, T * sizeof(double)));
      if (q.basis) EX_HIP(cp(q.basis + j * Lb * R, o.basis, Lb * R * sizeof(double)));
      if (q.dw0) EX_HIP(cp(q.dw0 + j * R, o.dw0, R * sizeof(double)));
      EX_HIP(cp(q.smaps + j * q.ncoils * R * 2, o.smaps, q.ncoils * R * sizeof(float2)));
      EX_HIP(cp(bp.groups[g].y + j * ny, y[m[j]], ny * sizeof(float2)));
      z0v.v[j % 64] = o.z0;
      if (j % 64 == 63 || j + 1 == m.size()) {
        const size_t base = j - j % 64;
        k_set_vals<<<1, 64, 0, s>>>(bp.z0s[g] + base, z0v, (int)(j - base + 1));
        EX_LAUNCHED("z0 table");
      }
    }
    FistaGroup &G = bp.groups[g];
    G.op = &bp.packed[g];
    G.opts = opts;
    G.f = f;
    G.refine = refine;
    G.L.status = bp.status;
    EX_TRY(G.prologue(s));
  }
  uint64_t key = 0x84222325cbf29ce4ull;
  key = fnv(key, &nprob, sizeof(nprob));
  key = fnv(key, ops, sizeof(expenc_op) * (size_t)nprob);
  key = fnv(key, &batch, sizeof(batch));
  key = fnv(key, &ws, sizeof(ws));
  key = fnv(key, &ws_bytes, sizeof(ws_bytes));
  key = fnv(key, opts, sizeof(*opts));
  const uint64_t gen = tuning_generation();
  key = fnv(key, &gen, sizeof(gen));
  if (opts->n_iter > 0) {
    std::vector<hipStream_t> fs;
    std::vector<hipEvent_t> ev;
    std::unique_lock<std::mutex> pool_hold;
    if (NG > 1) {
      int dev = 0;
      EX_HIP(hipGetDevice(&dev));
      EX_TRY(fork_resources(dev, NG, &fs, &ev, &pool_hold));
    }
    // Group g's work fn(g, stream) on a stream forked from cs, joined back.
    auto forked = [&](hipStream_t cs, auto &&fn) -> int {
      if (NG == 1) return fn(0, cs);
      int rc = EXPENC_OK;
      if (hipEventRecord(ev[NG], cs) != hipSuccess) return fail(EXPENC_EHIP, "fork record");
      for (int g = 0; g < NG && rc == EXPENC_OK; ++g) {
        hipStream_t gs = fs[g % fs.size()];
        if (hipStreamWaitEvent(gs, ev[NG], 0) != hipSuccess) {
          rc = fail(EXPENC_EHIP, "fork");
          break;
        }
        rc = fn(g, gs);
        // always join a forked stream back, also after an error, so that a
        // capture can end cleanly
        if (hipEventRecord(ev[g], gs) != hipSuccess || hipStreamWaitEvent(cs, ev[g], 0) != hipSuccess)
          rc = rc ? rc : fail(EXPENC_EHIP, "join");
      }
      return rc;
    };
    std::vector<const EncPlan *> plans(NG);
    std::vector<const EncBuffers *> bufs(NG);
    for (int g = 0; g < NG; ++g) {
      plans[g] = &bp.groups[g].L.p;
      bufs[g] = &bp.groups[g].L.eb;
    }
    EX_TRY(run_graph(key, s, [&](hipStream_t cs) -> int {
      if (!grouped) return forked(cs, [&](int g, hipStream_t gs) { return bp.groups[g].body(gs); });
      // lock-step groups: each iteration's two split contractions run as one
      // launch over every group's tiles
      constexpr int kAll = FistaGroup::kStageAll;
      for (int k = 0; k < opts->n_iter; ++k) {
        if (!bp.groups[0].split_difference(k)) {
          EX_TRY(forked(cs, [&](int g, hipStream_t gs) { return bp.groups[g].iteration(gs, k, kAll); }));
          continue;
        }
        EX_TRY(forked(cs, [&](int g, hipStream_t gs) {
          return bp.groups[g].iteration(gs, k, FistaGroup::kStagePre);
        }));
        EX_TRY(split_forward_grouped(plans.data(), bufs.data(), NG, cs));
        EX_TRY(forked(cs, [&](int g, hipStream_t gs) {
          return bp.groups[g].iteration(gs, k, FistaGroup::kStageMid);
        }));
        EX_TRY(split_adjoint_grouped(plans.data(), bufs.data(), NG, cs));
        EX_TRY(forked(cs, [&](int g, hipStream_t gs) {
          return bp.groups[g].iteration(gs, k, FistaGroup::kStagePost);
        }));
      }
      return EXPENC_OK;
    }));
  }
  for (int g = 0; g < NG; ++g) {
    const FistaGroup &G = bp.groups[g];
    const int K = opts->n_iter;
    const float2 *xK = (K == 0) ? G.L.x0 : ((K - 1) % 2 == 0 ? G.L.x1 : G.L.x0);
    const int64_t img = (int64_t)G.L.nxp * G.L.nyp;
    for (size_t j = 0; j < bp.members[g].size(); ++j) {
      k_crop<<<(unsigned)ceil_div((int64_t)G.L.p.R * batch, 256), 256, 0, s>>>(
          xK + j * batch * img, G.L.nxp, G.L.nyp, G.L.p.nx, G.L.p.ny, batch,
          reinterpret_cast<float2 *>(x[bp.members[g][j]]));
      EX_LAUNCHED("crop");
    }
  }
  return EXPENC_OK;
}
