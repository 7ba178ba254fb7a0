// Coil pre-whitening and coil compression (Methods 2.2.1: k-space data
// compressed to virtual coils for speed, receiver noise correlation removed
// by pre-whitening).
//
// Pre-whitening: Psi = L L^H (Cholesky, FP64, one workgroup), then every
// coil vector (one per sample of y, one per pixel of the maps) is replaced by
// L^{-1} v by forward substitution.
//
// Compression: the coil Gram matrix G = Y^H Y over all samples (FP64 partial
// sums per block of samples, summed in a fixed order), its eigenvectors by a
// cyclic Jacobi method in one workgroup (complex Hermitian rotations, the
// pairs of a sweep scheduled round-robin so that C/2 disjoint rotations run
// at once, everything in LDS), sorted by eigenvalue descending; then
// y_v = Y V_k and the virtual maps S_v[j] = sum_c V[c][j] S_c.
#include <cmath>

#include "internal.h"

namespace expenc {

namespace {

constexpr int kMaxCoils = 64;
constexpr int kGramChunk = 128;  // samples per Gram partial

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// part[blk][a][b] = sum over the block's samples of conj(y[t][a]) y[t][b]
__global__ __launch_bounds__(256) void k_gram_part(const float2 *__restrict__ y, int64_t T, int C,
                                                   double2 *__restrict__ part) {
  extern __shared__ float2 ys[];  // [kGramChunk][C]
  const int64_t t0 = (int64_t)blockIdx.x * kGramChunk;
  const int nt = (int)min<int64_t>(kGramChunk, T - t0);
  for (int i = threadIdx.x; i < nt * C; i += blockDim.x) ys[i] = y[t0 * C + i];
  __syncthreads();
  for (int o = threadIdx.x; o < C * C; o += blockDim.x) {
    const int a = o / C, b = o % C;
    double sr = 0.0, si = 0.0;
    for (int t = 0; t < nt; ++t) {
      const float2 u = ys[t * C + a], v = ys[t * C + b];
      sr += (double)u.x * v.x + (double)u.y * v.y;
      si += (double)u.x * v.y - (double)u.y * v.x;
    }
    part[(int64_t)blockIdx.x * C * C + o] = make_double2(sr, si);
  }
}

__global__ void k_gram_sum(const double2 *__restrict__ part, int nblk, int C, double2 *__restrict__ g) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= C * C) return;
  double sr = 0.0, si = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double2 v = part[(int64_t)b * C * C + o];
    sr += v.x;
    si += v.y;
  }
  g[o] = make_double2(sr, si);
}

// Eigen-decomposition of the Hermitian C x C matrix g: eigenvalues
// descending to w, eigenvectors as the columns of v ([C][C] row-major).
__global__ __launch_bounds__(256) void k_jacobi(const double2 *__restrict__ g, int C, int max_sweeps,
                                                double2 *__restrict__ v_out, double *__restrict__ w_out,
                                                unsigned *status) {
  extern __shared__ double2 sh[];
  double2 *A = sh;          // [C][C]
  double2 *V = sh + C * C;  // [C][C]
  __shared__ double rc[kMaxCoils / 2], rs[kMaxCoils / 2];
  __shared__ double2 rph[kMaxCoils / 2];
  __shared__ int rp[kMaxCoils / 2], rq[kMaxCoils / 2];
  __shared__ double red[256];
  __shared__ int perm[kMaxCoils];
  __shared__ int done;
  const int tid = threadIdx.x;
  for (int i = tid; i < C * C; i += blockDim.x) {
    A[i] = g[i];
    V[i] = make_double2((i / C) == (i % C) ? 1.0 : 0.0, 0.0);
  }
  const int n = C + (C & 1);  // players of the round-robin schedule (one dummy when C is odd)
  const int np = n / 2;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence test on the off-diagonal mass
    double off = 0.0, tot = 0.0;
    for (int i = tid; i < C * C; i += blockDim.x) {
      const double m = A[i].x * A[i].x + A[i].y * A[i].y;
      tot += m;
      if (i / C != i % C) off += m;
    }
    red[tid] = off;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) done = !(offs > 1e-30 * red[0]);
    __syncthreads();
    if (done) break;
    for (int r = 0; r < n - 1; ++r) {
      if (tid < np) {
        int p, q;
        if (tid == 0) {
          p = r;
          q = n - 1;
        } else {
          p = (r + tid) % (n - 1);
          q = (r - tid + (n - 1)) % (n - 1);
        }
        if (p > q) {
          const int tt = p;
          p = q;
          q = tt;
        }
        double c = 1.0, s = 0.0;
        double2 ph = make_double2(1.0, 0.0);
        if (q < C) {
          const double2 gpq = A[p * C + q];
          const double m = sqrt(gpq.x * gpq.x + gpq.y * gpq.y);
          const double a = A[p * C + p].x, b = A[q * C + q].x;
          if (m > 1e-300 && m > 1e-18 * (fabs(a) + fabs(b))) {
            // real Jacobi rotation of [[a, m], [m, b]]; the phase of g_pq is
            // removed by diag(1, e^{-i phi}) on index q
            const double th = (b - a) / (2.0 * m);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
            ph = make_double2(gpq.x / m, gpq.y / m);
          }
        }
        rp[tid] = p;
        rq[tid] = q;
        rc[tid] = c;
        rs[tid] = s;
        rph[tid] = ph;
      }
      __syncthreads();
      // rows:  A <- U^H A  (rows p, q of every pair)
      for (int idx = tid; idx < np * C; idx += blockDim.x) {
        const int k = idx / C, col = idx % C;
        const int p = rp[k], q = rq[k];
        if (q >= C || rs[k] == 0.0) continue;
        const double c = rc[k], s = rs[k];
        const double2 e = rph[k];
        const double2 ap = A[p * C + col], aq = A[q * C + col];
        const double2 eq = cmul(e, aq);
        A[p * C + col] = make_double2(c * ap.x - s * eq.x, c * ap.y - s * eq.y);
        A[q * C + col] = make_double2(s * ap.x + c * eq.x, s * ap.y + c * eq.y);
      }
      __syncthreads();
      // columns: A <- A U, and V <- V U
      for (int idx = tid; idx < np * C; idx += blockDim.x) {
        const int k = idx / C, row = idx % C;
        const int p = rp[k], q = rq[k];
        if (q >= C || rs[k] == 0.0) continue;
        const double c = rc[k], s = rs[k];
        const double2 ec = cconj(rph[k]);
        {
          const double2 ap = A[row * C + p], aq = A[row * C + q];
          const double2 eq = cmul(ec, aq);
          A[row * C + p] = make_double2(c * ap.x - s * eq.x, c * ap.y - s * eq.y);
          A[row * C + q] = make_double2(s * ap.x + c * eq.x, s * ap.y + c * eq.y);
        }
        {
          const double2 vp = V[row * C + p], vq = V[row * C + q];
          const double2 eq = cmul(ec, vq);
          V[row * C + p] = make_double2(c * vp.x - s * eq.x, c * vp.y - s * eq.y);
          V[row * C + q] = make_double2(s * vp.x + c * eq.x, s * vp.y + c * eq.y);
        }
      }
      __syncthreads();
    }
  }
  // eigenvalues descending (ties keep index order); status: any non-finite
  if (tid == 0) {
    unsigned bad = 0u;
    for (int i = 0; i < C; ++i)
      if (!isfinite(A[i * C + i].x)) bad = kStatusNonFinite;
    status[0] = bad;
    for (int i = 0; i < C; ++i) perm[i] = i;
    for (int i = 0; i < C; ++i) {
      int best = i;
      for (int j = i + 1; j < C; ++j)
        if (A[perm[j] * C + perm[j]].x > A[perm[best] * C + perm[best]].x) best = j;
      const int tt = perm[i];
      perm[i] = perm[best];
      perm[best] = tt;
    }
  }
  __syncthreads();
  for (int i = tid; i < C; i += blockDim.x)
    if (w_out) w_out[i] = A[perm[i] * C + perm[i]].x;
  for (int i = tid; i < C * C; i += blockDim.x) {
    const int row = i / C, col = i % C;
    v_out[i] = V[row * C + perm[col]];
  }
}

// y_out[t][j] = sum_c y[t][c] V[c][j]
__global__ void k_compress_y(const float2 *__restrict__ y, int64_t T, int C, const double2 *__restrict__ v, int nv,
                             float2 *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T * nv) return;
  const int64_t t = i / nv;
  const int j = (int)(i % nv);
  double sr = 0.0, si = 0.0;
  for (int c = 0; c < C; ++c) {
    const float2 a = y[t * C + c];
    const double2 b = v[c * C + j];
    sr += a.x * b.x - a.y * b.y;
    si += a.x * b.y + a.y * b.x;
  }
  out[i] = make_float2((float)sr, (float)si);
}

// s_out[j][r] = sum_c V[c][j] S[c][r]
__global__ void k_compress_s(const float2 *__restrict__ s, int R, int C, const double2 *__restrict__ v, int nv,
                             float2 *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nv * R) return;
  const int j = (int)(i / R);
  const int r = (int)(i % R);
  double sr = 0.0, si = 0.0;
  for (int c = 0; c < C; ++c) {
    const float2 a = s[(int64_t)c * R + r];
    const double2 b = v[c * C + j];
    sr += a.x * b.x - a.y * b.y;
    si += a.x * b.y + a.y * b.x;
  }
  out[i] = make_float2((float)sr, (float)si);
}

// L (lower, [C][C]) with L L^H = psi; NaN when psi is not positive definite
// status[0] = kStatusNonFinite when a pivot is not positive (psi not
// positive definite) or not finite, else 0.
__global__ __launch_bounds__(256) void k_cholesky(const double2 *__restrict__ psi, int C, double2 *__restrict__ L,
                                                  unsigned *status) {
  extern __shared__ double2 a[];  // [C][C]
  __shared__ double diag;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int i = tid; i < C * C; i += blockDim.x) a[i] = psi[i];
  __syncthreads();
  for (int j = 0; j < C; ++j) {
    if (tid == 0) {
      double d = a[j * C + j].x;
      for (int k = 0; k < j; ++k) d -= a[j * C + k].x * a[j * C + k].x + a[j * C + k].y * a[j * C + k].y;
      diag = sqrt(d);  // NaN for a non-positive pivot
      if (!(d > 0.0) || !isfinite(d)) bad = 1;
      a[j * C + j] = make_double2(diag, 0.0);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < C; i += blockDim.x) {
      double2 v = a[i * C + j];
      for (int k = 0; k < j; ++k) {
        const double2 t = cmul(a[i * C + k], cconj(a[j * C + k]));
        v.x -= t.x;
        v.y -= t.y;
      }
      a[i * C + j] = make_double2(v.x / diag, v.y / diag);
    }
    __syncthreads();
  }
  for (int i = tid; i < C * C; i += blockDim.x) L[i] = (i % C <= i / C) ? a[i] : make_double2(0.0, 0.0);
  if (tid == 0) status[0] = bad ? kStatusNonFinite : 0u;
}

// v <- L^{-1} v for n coil vectors v_k[c] = x[k * vstride + c * cstride]
__global__ __launch_bounds__(256) void k_whiten(const double2 *__restrict__ Lg, int C, float2 *__restrict__ x,
                                                int64_t n, int64_t vstride, int64_t cstride) {
  extern __shared__ double2 L[];  // [C][C]
  for (int i = threadIdx.x; i < C * C; i += blockDim.x) L[i] = Lg[i];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double2 w[kMaxCoils];
  for (int i = 0; i < C; ++i) {
    const float2 v = x[k * vstride + i * cstride];
    double2 s = make_double2(v.x, v.y);
    for (int m = 0; m < i; ++m) {
      const double2 t = cmul(L[i * C + m], w[m]);
      s.x -= t.x;
      s.y -= t.y;
    }
    const double d = L[i * C + i].x;
    w[i] = make_double2(s.x / d, s.y / d);
    x[k * vstride + i * cstride] = make_float2((float)w[i].x, (float)w[i].y);
  }
}

struct CoilLayout {
  unsigned *status = nullptr;  // the call's status word (start of the workspace)
  double2 *part = nullptr, *g = nullptr, *v = nullptr, *L = nullptr;
  int nblk = 0;
};

int layout_coils(int32_t C, int64_t T, Arena &a, CoilLayout *cl) {
  if (C < 1 || C > kMaxCoils) return fail(EXPENC_EINVAL, "ncoils must be in [1, %d] (got %d)", kMaxCoils, C);
  if (T < 0) return fail(EXPENC_EINVAL, "nsamples must be >= 0");
  cl->status = take_status(a);
  cl->nblk = (int)std::max<int64_t>(1, ceil_div(T, kGramChunk));
  cl->part = a.take<double2>((size_t)cl->nblk * C * C);
  cl->g = a.take<double2>((size_t)C * C);
  cl->v = a.take<double2>((size_t)C * C);
  cl->L = a.take<double2>((size_t)C * C);
  return a.ok() ? EXPENC_OK : EXPENC_EWORKSPACE;
}

}  // namespace
}  // namespace expenc

using namespace expenc;

extern "C" size_t expenc_coil_workspace_size(int32_t ncoils, int64_t nsamples) {
  Arena a;
  CoilLayout cl;
  if (layout_coils(ncoils, nsamples, a, &cl) == EXPENC_EINVAL) return 0;
  return a.used + 256;
}

extern "C" int expenc_prewhiten(int32_t ncoils, const double *psi, int64_t nsamples, float *y, int32_t npix,
                                float *smaps, void *ws, size_t ws_bytes, void *stream) {
  if (!psi) return fail(EXPENC_EINVAL, "psi is NULL");
  if ((nsamples > 0 && !y) || (npix > 0 && !smaps) || npix < 0)
    return fail(EXPENC_EINVAL, "y or smaps is NULL for a non-empty size");
  CoilLayout cl;
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  const int st = layout_coils(ncoils, 0, a, &cl);
  if (st == EXPENC_EWORKSPACE || !ws)
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                expenc_coil_workspace_size(ncoils, 0));
  EX_TRY(st);
  hipStream_t s = (hipStream_t)stream;
  const int C = ncoils;
  const size_t lds = (size_t)C * C * sizeof(double2);
  k_cholesky<<<1, 256, lds, s>>>(reinterpret_cast<const double2 *>(psi), C, cl.L, cl.status);
  EX_LAUNCHED("cholesky");
  if (nsamples > 0) {
    k_whiten<<<(unsigned)ceil_div(nsamples, 256), 256, lds, s>>>(cl.L, C, reinterpret_cast<float2 *>(y), nsamples,
                                                                  C, 1);
    EX_LAUNCHED("whiten data");
  }
  if (npix > 0) {
    k_whiten<<<(unsigned)ceil_div(npix, 256), 256, lds, s>>>(cl.L, C, reinterpret_cast<float2 *>(smaps), npix, 1,
                                                              npix);
    EX_LAUNCHED("whiten maps");
  }
  return EXPENC_OK;
}

extern "C" int expenc_coil_compress(int32_t ncoils, int32_t nvirtual, int64_t nsamples, const float *y, int32_t npix,
                                    const float *smaps, float *y_out, float *smaps_out, double *eigvec,
                                    double *eigval, void *ws, size_t ws_bytes, void *stream) {
  if (nsamples < 1 || !y) return fail(EXPENC_EINVAL, "compression needs data (nsamples >= 1, y not NULL)");
  if (nvirtual < 1 || nvirtual > ncoils) return fail(EXPENC_EINVAL, "nvirtual must be in [1, ncoils]");
  if (npix < 0 || (npix > 0 && (!smaps || !smaps_out))) return fail(EXPENC_EINVAL, "smaps or smaps_out is NULL");
  CoilLayout cl;
  Arena a{static_cast<char *>(ws), ws_bytes, 0};
  const int st = layout_coils(ncoils, nsamples, a, &cl);
  if (st == EXPENC_EWORKSPACE || !ws)
    return fail(EXPENC_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                expenc_coil_workspace_size(ncoils, nsamples));
  EX_TRY(st);
  hipStream_t s = (hipStream_t)stream;
  const int C = ncoils;
  k_gram_part<<<cl.nblk, 256, (size_t)kGramChunk * C * sizeof(float2), s>>>(reinterpret_cast<const float2 *>(y),
                                                                             nsamples, C, cl.part);
  EX_LAUNCHED("gram partials");
  k_gram_sum<<<(unsigned)ceil_div(C * C, 256), 256, 0, s>>>(cl.part, cl.nblk, C, cl.g);
  EX_LAUNCHED("gram sum");
  double2 *v = eigvec ? reinterpret_cast<double2 *>(eigvec) : cl.v;
  const size_t jlds = 2 * (size_t)C * C * sizeof(double2);
  if (jlds > 65536)
    EX_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_jacobi), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)jlds));
  k_jacobi<<<1, 256, jlds, s>>>(cl.g, C, 40, v, eigval, cl.status);
  EX_LAUNCHED("jacobi");
  if (y_out) {
    k_compress_y<<<(unsigned)ceil_div(nsamples * nvirtual, 256), 256, 0, s>>>(
        reinterpret_cast<const float2 *>(y), nsamples, C, v, nvirtual, reinterpret_cast<float2 *>(y_out));
    EX_LAUNCHED("compress data");
  }
  if (npix > 0) {
    k_compress_s<<<(unsigned)ceil_div((int64_t)nvirtual * npix, 256), 256, 0, s>>>(
        reinterpret_cast<const float2 *>(smaps), npix, C, v, nvirtual, reinterpret_cast<float2 *>(smaps_out));
    EX_LAUNCHED("compress maps");
  }
  return EXPENC_OK;
}
