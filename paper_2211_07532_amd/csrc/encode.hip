// Expanded encoding operator A_exp and its adjoint on gfx950.
//
// The entry of A_exp (eq. 1; the Introduction and Methods 2.1 list its
// ingredients: B0 map, spherical-harmonic field dynamics, coil maps, any
// trajectory) is
//     A[(t,c), r] = S_c(r) exp(i phi(t,r)),  phi = sum_l k_l(t) b_l(r) + dw0(r) t.
// Both operators are evaluated as complex GEMMs whose phase tile E = exp(i phi)
// is generated on the fly and never stored:
//   forward  Y[t, col] = sum_r E(t,r) Z[r, col],        Z[r, b*C+c] = S_c(r) x_b(r)
//   adjoint  X[r, col] = sum_t conj(E(t,r)) Y[t, col],  x_b(r) = sum_c conj(S_c(r)) X[r, b*C+c]
// Phase in turns: kap[t][.] = (k_l(t)/2pi, t), bet[r][.] = (b_l(r), dw0(r)/2pi);
// phi/2pi = sum_j kap[t][j] bet[r][j] is accumulated in FP64 (|phi| reaches
// tens of turns, and the sine needs ~1e-8 turn accuracy), reduced to [0,1)
// with v_fract_f64, and fed to the hardware v_sin/v_cos (argument in turns).
//
// FP32 form: v_mfma_f32_32x32x2_f32.  A wave owns 64 output rows (two 32-row
// MFMA blocks) and walks the reduction index two at a time.  Every lane
// evaluates two distinct phase entries (its own row, two reduction indices
// shared by the whole wave, whose basis/field values arrive through scalar
// loads); v_permlane32_swap then moves them into the A-operand layout
// (lane l holds A[l%32][l/32]).  The B operand holds 16 columns x (re, im)
// per 32-wide block: [Zr|Zi] against cos and [-Zi|Zr] against sin give
// [Yr|Yi] in one accumulator.  The reduction index is split across
// workgroups (split-K); partial sums are added in fixed order afterwards,
// so results are bitwise reproducible.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "internal.h"

namespace expenc {


static constexpr double kInv2Pi = 0.15915494309189533576888376337251436;

// ---------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------

__global__ void k_prep_kap(const double *__restrict__ coef, const double *__restrict__ time,
                           double *__restrict__ kap, int64_t T, int64_t Tp, int L, int NT) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Tp * NT) return;
  const int pz = blockIdx.y;  // problem
  if (coef) coef += pz * T * L;
  time += pz * T;
  kap += pz * Tp * NT;
  int64_t t = i / NT;
  int j = (int)(i % NT);
  double v = 0.0;
  if (t < T) {
    if (j < L) v = coef[t * L + j] * kInv2Pi;
    else if (j == L) v = time[t];
  }
  kap[i] = v;
}

__global__ void k_prep_bet(const double *__restrict__ basis, const double *__restrict__ dw0,
                           double *__restrict__ bet, int R, int Rp, int L, int NT) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Rp * NT) return;
  const int pz = blockIdx.y;
  if (basis) basis += (int64_t)pz * L * R;
  if (dw0) dw0 += (int64_t)pz * R;
  bet += (int64_t)pz * Rp * NT;
  int r = (int)(i / NT);
  int j = (int)(i % NT);
  double v = 0.0;
  if (r < R) {
    if (j < L) v = basis[(int64_t)j * R + r];
    else if (j == L && dw0) v = dw0[r] * kInv2Pi;
  }
  bet[i] = v;
}

// Z[r'][col] = S_c(r) * x_b(r), col = b*C + c, row r' = y*nxq + x of pixel
// r = y*nx + x (nxq = nx, or nx rounded up to 16 for the solid-harmonic
// kind's row-padded layout); zero for padded pixels/columns.
__global__ void k_build_z_f32(const float2 *__restrict__ smaps, const float2 *__restrict__ x,
                              int64_t x_stride, int x_row_stride, int nx, int R, int Rp, int C,
                              int NC, int NCP, float2 *__restrict__ z, int64_t x_pstride, int nxq) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Rp * NCP) return;
  const int pz = blockIdx.y;
  smaps += (int64_t)pz * C * R;
  x += pz * x_pstride;
  z += (int64_t)pz * Rp * NCP;
  const int rq = (int)(i / NCP);
  const int yy = rq / nxq, xx = rq % nxq;
  const int r = yy * nx + xx;
  int col = (int)(i % NCP);
  float2 v = make_float2(0.f, 0.f);
  if (xx < nx && r < R && col < NC) {
    int b = col / C, c = col % C;
    float2 s = smaps[(int64_t)c * R + r];
    float2 u = x[b * x_stride + (int64_t)yy * x_row_stride + xx];
    v = make_float2(s.x * u.x - s.y * u.y, s.x * u.y + s.y * u.x);
  }
  z[i] = v;
}

// Y operand [Tp][NCP] from y [B][T][C].
__global__ void k_pack_y_f32(const float2 *__restrict__ y, int64_t T, int64_t Tp, int C, int NC,
                             int NCP, float2 *__restrict__ yop, float sign) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Tp * NCP) return;
  const int pz = blockIdx.y;
  y += pz * T * NC;
  yop += pz * Tp * NCP;
  int64_t t = i / NCP;
  int col = (int)(i % NCP);
  float2 v = make_float2(0.f, 0.f);
  if (t < T && col < NC) {
    int b = col / C, c = col % C;
    v = y[((int64_t)b * T + t) * C + c];
  }
  yop[i] = make_float2(sign * v.x, sign * v.y);
}

// ---------------------------------------------------------------------------
// FP32 contraction kernels
// ---------------------------------------------------------------------------

// Forward: rows = samples, reduction over pixels.
template <int NT, int GW>
__global__ __launch_bounds__(256) void k_fwd_f32(const double *__restrict__ kap,
                                                 const double *__restrict__ bet,
                                                 const float2 *__restrict__ zop,
                                                 float *__restrict__ part, int64_t Tp, int Rp,
                                                 int NCP, int chunk, int nsplit) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int split, rb;
  if (!split_tile(blockIdx.x, (int)(Tp / 256), nsplit, &split, &rb)) return;
  const int64_t row0 = (int64_t)rb * 256 + wave * 64;
  const int g0 = blockIdx.y * GW;
  const int half = lane >> 5, c16 = lane & 15, im = (lane >> 4) & 1;
  const int pz = blockIdx.z;  // problem
  kap += pz * Tp * NT;
  bet += (int64_t)pz * Rp * NT;
  zop += (int64_t)pz * Rp * NCP;
  part += pz * nsplit * Tp * NCP * 2;

  double kv[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) kv[j] = kap[(row0 + lane) * NT + j];

  f32x16 acc[2][GW];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][g][v] = 0.f;

  const int r0 = split * chunk;
  const int r1 = min(Rp, r0 + chunk);
  const float2 *zl = zop + (int64_t)half * NCP + g0 * 16 + c16;
#pragma unroll 2
  for (int r = r0; r < r1; r += 2) {
    const double *ba = bet + (int64_t)r * NT;
    double pa = 0.0, pb = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      pa = fma(kv[j], ba[j], pa);
      pb = fma(kv[j], ba[NT + j], pb);
    }
    // centred reduction to [-1/2, 1/2] turns before rounding to FP32
    const float fa = (float)(pa - __builtin_rint(pa));
    const float fb = (float)(pb - __builtin_rint(pb));
    const float ca = __builtin_amdgcn_cosf(fa), sa = __builtin_amdgcn_sinf(fa);
    const float cb = __builtin_amdgcn_cosf(fb), sb = __builtin_amdgcn_sinf(fb);
    const auto cc = __builtin_amdgcn_permlane32_swap(__float_as_uint(ca), __float_as_uint(cb), false, false);
    const auto ss = __builtin_amdgcn_permlane32_swap(__float_as_uint(sa), __float_as_uint(sb), false, false);
    const float c_lo = __uint_as_float(cc[0]), c_hi = __uint_as_float(cc[1]);
    const float s_lo = __uint_as_float(ss[0]), s_hi = __uint_as_float(ss[1]);
#pragma unroll
    for (int g = 0; g < GW; ++g) {
      const float2 z = zl[(int64_t)r * NCP + g * 16];
      const float b1 = im ? z.y : z.x;
      const float b2 = im ? z.x : -z.y;
      acc[0][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(c_lo, b1, acc[0][g], 0, 0, 0);
      acc[1][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(c_hi, b1, acc[1][g], 0, 0, 0);
      acc[0][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(s_lo, b2, acc[0][g], 0, 0, 0);
      acc[1][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(s_hi, b2, acc[1][g], 0, 0, 0);
    }
  }

  float *dst = part + (int64_t)split * Tp * NCP * 2;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row0 + a * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        const int col = (g0 + g) * 16 + c16;
        dst[(row * NCP + col) * 2 + im] = acc[a][g][v];
      }
}

// Adjoint: rows = pixels, reduction over samples.
template <int NT, int GW>
__global__ __launch_bounds__(256) void k_adj_f32(const double *__restrict__ kap,
                                                 const double *__restrict__ bet,
                                                 const float2 *__restrict__ yop,
                                                 float *__restrict__ part, int Rp, int64_t Tp,
                                                 int NCP, int chunk, int nsplit) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int split, rb;
  if (!split_tile(blockIdx.x, Rp / 256, nsplit, &split, &rb)) return;
  const int64_t row0 = (int64_t)rb * 256 + wave * 64;
  const int g0 = blockIdx.y * GW;
  const int half = lane >> 5, c16 = lane & 15, im = (lane >> 4) & 1;
  const int pz = blockIdx.z;  // problem
  kap += pz * Tp * NT;
  bet += (int64_t)pz * Rp * NT;
  yop += pz * Tp * NCP;

  double bv[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) bv[j] = bet[(row0 + lane) * NT + j];

  f32x16 acc[2][GW];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][g][v] = 0.f;

  const int64_t t0 = (int64_t)split * chunk;
  const int64_t t1 = min(Tp, t0 + chunk);
  const float2 *yl = yop + (int64_t)half * NCP + g0 * 16 + c16;
#pragma unroll 2
  for (int64_t t = t0; t < t1; t += 2) {
    const double *ka = kap + t * NT;
    double pa = 0.0, pb = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      pa = fma(ka[j], bv[j], pa);
      pb = fma(ka[NT + j], bv[j], pb);
    }
    // centred reduction to [-1/2, 1/2] turns before rounding to FP32
    const float fa = (float)(pa - __builtin_rint(pa));
    const float fb = (float)(pb - __builtin_rint(pb));
    const float ca = __builtin_amdgcn_cosf(fa), sa = __builtin_amdgcn_sinf(fa);
    const float cb = __builtin_amdgcn_cosf(fb), sb = __builtin_amdgcn_sinf(fb);
    const auto cc = __builtin_amdgcn_permlane32_swap(__float_as_uint(ca), __float_as_uint(cb), false, false);
    const auto ss = __builtin_amdgcn_permlane32_swap(__float_as_uint(sa), __float_as_uint(sb), false, false);
    const float c_lo = __uint_as_float(cc[0]), c_hi = __uint_as_float(cc[1]);
    const float s_lo = __uint_as_float(ss[0]), s_hi = __uint_as_float(ss[1]);
#pragma unroll
    for (int g = 0; g < GW; ++g) {
      const float2 y = yl[t * NCP + g * 16];
      // conj(E) * Y = Er*[Yr|Yi] + Ei*[Yi|-Yr]
      const float b1 = im ? y.y : y.x;
      const float b2 = im ? -y.x : y.y;
      acc[0][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(c_lo, b1, acc[0][g], 0, 0, 0);
      acc[1][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(c_hi, b1, acc[1][g], 0, 0, 0);
      acc[0][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(s_lo, b2, acc[0][g], 0, 0, 0);
      acc[1][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(s_hi, b2, acc[1][g], 0, 0, 0);
    }
  }

  adj_epilogue<GW>(part, nullptr, Rp, NCP, nsplit, split, pz, blockIdx.y, gridDim.y, row0, g0, lane, acc);
}

// ---------------------------------------------------------------------------
// FP32 contractions with the solid-harmonic basis in polynomial form.  With
// z fixed, phi(t, r)/2pi = sum_m P_m(t) mono_m(x, y) + t dw0(r)/2pi, where
// mono runs over 1, x, y, x^2, xy, y^2, x^3, x^2 y, x y^2, y^3 and P_m(t) =
// pmono[t][m] (split.hip builds the table): ten FP64 terms per entry
// instead of the 17 of the general basis, still in FP64 throughout, so the
// phase keeps the general kernels' accuracy for any field strength.  Pixels
// are laid out row-padded (r' = y nxq + x, nxq = nx rounded up to 16, as in
// the split forms).  The contraction is that of k_fwd_f32 / k_adj_f32.
// ---------------------------------------------------------------------------

// Forward: rows = samples.  Along a 16-pixel tile of one image row the
// lane's phase is a cubic in the offset k = j - 8 from the tile centre
// (coefficients from the FP64 row polynomial at the centre), evaluated in
// FP64, plus t dw0(r)/2pi.
template <int GW>
__global__ __launch_bounds__(256) void k_fwd_f32_sh(const double *__restrict__ pmono, const double *__restrict__ dwq,
                                                    const float2 *__restrict__ zop, float *__restrict__ part,
                                                    int64_t Tp, int Rp, int NCP, int chunk, int nsplit, int nxq,
                                                    int nx, int ny, double dx, double dy) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int split, rb;
  if (!split_tile(blockIdx.x, (int)(Tp / 256), nsplit, &split, &rb)) return;
  const int64_t row0 = (int64_t)rb * 256 + wave * 64;
  const int g0 = blockIdx.y * GW;
  const int half = lane >> 5, c16 = lane & 15, im = (lane >> 4) & 1;
  const int pz = blockIdx.z;  // problem
  pmono += pz * Tp * 12;
  dwq += (int64_t)pz * Rp;
  zop += (int64_t)pz * Rp * NCP;
  part += pz * nsplit * Tp * NCP * 2;
  double P[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) P[m] = pmono[(row0 + lane) * 12 + m];
  const double tt = pmono[(row0 + lane) * 12 + 10];
  const double dx2 = dx * dx, dx3 = dx2 * dx;
  f32x16 acc[2][GW];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][g][v] = 0.f;
  const int r0 = split * chunk;
  const int r1 = min(Rp, r0 + chunk);
  const float2 *zl = zop + (int64_t)half * NCP + g0 * 16 + c16;
  for (int r = r0; r < r1; r += 16) {
    const int yi = r / nxq, xi = r % nxq + 8;
    const double ym = (yi - 0.5 * ny) * dy, xc = (xi - 0.5 * nx) * dx;
    const double a0 = P[0] + ym * (P[2] + ym * (P[5] + ym * P[9]));
    const double a1 = P[1] + ym * (P[4] + ym * P[8]);
    const double a2 = P[3] + ym * P[7];
    const double a3 = P[6];
    const double c0 = a0 + xc * (a1 + xc * (a2 + xc * a3));
    const double d1 = (a1 + xc * (2.0 * a2 + 3.0 * a3 * xc)) * dx;
    const double d2 = (a2 + 3.0 * a3 * xc) * dx2;
    const double d3 = a3 * dx3;
#pragma unroll
    for (int j = 0; j < 16; j += 2) {
      const double ka = j - 8, kb = j - 7;
      const double pa = fma(tt, dwq[r + j], fma(fma(fma(d3, ka, d2), ka, d1), ka, c0));
      const double pb = fma(tt, dwq[r + j + 1], fma(fma(fma(d3, kb, d2), kb, d1), kb, c0));
      // centred reduction to [-1/2, 1/2] turns before rounding to FP32
      const float fa = (float)(pa - __builtin_rint(pa));
      const float fb = (float)(pb - __builtin_rint(pb));
      const float ca = __builtin_amdgcn_cosf(fa), sa = __builtin_amdgcn_sinf(fa);
      const float cb = __builtin_amdgcn_cosf(fb), sb = __builtin_amdgcn_sinf(fb);
      const auto cc = __builtin_amdgcn_permlane32_swap(__float_as_uint(ca), __float_as_uint(cb), false, false);
      const auto ss = __builtin_amdgcn_permlane32_swap(__float_as_uint(sa), __float_as_uint(sb), false, false);
      const float c_lo = __uint_as_float(cc[0]), c_hi = __uint_as_float(cc[1]);
      const float s_lo = __uint_as_float(ss[0]), s_hi = __uint_as_float(ss[1]);
#pragma unroll
      for (int g = 0; g < GW; ++g) {
        const float2 z = zl[(int64_t)(r + j) * NCP + g * 16];
        const float b1 = im ? z.y : z.x;
        const float b2 = im ? z.x : -z.y;
        acc[0][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(c_lo, b1, acc[0][g], 0, 0, 0);
        acc[1][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(c_hi, b1, acc[1][g], 0, 0, 0);
        acc[0][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(s_lo, b2, acc[0][g], 0, 0, 0);
        acc[1][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(s_hi, b2, acc[1][g], 0, 0, 0);
      }
    }
  }
  float *dst = part + (int64_t)split * Tp * NCP * 2;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row0 + a * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        const int col = (g0 + g) * 16 + c16;
        dst[(row * NCP + col) * 2 + im] = acc[a][g][v];
      }
}

// Adjoint: rows = pixels.  The lane's pixel holds its monomials (FP64); per
// sample the ten coefficients P_m(t) and t arrive as wave-uniform scalar
// loads, and the phase is their FP64 dot product.  COMB: coils combined in
// the epilogue (sq), else per-coil partial sums (its register use, not the
// loop's, would set the occupancy of the other variant).
template <int GW, bool COMB>
__global__ __launch_bounds__(256) void k_adj_f32_sh(const double *__restrict__ pmono, const double *__restrict__ dwq,
                                                    const float2 *__restrict__ yop, float *__restrict__ part, int Rp,
                                                    int64_t Tp, int NCP, int chunk, int nsplit, int nxq, int nx,
                                                    int ny, double dx, double dy, const float2 *__restrict__ sq) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int split, rb;
  if (!(COMB ? split_tile_rows(blockIdx.x, Rp / 256, nsplit, &split, &rb) : split_tile(blockIdx.x, Rp / 256, nsplit, &split, &rb))) return;
  const int64_t row0 = (int64_t)rb * 256 + wave * 64;
  const int g0 = blockIdx.y * GW;
  const int half = lane >> 5, c16 = lane & 15, im = (lane >> 4) & 1;
  const int pz = blockIdx.z;  // problem
  pmono += pz * Tp * 12;
  dwq += (int64_t)pz * Rp;
  yop += pz * Tp * NCP;
  const int rq = (int)(row0 + lane);
  const double x = (rq % nxq - 0.5 * nx) * dx, y = (rq / nxq - 0.5 * ny) * dy;
  const double x2 = x * x, y2 = y * y;
  // monomials 1..9 in the order of pmono (x, y, x^2, xy, y^2, x^3, x^2 y, x y^2, y^3), then dw0/2pi
  const double mo[10] = {x, y, x2, x * y, y2, x2 * x, x2 * y, x * y2, y2 * y, dwq[rq]};
  f32x16 acc[2][GW];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][g][v] = 0.f;
  const int64_t t0 = (int64_t)split * chunk;
  const int64_t t1 = min(Tp, t0 + chunk);
  const float2 *yl = yop + (int64_t)half * NCP + g0 * 16 + c16;
#pragma unroll 2
  for (int64_t t = t0; t < t1; t += 2) {
    const double *ka = pmono + t * 12;
    double pa = ka[0], pb = ka[12];
#pragma unroll
    for (int m = 0; m < 10; ++m) {
      pa = fma(ka[1 + m], mo[m], pa);
      pb = fma(ka[13 + m], mo[m], pb);
    }
    // centred reduction to [-1/2, 1/2] turns before rounding to FP32
    const float fa = (float)(pa - __builtin_rint(pa));
    const float fb = (float)(pb - __builtin_rint(pb));
    const float ca = __builtin_amdgcn_cosf(fa), sa = __builtin_amdgcn_sinf(fa);
    const float cb = __builtin_amdgcn_cosf(fb), sb = __builtin_amdgcn_sinf(fb);
    const auto cc = __builtin_amdgcn_permlane32_swap(__float_as_uint(ca), __float_as_uint(cb), false, false);
    const auto ss = __builtin_amdgcn_permlane32_swap(__float_as_uint(sa), __float_as_uint(sb), false, false);
    const float c_lo = __uint_as_float(cc[0]), c_hi = __uint_as_float(cc[1]);
    const float s_lo = __uint_as_float(ss[0]), s_hi = __uint_as_float(ss[1]);
#pragma unroll
    for (int g = 0; g < GW; ++g) {
      const float2 yv = yl[t * NCP + g * 16];
      // conj(E) * Y = Er*[Yr|Yi] + Ei*[Yi|-Yr]
      const float b1 = im ? yv.y : yv.x;
      const float b2 = im ? -yv.x : yv.y;
      acc[0][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(c_lo, b1, acc[0][g], 0, 0, 0);
      acc[1][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(c_hi, b1, acc[1][g], 0, 0, 0);
      acc[0][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(s_lo, b2, acc[0][g], 0, 0, 0);
      acc[1][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(s_hi, b2, acc[1][g], 0, 0, 0);
    }
  }
  adj_epilogue<GW>(part, COMB ? sq : nullptr, Rp, NCP, nsplit, split, pz, blockIdx.y, gridDim.y, row0, g0, lane, acc);
}

// ---------------------------------------------------------------------------
// Split-K reductions (fixed summation order)
// ---------------------------------------------------------------------------

// Sum of n float2 values p[k * step], k = 0 .. n - 1, in FP64 and in k
// order, eight loads in flight per step (a loop that loads and adds one at a
// time waits for memory once per value).
__device__ inline void sum_strided(const float2 *__restrict__ p, int64_t step, int n, double &sx, double &sy) {
  int k = 0;
  for (; k + 8 <= n; k += 8) {
    float2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(k + u) * step];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sx += v[u].x;
      sy += v[u].y;
    }
  }
  for (; k < n; ++k) {
    const float2 v = p[k * step];
    sx += v.x;
    sy += v.y;
  }
}

// scl: the scaled form's operand powers of two ([P][2]), or NULL.
__global__ void k_fwd_reduce_out(const float2 *__restrict__ part, int nsplit, int64_t T,
                                 int64_t Tp, int C, int NC, int NCP, float2 *__restrict__ y,
                                 const float *__restrict__ scl) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T * NC) return;
  const int pz = blockIdx.y;
  part += pz * nsplit * Tp * NCP;
  y += pz * T * NC;
  int64_t t = i / NC;
  int col = (int)(i % NC);
  double sx = 0.0, sy = 0.0;
  sum_strided(part + t * NCP + col, Tp * NCP, nsplit, sx, sy);
  if (scl) {
    const double inv = 1.0 / scl[2 * pz];
    sx *= inv;
    sy *= inv;
  }
  int b = col / C, c = col % C;
  y[((int64_t)b * T + t) * C + c] = make_float2((float)sx, (float)sy);
}

// Residual into the adjoint operand: yop[t][col] = sum_split part - y_meas
// (y_meas may be NULL: then yop = A z).  Padded rows/columns are zero.
__global__ void k_fwd_residual(const float2 *__restrict__ part, int nsplit, int64_t T, int64_t Tp,
                               int C, int NC, int NCP, const float2 *__restrict__ y_meas,
                               float2 *__restrict__ yop) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Tp * NCP) return;
  const int pz = blockIdx.y;
  part += pz * nsplit * Tp * NCP;
  if (y_meas) y_meas += pz * T * NC;
  yop += pz * Tp * NCP;
  int64_t t = i / NCP;
  int col = (int)(i % NCP);
  double sx = 0.0, sy = 0.0;
  if (t < T && col < NC) {
    sum_strided(part + t * NCP + col, Tp * NCP, nsplit, sx, sy);
    if (y_meas) {
      const int b = col / C, c = col % C;
      const float2 m = y_meas[((int64_t)b * T + t) * C + c];
      sx -= m.x;
      sy -= m.y;
    }
  }
  yop[i] = make_float2((float)sx, (float)sy);
}

// x_b(r) = alpha * sum_c conj(S_c(r)) sum_split part[split][r][b*C+c].
// Block: 8 pixels x 32 lanes; lanes stride over coils, then a shuffle sum.
__global__ __launch_bounds__(256) void k_adj_reduce_out(const float2 *__restrict__ part, int nsplit,
                                                        int R, int Rp, int nx, int C, int B, int NCP,
                                                        const float2 *__restrict__ smaps,
                                                        float2 *__restrict__ x, int64_t x_stride,
                                                        int x_row_stride, const double *__restrict__ alpha_dev,
                                                        const float2 *__restrict__ add,
                                                        const float2 *__restrict__ base, int nxq,
                                                        int64_t x_pstride, int pad_nx, int pad_ny,
                                                        const float *__restrict__ scl) {
  const int sub = threadIdx.x & 31;
  const int q = blockIdx.x * 8 + (threadIdx.x >> 5);  // pixel of x's grid
  const int npx = pad_nx > 0 ? pad_nx * pad_ny : R;
  if (q >= npx) return;  // uniform per 32-lane group
  const int pz = blockIdx.y;  // problem
  part += (int64_t)pz * nsplit * Rp * NCP;
  smaps += (int64_t)pz * C * R;
  x += pz * x_pstride;
  if (alpha_dev) alpha_dev += pz;
  if (add) add += pz * x_pstride;
  if (base) base += pz * x_pstride;
  if (pad_nx > 0) {
    // padded grid: outside the encoded nx x ny block x = add (or 0)
    const int yy = q / pad_nx, xx = q % pad_nx;
    if (yy >= R / nx || xx >= nx) {
      if (sub == 0)
        for (int b = 0; b < B; ++b) {
          const int64_t o = b * x_stride + (int64_t)yy * x_row_stride + xx;
          x[o] = add ? add[o] : make_float2(0.f, 0.f);
        }
      return;
    }
  }
  const int r = pad_nx > 0 ? (q / pad_nx) * nx + q % pad_nx : q;
  const int64_t rq = (int64_t)(r / nx) * nxq + (r % nx);  // row of the partial sums
  for (int b = 0; b < B; ++b) {
    double sx = 0.0, sy = 0.0;
    for (int c = sub; c < C; c += 32) {
      const int col = b * C + c;
      double ux = 0.0, uy = 0.0;
      sum_strided(part + rq * NCP + col, (int64_t)Rp * NCP, nsplit, ux, uy);
      float2 s = smaps[(int64_t)c * R + r];
      sx += s.x * ux + s.y * uy;  // conj(s) * u
      sy += s.x * uy - s.y * ux;
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      sx += __shfl_xor(sx, o, 32);
      sy += __shfl_xor(sy, o, 32);
    }
    if (sub == 0) {
      if (scl) {
        const double inv = 1.0 / scl[2 * pz + 1];
        sx *= inv;
        sy *= inv;
      }
      const int yy = r / nx, xx = r % nx;
      const int64_t o = b * x_stride + (int64_t)yy * x_row_stride + xx;
      const double alpha = alpha_dev ? *alpha_dev : 1.0;
      if (base) {
        sx += base[o].x;
        sy += base[o].y;
      }
      float2 v = make_float2((float)(alpha * sx), (float)(alpha * sy));
      if (add) {
        v.x += add[o].x;
        v.y += add[o].y;
      }
      x[o] = v;
    }
  }
}

// Single image: x(r) = alpha * (sum over splits and column blocks of the
// coil-combined partial images at row (r / nx) * nxq + r % nx), with the
// same base / add terms as k_adj_reduce_out.  Four lanes per pixel: lane j
// sums slices j, j+4, j+8, ... in order (eight loads in flight), then the
// four partial sums are added in lane order.  With pad_nx > 0 the pixels are
// those of the pad_nx x pad_ny grid, and those outside the encoded block get
// add (or 0).
__global__ __launch_bounds__(256) void k_adj_reduce_comb(const float2 *__restrict__ part, int nslice, int Rp,
                                                         int nx, int ny, float2 *__restrict__ x, int x_row_stride,
                                                         const double *__restrict__ alpha_dev,
                                                         const float2 *__restrict__ add,
                                                         const float2 *__restrict__ base, int nxq, int64_t x_pstride,
                                                         int pad_nx, int pad_ny, const float *__restrict__ scl) {
  const int q = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 2), j = threadIdx.x & 3;
  const int gx = pad_nx > 0 ? pad_nx : nx;
  if (q >= (pad_nx > 0 ? pad_nx * pad_ny : nx * ny)) return;  // uniform per group of four lanes
  const int pz = blockIdx.y;  // problem
  part += (int64_t)pz * nslice * Rp;
  x += pz * x_pstride;
  if (alpha_dev) alpha_dev += pz;
  if (add) add += pz * x_pstride;
  if (base) base += pz * x_pstride;
  const int yy = q / gx, xx = q % gx;
  const int64_t o = (int64_t)yy * x_row_stride + xx;
  if (yy >= ny || xx >= nx) {
    if (j == 0) x[o] = add ? add[o] : make_float2(0.f, 0.f);
    return;
  }
  const int64_t rq = (int64_t)yy * nxq + xx;
  double sx = 0.0, sy = 0.0;
  int k0 = j;
  // steps whose eight slices exist for all four lanes: unconditional loads,
  // all in flight before the first add
  for (; k0 - j + 31 < nslice; k0 += 32) {
    float2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(k0 + 4 * u) * Rp + rq];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sx += v[u].x;
      sy += v[u].y;
    }
  }
  if (k0 < nslice) {
    float2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = k0 + 4 * u < nslice ? part[(int64_t)(k0 + 4 * u) * Rp + rq] : make_float2(0.f, 0.f);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sx += v[u].x;
      sy += v[u].y;
    }
  }
  // lane order: ((s0 + s1) + s2) + s3
  const int l0 = (threadIdx.x & 63) & ~3;
  double tx = __shfl(sx, l0), ty = __shfl(sy, l0);
#pragma unroll
  for (int u = 1; u < 4; ++u) {
    tx += __shfl(sx, l0 + u);
    ty += __shfl(sy, l0 + u);
  }
  if (j != 0) return;
  if (scl) {
    const double inv = 1.0 / scl[2 * pz + 1];
    tx *= inv;
    ty *= inv;
  }
  if (base) {
    tx += base[o].x;
    ty += base[o].y;
  }
  const double alpha = alpha_dev ? *alpha_dev : 1.0;
  float2 v = make_float2((float)(alpha * tx), (float)(alpha * ty));
  if (add) {
    v.x += add[o].x;
    v.y += add[o].y;
  }
  x[o] = v;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static int phase_terms(int L) {
  if (L + 1 <= 4) return 4;
  if (L + 1 <= 10) return 10;
  return 17;
}

static int target_workgroups() {
  static int v = [] {
    const char *e = getenv("EXPENC_TARGET_WG");
    int t = e ? atoi(e) : 0;
    return t > 0 ? t : 2048;
  }();
  return v;
}

// Workgroup targets per operator geometry, batch and precision, set by the
// autotuner through expenc_set_tuning.  Plans made after a change differ, so
// the generation counter is part of every graph-cache key.
struct TuneEntry {
  int32_t nx, ny, ncoils, nbasis, basis_kind, batch, precision;
  int64_t nsamples;
  int32_t fwd_target, adj_target, col_groups;
};
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;
static std::atomic<uint64_t> g_tune_gen{0};

uint64_t tuning_generation() { return g_tune_gen.load(); }

static bool tune_match(const TuneEntry &e, const expenc_op *op, int32_t batch, int32_t precision) {
  return e.nx == op->nx && e.ny == op->ny && e.ncoils == op->ncoils && e.nbasis == op->nbasis &&
         e.basis_kind == op->basis_kind && e.batch == batch && e.precision == precision &&
         e.nsamples == op->nsamples;
}

static void tuned_targets(const expenc_op *op, int32_t batch, int32_t precision, int *fwd, int *adj, int *gw) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const TuneEntry &e : g_tune)
    if (tune_match(e, op, batch, precision)) {
      if (e.fwd_target > 0) *fwd = e.fwd_target;
      if (e.adj_target > 0) *adj = e.adj_target;
      if (e.col_groups > 0) *gw = e.col_groups;
      return;
    }
}

int set_tuning(const expenc_op *op, int32_t batch, int32_t precision, int32_t fwd_target, int32_t adj_target,
               int32_t col_groups) {
  if (!op) return fail(EXPENC_EINVAL, "operator descriptor is NULL");
  if (fwd_target < 0 || adj_target < 0 || fwd_target > (1 << 20) || adj_target > (1 << 20))
    return fail(EXPENC_EINVAL, "workgroup targets must be in [0, 2^20]");
  if (col_groups < 0 || col_groups > 2) return fail(EXPENC_EINVAL, "col_groups must be 0, 1 or 2");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (size_t i = 0; i < g_tune.size(); ++i)
    if (tune_match(g_tune[i], op, batch, precision)) {
      g_tune.erase(g_tune.begin() + i);
      break;
    }
  if (fwd_target > 0 || adj_target > 0 || col_groups > 0)
    g_tune.push_back(TuneEntry{op->nx, op->ny, op->ncoils, op->nbasis, op->basis_kind, batch, precision,
                               op->nsamples, fwd_target, adj_target, col_groups});
  g_tune_gen.fetch_add(1);
  return EXPENC_OK;
}

int make_plan(const expenc_op *op, int32_t batch, int32_t precision, EncPlan *p, int32_t nprob) {
  if (!op) return fail(EXPENC_EINVAL, "operator descriptor is NULL");
  if (op->nx < 1 || op->ny < 1) return fail(EXPENC_EINVAL, "image grid %dx%d is empty", op->nx, op->ny);
  if ((int64_t)op->nx * op->ny > (1 << 26)) return fail(EXPENC_EINVAL, "image grid too large");
  if (op->ncoils < 1) return fail(EXPENC_EINVAL, "ncoils must be >= 1 (got %d)", op->ncoils);
  if (op->nbasis < 0 || op->nbasis > 16) return fail(EXPENC_EINVAL, "nbasis must be in [0,16] (got %d)", op->nbasis);
  if (op->nsamples < 1 || op->nsamples > (int64_t(1) << 31)) return fail(EXPENC_EINVAL, "nsamples out of range");
  if (op->basis_kind != EXPENC_BASIS_MAPS && op->basis_kind != EXPENC_BASIS_SH)
    return fail(EXPENC_EINVAL, "unknown basis_kind %d", op->basis_kind);
  if (op->reserved != 0) return fail(EXPENC_EINVAL, "reserved field must be 0");
  if (op->basis_kind == EXPENC_BASIS_SH && !(op->fov_x > 0 && op->fov_y > 0))
    return fail(EXPENC_EINVAL, "EXPENC_BASIS_SH needs fov_x, fov_y > 0");
  if (op->nbasis > 0 && !op->coef) return fail(EXPENC_EINVAL, "coef NULL with nbasis > 0");
  if (op->nbasis > 0 && op->basis_kind == EXPENC_BASIS_MAPS && !op->basis)
    return fail(EXPENC_EINVAL, "basis NULL with nbasis > 0 and EXPENC_BASIS_MAPS");
  if (!op->time) return fail(EXPENC_EINVAL, "time array is NULL");
  if (!op->smaps) return fail(EXPENC_EINVAL, "smaps is NULL");
  if (batch < 1) return fail(EXPENC_EINVAL, "batch must be >= 1 (got %d)", batch);
  if (nprob < 1 || nprob > 65535) return fail(EXPENC_EINVAL, "problem count %d out of range", nprob);
  if (precision != EXPENC_FP32 && precision != EXPENC_BF16_SPLIT && precision != EXPENC_FP16_SPLIT)
    return fail(EXPENC_EINVAL, "unknown precision %d", precision);
  if ((int64_t)op->ncoils * batch > 4096) return fail(EXPENC_EUNSUPPORTED, "ncoils*batch > 4096");
  EncPlan q;
  q.nx = op->nx;
  q.ny = op->ny;
  q.R = op->nx * op->ny;
  q.sh = op->basis_kind == EXPENC_BASIS_SH;
  q.nxq = q.sh ? (int32_t)round_up(op->nx, 16) : op->nx;
  q.dx = q.sh ? op->fov_x / op->nx : 0.0;
  q.dy = q.sh ? op->fov_y / op->ny : 0.0;
  q.z0 = q.sh ? op->z0 : 0.0;
  q.Rp = (int32_t)round_up((int64_t)q.nxq * op->ny, 256);
  q.T = op->nsamples;
  q.Tp = round_up(q.T, 256);
  q.C = op->ncoils;
  q.B = batch;
  q.NC = q.C * q.B;
  q.G = (int32_t)ceil_div(q.NC, 16);
  int tgt_fwd = target_workgroups(), tgt_adj = tgt_fwd, tuned_gw = 0;
  tuned_targets(op, batch, precision, &tgt_fwd, &tgt_adj, &tuned_gw);
  // 16-column groups per wave: two (one phase tile feeds both) unless tuned
  // to one or there is only one
  q.GW = (q.G >= 2 && tuned_gw != 1) ? 2 : 1;
  q.NGY = (int32_t)ceil_div(q.G, q.GW);
  q.comb = (batch == 1 && precision != EXPENC_FP32);
  q.NCP = q.NGY * q.GW * 16;  // every wave's column groups exist (zero-filled past NC)
  q.L = op->nbasis;
  q.NT = phase_terms(q.L);
  q.prec = precision;
  q.has_dw0 = op->dw0 != nullptr;
  q.P = nprob;
  q.scaled = precision == EXPENC_FP16_SPLIT;
  q.adj_anc = q.sh && precision != EXPENC_FP32;
  // forward: 256 sample rows per workgroup, split over pixels
  {
    int64_t nrb = q.Tp / 256 * q.P;
    int64_t want = ceil_div(tgt_fwd, nrb * q.NGY);
    want = std::max<int64_t>(1, std::min<int64_t>(want, q.Rp / 16));
    q.fwd_chunk = (int32_t)round_up(ceil_div(q.Rp, want), 16);
    if (precision == EXPENC_FP32) q.fwd_chunk = std::min(q.fwd_chunk, kF32ChunkMax);
    q.fwd_split = (int32_t)ceil_div(q.Rp, q.fwd_chunk);
    q.nwmax = (int32_t)split_grid(q.Tp / 256 * q.fwd_split) * q.NGY * 4;
  }
  // adjoint: 256 pixel rows per workgroup, split over samples
  {
    int64_t nrb = q.Rp / 256 * q.P;
    int64_t want = ceil_div(tgt_adj, nrb * q.NGY);
    want = std::max<int64_t>(1, std::min<int64_t>(want, q.Tp / 16));
    // (the polynomial split adjoint steps over 32 samples at a time)
    q.adj_chunk = (int32_t)round_up(ceil_div(q.Tp, want), (q.sh && precision != EXPENC_FP32) ? 32 : 16);
    // The error of a contraction grows with the length of the sums one
    // workgroup accumulates on the matrix cores.  Measured on a 200 px,
    // T = 20000 fp16 solve: NRMSE 1.8e-5 at 562 samples per split adjoint
    // chunk, 2.9e-5 at 5056, 5.0e-5 at 10112 (the split forward's chunk
    // length did not matter); with 12 problems per launch the FP32 anchors'
    // chunks (3 forward, 2 adjoint splits) alone took it from 2.2e-5 to
    // 4.9e-5.  So chunks are capped (the tuned single-problem shapes are
    // below the caps).
    q.adj_chunk = std::min(q.adj_chunk, precision == EXPENC_FP32 ? kF32ChunkMax : kSplitAdjChunkMax);
    q.adj_split = (int32_t)ceil_div(q.Tp, q.adj_chunk);
  }
  *p = q;
  return EXPENC_OK;
}

size_t enc_operand_bytes(const EncPlan &p) {
  Arena a;
  EncBuffers b;
  carve_enc(p, a, &b);
  return a.used + 256;
}

int plan_forward_within(const expenc_op *op, int32_t batch, int32_t precision, size_t cap, EncPlan *p) {
  EncPlan q;
  EX_TRY(make_plan(op, batch, precision, &q));
  // the forward uses no adjoint partial sums: one adjoint split keeps them small
  q.adj_split = 1;
  q.adj_anc = false;
  q.adj_chunk = (int32_t)q.Tp;
  const int32_t min_split = q.prec == EXPENC_FP32 ? (int32_t)ceil_div(q.Rp, kF32ChunkMax) : 1;
  auto set_split = [&](int32_t want) {
    q.fwd_chunk = (int32_t)round_up(ceil_div(q.Rp, want), 16);
    if (q.prec == EXPENC_FP32) q.fwd_chunk = std::min(q.fwd_chunk, kF32ChunkMax);
    q.fwd_split = (int32_t)ceil_div(q.Rp, q.fwd_chunk);
    q.nwmax = (int32_t)split_grid(q.Tp / 256 * q.fwd_split) * q.NGY * 4;
  };
  while (enc_operand_bytes(q) > cap && q.fwd_split > min_split)
    set_split(std::max<int32_t>(min_split, q.fwd_split - std::max<int32_t>(1, q.fwd_split / 4)));
  if (enc_operand_bytes(q) > cap)
    return fail(EXPENC_EWORKSPACE, "the forward of this operator needs %zu bytes of scratch, more than the %zu "
                "of the static scratch (use expenc_forward with a workspace)", enc_operand_bytes(q), cap);
  *p = q;
  return EXPENC_OK;
}

size_t enc_part_elems(const EncPlan &p) {
  const size_t pf = (size_t)p.fwd_split * p.Tp * p.NCP;
  const size_t pa = (size_t)p.adj_split * p.Rp * (p.comb ? p.NGY : p.NCP);
  return std::max(pf, pa) * p.P;
}

int carve_enc(const EncPlan &p, Arena &a, EncBuffers *b, size_t min_part) {
  const size_t P = p.P;
  b->kap = a.take<double>(P * p.Tp * p.NT);
  b->bet = a.take<double>(P * p.Rp * p.NT);
  b->zop = a.take<float2>(P * p.Rp * p.NCP);
  b->yop = a.take<float2>(P * p.Tp * p.NCP);
  b->part = a.take<float2>(std::max(enc_part_elems(p), min_part));
  if (p.sh) {
    // polynomial phase tables (every precision; dpa: the split adjoint's
    // increment operand)
    b->pmono = a.take<double>(P * p.Tp * 12);
    b->dpa = a.take<float>(P * p.Tp * 16);
    b->dwq = a.take<double>(P * p.Rp);
    b->ddw = a.take<float>(P * p.Rp);
    if (p.adj_anc) b->anc = a.take<float>(P * (p.Tp / 32) * p.Rp);
  }
  if (p.prec != EXPENC_FP32) {
    b->zs = a.take<char>(P * p.Rp * (p.NCP / 16) * 256);
    b->ys = a.take<char>(P * p.Tp * (p.NCP / 16) * 256);
    if (p.comb) b->sq = a.take<float2>(P * p.Rp * p.NCP);
    if (p.scaled) {
      b->scl = a.take<float>(P * 2);
      b->amax = a.take<float>(P * 3 * kAmaxBlocks);
      b->wmax = a.take<float>(P * p.nwmax);
    }
    if (!p.sh) {
      b->dbet = a.take<float>(P * p.Rp * p.NT);
      b->dkap = a.take<float>(P * p.Tp * p.NT);
    }
  }
  return a.ok() ? EXPENC_OK : EXPENC_EWORKSPACE;
}

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)ceil_div(n, bs); }
static inline dim3 grid_p(int64_t n, int bs, int P) { return dim3((unsigned)ceil_div(n, bs), (unsigned)P); }

int enc_prepare(const EncPlan &p, const expenc_op *op, const EncBuffers &b, hipStream_t s) {
  k_prep_kap<<<grid_p(p.Tp * p.NT, 256, p.P), 256, 0, s>>>(op->coef, op->time, b.kap, p.T, p.Tp, p.L, p.NT);
  EX_LAUNCHED("prep_kap");
  const bool split = p.prec != EXPENC_FP32;
  if (!p.sh) {  // the polynomial (solid-harmonic) kernels do not read bet
    k_prep_bet<<<grid_p((int64_t)p.Rp * p.NT, 256, p.P), 256, 0, s>>>(op->basis, op->dw0, b.bet, p.R, p.Rp, p.L,
                                                                       p.NT);
    EX_LAUNCHED("prep_bet");
  }
  if (split) return split_prepare(p, op, b, s);
  if (p.sh) return sh_prepare(p, op, b, s);
  return EXPENC_OK;
}

int enc_build_z(const EncPlan &p, const float *smaps, const float2 *x, int64_t x_stride,
                int32_t x_row_stride, const EncBuffers &b, hipStream_t s, const float2 *xsub, int64_t x_pstride) {
  if (p.prec != EXPENC_FP32) return split_build_z(p, smaps, x, xsub, x_stride, x_row_stride, b, s, x_pstride);
  if (xsub) return fail(EXPENC_EUNSUPPORTED, "operand difference is only built for split forms");
  k_build_z_f32<<<grid_p((int64_t)p.Rp * p.NCP, 256, p.P), 256, 0, s>>>(
      reinterpret_cast<const float2 *>(smaps), x, x_stride, x_row_stride, p.nx, p.R, p.Rp, p.C, p.NC,
      p.NCP, b.zop, x_pstride, p.nxq);
  EX_LAUNCHED("build_z");
  return EXPENC_OK;
}

int enc_pack_y(const EncPlan &p, const float2 *y, const EncBuffers &b, hipStream_t s, float sign) {
  if (p.prec != EXPENC_FP32) {
    if (sign != 1.f) return fail(EXPENC_EUNSUPPORTED, "scaled operand packing is FP32 only");
    return split_pack_y(p, y, false, nullptr, b, s);
  }
  k_pack_y_f32<<<grid_p(p.Tp * p.NCP, 256, p.P), 256, 0, s>>>(y, p.T, p.Tp, p.C, p.NC, p.NCP, b.yop, sign);
  EX_LAUNCHED("pack_y");
  return EXPENC_OK;
}

// ---------------------------------------------------------------------------
// Opt-in per-kernel timing of the two contraction kernels with HIP events
// recorded on the launch stream (eager launches only; skipped while the
// stream is being captured into a graph).
// ---------------------------------------------------------------------------
namespace {
struct KernelTimer {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[2];
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
  }
  void clear() {
    for (auto &v : ev)
      for (auto &pr : v) {
        pool.push_back(pr.first);
        pool.push_back(pr.second);
      }
    ev[0].clear();
    ev[1].clear();
  }
};
KernelTimer g_timer;

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return true;
  return st != hipStreamCaptureStatusNone;
}

template <class F>
void timed(int kind, hipStream_t s, F launch) {
  hipEvent_t a = nullptr, b = nullptr;
  bool t = false;
  {
    std::lock_guard<std::mutex> lk(g_timer.mu);
    t = g_timer.on && !capturing(s);
    if (t) {
      a = g_timer.get();
      b = g_timer.get();
    }
  }
  if (t) hipEventRecord(a, s);
  launch();
  if (t) {
    hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_timer.mu);
    g_timer.ev[kind].push_back({a, b});
  }
}
}  // namespace

int kernel_timing(int32_t mode, double *out) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  if (mode == 0 || mode == 1) {
    g_timer.clear();
    g_timer.on = (mode == 1);
    return EXPENC_OK;
  }
  if (mode != 2 || !out) return fail(EXPENC_EINVAL, "bad timing mode");
  for (int k = 0; k < 2; ++k) {
    double tot = 0;
    for (auto &pr : g_timer.ev[k]) {
      EX_HIP(hipEventSynchronize(pr.second));
      float ms = 0;
      EX_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
      tot += ms;
    }
    out[2 * k] = tot;
    out[2 * k + 1] = (double)g_timer.ev[k].size();
  }
  return EXPENC_OK;
}

template <int NT>
static void launch_fwd(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid(p.Tp / 256 * p.fwd_split), (unsigned)p.NGY, (unsigned)p.P);
  float *part = reinterpret_cast<float *>(b.part);
  if (p.GW == 2)
    k_fwd_f32<NT, 2><<<grid, 256, 0, s>>>(b.kap, b.bet, b.zop, part, p.Tp, p.Rp, p.NCP, p.fwd_chunk, p.fwd_split);
  else
    k_fwd_f32<NT, 1><<<grid, 256, 0, s>>>(b.kap, b.bet, b.zop, part, p.Tp, p.Rp, p.NCP, p.fwd_chunk, p.fwd_split);
}

template <int NT>
static void launch_adj(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid((int64_t)p.Rp / 256 * p.adj_split), (unsigned)p.NGY, (unsigned)p.P);
  float *part = reinterpret_cast<float *>(b.part);
  if (p.GW == 2)
    k_adj_f32<NT, 2><<<grid, 256, 0, s>>>(b.kap, b.bet, b.yop, part, p.Rp, p.Tp, p.NCP, p.adj_chunk, p.adj_split);
  else
    k_adj_f32<NT, 1><<<grid, 256, 0, s>>>(b.kap, b.bet, b.yop, part, p.Rp, p.Tp, p.NCP, p.adj_chunk, p.adj_split);
}

static void launch_fwd_sh(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid(p.Tp / 256 * p.fwd_split), (unsigned)p.NGY, (unsigned)p.P);
  float *part = reinterpret_cast<float *>(b.part);
  if (p.GW == 2)
    k_fwd_f32_sh<2><<<grid, 256, 0, s>>>(b.pmono, b.dwq, b.zop, part, p.Tp, p.Rp, p.NCP, p.fwd_chunk, p.fwd_split,
                                         p.nxq, p.nx, p.ny, p.dx, p.dy);
  else
    k_fwd_f32_sh<1><<<grid, 256, 0, s>>>(b.pmono, b.dwq, b.zop, part, p.Tp, p.Rp, p.NCP, p.fwd_chunk, p.fwd_split,
                                         p.nxq, p.nx, p.ny, p.dx, p.dy);
}

static void launch_adj_sh(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid((int64_t)p.Rp / 256 * p.adj_split), (unsigned)p.NGY, (unsigned)p.P);
  float *part = reinterpret_cast<float *>(b.part);
  auto go = [&](auto gw, auto comb) {
    k_adj_f32_sh<decltype(gw)::value, decltype(comb)::value><<<grid, 256, 0, s>>>(
        b.pmono, b.dwq, b.yop, part, p.Rp, p.Tp, p.NCP, p.adj_chunk, p.adj_split, p.nxq, p.nx, p.ny, p.dx, p.dy,
        b.sq);
  };
  using T1 = std::integral_constant<int, 1>;
  using T2 = std::integral_constant<int, 2>;
  using On = std::true_type;
  using Off = std::false_type;
  if (p.GW == 2) {
    if (p.comb) go(T2{}, On{});
    else go(T2{}, Off{});
  } else {
    if (p.comb) go(T1{}, On{});
    else go(T1{}, Off{});
  }
}

int enc_forward_partials(const EncPlan &p, const EncBuffers &b, hipStream_t s, bool timing) {
  auto launch = [&] {
    if (p.prec != EXPENC_FP32) {
      split_forward_launch(p, b, s);
      return;
    }
    if (p.sh) {
      launch_fwd_sh(p, b, s);
      return;
    }
    switch (p.NT) {
      case 4: launch_fwd<4>(p, b, s); break;
      case 10: launch_fwd<10>(p, b, s); break;
      default: launch_fwd<17>(p, b, s); break;
    }
  };
  if (timing) timed(0, s, launch);
  else launch();
  EX_LAUNCHED("forward contraction");
  return EXPENC_OK;
}

int enc_adjoint_partials(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  if (p.comb && !b.sq) return fail(EXPENC_EINVAL, "coil table of a single-image split plan is not carved");
  if (p.adj_anc && !b.anc) return fail(EXPENC_EINVAL, "anchor table of a split plan is not carved");
  if (p.sh && p.prec != EXPENC_FP32 && !p.adj_anc) return fail(EXPENC_EINVAL, "forward-only plan");
  timed(1, s, [&] {
    if (p.prec != EXPENC_FP32) {
      split_adjoint_launch(p, b, s);
      return;
    }
    if (p.sh) {
      launch_adj_sh(p, b, s);
      return;
    }
    switch (p.NT) {
      case 4: launch_adj<4>(p, b, s); break;
      case 10: launch_adj<10>(p, b, s); break;
      default: launch_adj<17>(p, b, s); break;
    }
  });
  EX_LAUNCHED("adjoint contraction");
  return EXPENC_OK;
}

int enc_forward_reduce_out(const EncPlan &p, const EncBuffers &b, float2 *y, hipStream_t s) {
  k_fwd_reduce_out<<<grid_p(p.T * p.NC, 256, p.P), 256, 0, s>>>(b.part, p.fwd_split, p.T, p.Tp, p.C, p.NC, p.NCP, y,
                                                                  p.scaled ? b.scl : nullptr);
  EX_LAUNCHED("forward reduce");
  return EXPENC_OK;
}

int enc_forward_residual(const EncPlan &p, const EncBuffers &b, const float2 *y_meas, hipStream_t s) {
  if (p.prec != EXPENC_FP32) return split_pack_y(p, nullptr, true, y_meas, b, s);
  k_fwd_residual<<<grid_p(p.Tp * p.NCP, 256, p.P), 256, 0, s>>>(b.part, p.fwd_split, p.T, p.Tp, p.C, p.NC,
                                                                  p.NCP, y_meas, b.yop);
  EX_LAUNCHED("forward residual");
  return EXPENC_OK;
}

int enc_adjoint_reduce_out(const EncPlan &p, const EncBuffers &b, const float *smaps, float2 *x,
                           int64_t x_stride, int32_t x_row_stride, const double *alpha_dev,
                           const float2 *add, hipStream_t s, const float2 *base, int64_t x_pstride,
                           int32_t pad_nx, int32_t pad_ny) {
  const int64_t npx = pad_nx > 0 ? (int64_t)pad_nx * pad_ny : p.R;
  if (pad_nx > 0 && (pad_nx < p.nx || pad_ny < p.ny || x_row_stride < pad_nx))
    return fail(EXPENC_EINVAL, "padded grid %dx%d smaller than the image", pad_nx, pad_ny);
  if (p.comb) {
    k_adj_reduce_comb<<<grid_p(npx * 4, 256, p.P), 256, 0, s>>>(b.part, p.adj_split * p.NGY, p.Rp, p.nx, p.ny, x,
                                                          x_row_stride, alpha_dev, add, base, p.nxq, x_pstride,
                                                          pad_nx, pad_ny, p.scaled ? b.scl : nullptr);
    EX_LAUNCHED("adjoint reduce");
    return EXPENC_OK;
  }
  k_adj_reduce_out<<<grid_p(npx, 8, p.P), 256, 0, s>>>(b.part, p.adj_split, p.R, p.Rp, p.nx, p.C, p.B, p.NCP,
                                                       reinterpret_cast<const float2 *>(smaps), x, x_stride,
                                                       x_row_stride, alpha_dev, add, base, p.nxq, x_pstride,
                                                       pad_nx, pad_ny, p.scaled ? b.scl : nullptr);
  EX_LAUNCHED("adjoint reduce");
  return EXPENC_OK;
}

}  // namespace expenc
