// Split-precision (bf16 or fp16 hi+lo) forms of the encoding contractions.
//
// Every operand value v (FP32) is written as hi + lo with hi = rnd(v) and
// lo = rnd(v - hi) in the 16-bit format; a product a*b is taken as
// a_hi*b_hi + a_hi*b_lo + a_lo*b_hi on v_mfma_f32_32x32x16_{bf16,f16} with FP32
// accumulation (the lo*lo term, ~2^-2p relative, is dropped).  This runs the
// contraction at the 16-bit MFMA rate with an error of about 3*2^-16 per
// product (bf16) or 3*2^-22 (fp16) instead of 2^-8 / 2^-11 for a plain
// 16-bit product.
//
// Layout of one MFMA step (K = 16 reduction indices): lane l holds 8
// consecutive reduction indices 8*(l/32) .. 8*(l/32)+7 of row l%32 for the A
// operand and of column l%32 for the B operand.  As in the FP32 kernels, each
// lane first evaluates the phase tile for ITS OWN row against all 16
// reduction indices (which are wave-uniform, so their field/basis values
// come through scalar loads), splits and packs pairs into 32-bit words, and
// v_permlane32_swap exchanges the half-waves so that the two 32-row MFMA
// blocks receive their operands.  The B operand is pre-split and packed in
// exactly the per-lane order (four 16-byte records per lane and step: b1 hi,
// b1 lo, b2 hi, b2 lo), so the inner loop loads it with dwordx4 loads.
#include "internal.h"
#include "split_dev.h"

namespace expenc {

__device__ inline uint32_t swap_lo(uint32_t a, uint32_t b, uint32_t &hi_out) {
  const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  hi_out = r[1];
  return r[0];
}

// Split the 16 (cos, sin) values of one lane into hi/lo 16-bit pairs, pack
// them into 32-bit words and exchange half-waves so that
//   A[blk][kind] (blk 0: rows 0..31, 1: rows 32..63; kind 0 c_hi, 1 c_lo, 2 s_hi, 3 s_lo)
// are the A operands of this step.
template <bool BF>
__device__ inline void pack_tile16(const float (&c)[16], const float (&sn)[16], u32x4 (&A)[2][4]) {
  uint32_t w[4][2][4];  // [kind][half of the 16 indices][word]
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int hf = m >> 2, wd = m & 3;
    split_pair<BF>(c[2 * m], c[2 * m + 1], w[0][hf][wd], w[1][hf][wd]);
    split_pair<BF>(sn[2 * m], sn[2 * m + 1], w[2][hf][wd], w[3][hf][wd]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t hi0, hi1, hi2, hi3;
    const uint32_t lo0 = swap_lo(w[k][0][0], w[k][1][0], hi0);
    const uint32_t lo1 = swap_lo(w[k][0][1], w[k][1][1], hi1);
    const uint32_t lo2 = swap_lo(w[k][0][2], w[k][1][2], hi2);
    const uint32_t lo3 = swap_lo(w[k][0][3], w[k][1][3], hi3);
    A[0][k] = u32x4{lo0, lo1, lo2, lo3};
    A[1][k] = u32x4{hi0, hi1, hi2, hi3};
  }
}

// Phase tile of one lane against 16 wave-uniform reduction indices, split,
// packed and redistributed.
//
// The phase of the tile's centre index (index 8) is accumulated in FP64 and
// reduced to [0,1) turns (anchor a).  The other 15 follow as
//   phi_j = a + sum_k pf[k] * dq[j][k]          (FP32)
// where pf is this lane's phase terms rounded to FP32 and dq[j] the
// wave-uniform differences (index j minus index 8) of the other factor,
// precomputed per tile in FP64 and rounded once.  Within a tile the
// increments stay small (a few turns for 16 pixels along a row, under one
// turn for 16 samples), so the FP32 rounding error of the increment is
// about 1e-6 turn, well inside the split forms' error budget.  The uniform
// differences (NT floats per index) are scalar-loaded one index ahead.
//
//   pv: this lane's FP64 terms; qc: the centre index's NT uniform FP64
//   terms; dq: 16 x NT uniform FP32 differences.  On return A[blk][kind]
//   (blk 0: rows 0..31, 1: rows 32..63; kind 0 c_hi, 1 c_lo, 2 s_hi, 3 s_lo)
//   are the A operands of this step.
template <int NT, bool BF>
__device__ inline void phase_tile16(const double (&pv)[NT], const float (&pf)[NT], const double *__restrict__ qc,
                                    const float *__restrict__ dq, u32x4 (&A)[2][4]) {
  double pa = 0.0;
#pragma unroll
  for (int j = 0; j < NT; ++j) pa = fma(pv[j], qc[j], pa);
  const float a = (float)__builtin_amdgcn_fract(pa);
  __builtin_amdgcn_sched_barrier(0);
  float c[16], sn[16];
  float buf[2][NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) buf[0][j] = dq[j];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i + 1 < 16) {
      // An opaque (empty) redefinition of the uniform offset: the scalar
      // loads of index i+1 cannot be merged with, or hoisted above, those of
      // earlier indices, so only two indices' terms are live at a time.
      int off = (i + 1) * NT;
      __asm__ volatile("" : "+s"(off));
#pragma unroll
      for (int j = 0; j < NT; ++j) buf[(i + 1) & 1][j] = dq[off + j];
    }
    float ph = a;
#pragma unroll
    for (int j = 0; j < NT; ++j) ph = fmaf(pf[j], buf[i & 1][j], ph);
    const float f = __builtin_amdgcn_fractf(ph);
    c[i] = __builtin_amdgcn_cosf(f);
    sn[i] = __builtin_amdgcn_sinf(f);
  }
  pack_tile16<BF>(c, sn, A);
}

// Slot of this wave in the per-problem maxima array of a forward launch
// (workgroup bx, by of a grid gx wide).
__device__ inline int wave_slot(int bx, int by, int gx) { return (by * gx + bx) * 4 + (threadIdx.x >> 6); }
__device__ inline int wave_slot() { return wave_slot(blockIdx.x, blockIdx.y, gridDim.x); }

// Writes a wave's forward partial sums; with wmax (scaled form) also the
// wave's max |value| into its slot (a bound for the residual operand), per
// wave and without a workgroup barrier.
template <int GW>
__device__ inline void store_partials(float *dst, int64_t row0, int NCP, int g0, int lane, f32x16 (&acc)[2][GW],
                                      float *wmax, int slot) {
  const int half = lane >> 5, c16 = lane & 15, im = (lane >> 4) & 1;
  float m = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row0 + a * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        const int col = (g0 + g) * 16 + c16;
        dst[(row * NCP + col) * 2 + im] = acc[a][g][v];
        m = fmaxf(m, fabsf(acc[a][g][v]));
      }
  if (wmax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if (lane == 0) wmax[slot] = m;
  }
}

// Forward, split form: rows = samples, reduction over pixels (16 per step).
template <int NT, int GW, bool BF>
__global__ __launch_bounds__(256) void k_fwd_split(const double *__restrict__ kap, const double *__restrict__ bet,
                                                   const float *__restrict__ dbet, const u32x4 *__restrict__ zs,
                                                   float *__restrict__ part, int64_t Tp, int Rp, int NCP, int chunk,
                                                   int nsplit) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int split, rb;
  if (!split_tile(blockIdx.x, (int)(Tp / 256), nsplit, &split, &rb)) return;
  const int64_t row0 = (int64_t)rb * 256 + wave * 64;
  const int g0 = blockIdx.y * GW;
  const int NGP = NCP / 16;
  const int pz = blockIdx.z;  // problem
  kap += pz * Tp * NT;
  bet += (int64_t)pz * Rp * NT;
  dbet += (int64_t)pz * Rp * NT;
  zs += (int64_t)pz * Rp * NGP * 16;
  part += pz * nsplit * Tp * NCP * 2;
  double kv[NT];
  float kf[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    kv[j] = kap[(row0 + lane) * NT + j];
    kf[j] = (float)kv[j];
  }
  f32x16 acc[2][GW];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][g][v] = 0.f;
  const int r0 = split * chunk;
  const int r1 = min(Rp, r0 + chunk);
  for (int r = r0; r < r1; r += 16) {
    u32x4 A[2][4];
    phase_tile16<NT, BF>(kv, kf, bet + (int64_t)(r + 8) * NT, dbet + (int64_t)r * NT, A);
#pragma unroll
    for (int g = 0; g < GW; ++g) {
      const u32x4 *zq = zs + ((int64_t)(r >> 4) * NGP + (g0 + g)) * 256 + lane;
      const u32x4 b[4] = {zq[0], zq[64], zq[128], zq[192]};
      acc[0][g] = step6<BF>(A[0], b, acc[0][g]);
      acc[1][g] = step6<BF>(A[1], b, acc[1][g]);
    }
  }
  store_partials<GW>(part + (int64_t)split * Tp * NCP * 2, row0, NCP, g0, lane, acc, nullptr, 0);
}

// Adjoint, split form: rows = pixels, reduction over samples (16 per step).
// The A operand is exp(+i phi); the conjugation lives in the packed B operand.
template <int NT, int GW, bool BF>
__global__ __launch_bounds__(256) void k_adj_split(const double *__restrict__ kap, const double *__restrict__ bet,
                                                   const float *__restrict__ dkap, const u32x4 *__restrict__ ys,
                                                   float *__restrict__ part, int Rp, int64_t Tp, int NCP, int chunk,
                                                   int nsplit, const float2 *__restrict__ sq) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int split, rb;
  if (!(sq ? split_tile_rows(blockIdx.x, Rp / 256, nsplit, &split, &rb) : split_tile(blockIdx.x, Rp / 256, nsplit, &split, &rb))) return;
  const int64_t row0 = (int64_t)rb * 256 + wave * 64;
  const int g0 = blockIdx.y * GW;
  const int NGP = NCP / 16;
  const int pz = blockIdx.z;  // problem
  kap += pz * Tp * NT;
  dkap += pz * Tp * NT;
  bet += (int64_t)pz * Rp * NT;
  ys += pz * Tp * NGP * 16;
  double bv[NT];
  float bf[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    bv[j] = bet[(row0 + lane) * NT + j];
    bf[j] = (float)bv[j];
  }
  f32x16 acc[2][GW];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][g][v] = 0.f;
  const int64_t t0 = (int64_t)split * chunk;
  const int64_t t1 = min(Tp, t0 + chunk);
  for (int64_t t = t0; t < t1; t += 16) {
    u32x4 A[2][4];
    phase_tile16<NT, BF>(bv, bf, kap + (t + 8) * NT, dkap + t * NT, A);
#pragma unroll
    for (int g = 0; g < GW; ++g) {
      const u32x4 *yq = ys + ((t >> 4) * NGP + (g0 + g)) * 256 + lane;
      const u32x4 b[4] = {yq[0], yq[64], yq[128], yq[192]};
      acc[0][g] = step6<BF>(A[0], b, acc[0][g]);
      acc[1][g] = step6<BF>(A[1], b, acc[1][g]);
    }
  }
  adj_epilogue<GW>(part, sq, Rp, NCP, nsplit, split, pz, blockIdx.y, gridDim.y, row0, g0, lane, acc);
}


// ---------------------------------------------------------------------------
// Split forms with the solid-harmonic basis in polynomial form.  With z
// fixed, sum_l k_l(t) b_l(x, y) is a cubic polynomial in (x, y) whose ten
// monomial coefficients P_m(t) (turns) are formed once per sample.
//
// Forward (lane = sample t, 16 pixels of one image row per step): along the
// row the phase is a cubic in x.  Each lane expands it around the tile
// centre x_c in FP64: the anchor phi(x_c) reduced to [0,1), and the scaled
// Taylor coefficients d1 = phi_x dx, d2 = phi_xx dx^2 / 2, d3 = phi_xxx dx^3 / 6.
// Pixel x_c + k dx (k = -8..7, a literal) then costs three FP32 FMAs, plus
// one for the off-resonance difference t (dw0(r) - dw0(r_c)) / 2pi.
//
// Adjoint (32 samples x 64 pixels per wave and step): the phase is the
// FP64 anchor of the tile's centre sample t_c at each pixel (a table written
// at preparation) plus the increment sum_m (P_m(t) - P_m(t_c)) mono_m(r) +
// (t - t_c) dw0(r)/2pi.  Inside one image row the increment is a cubic in x
// whose four coefficients are polynomials in the row's y, so for a block of
// 32 pixels of one row it is a rank-6 product (the cubic, dw0 and the
// anchor with a unit A entry) of a [32 samples x 6] operand, evaluated per
// block from per-sample coefficients, with a [6 x 32 pixels] operand: three
// v_mfma_f32_32x32x2_f32 per block (five for a block that continues into
// the next row), instead of eleven FP32 FMAs per entry on the vector unit.
// The product's output layout gives each lane 16 samples of ONE
// pixel, which is the A-operand layout of the contraction up to a fixed
// permutation of the samples inside each group of 16; the adjoint records
// are packed in that order, so no exchange between lanes is needed.
// ---------------------------------------------------------------------------

// Arguments of one problem group's forward launch.
struct FwdShArgs {
  const double *pmono, *dwq;
  const float *ddw;
  const u32x4 *zs;
  float *part, *wmax;
  int64_t Tp;
  int Rp, NCP, chunk, nsplit, nxq, nx, ny;
  double dx, dy;
};

// One workgroup of the forward (workgroup bx, by, bz of a gx x gy x P grid).
template <int GW, bool BF>
__device__ inline void fwd_split_sh_body(const FwdShArgs &a, int bx, int by, int bz, int gx, int gy) {
  const double *__restrict__ pmono = a.pmono;
  const double *__restrict__ dwq = a.dwq;
  const float *__restrict__ ddw = a.ddw;
  const u32x4 *__restrict__ zs = a.zs;
  float *__restrict__ part = a.part;
  float *__restrict__ wmax = a.wmax;
  const int64_t Tp = a.Tp;
  const int Rp = a.Rp, NCP = a.NCP, chunk = a.chunk, nsplit = a.nsplit, nxq = a.nxq, nx = a.nx, ny = a.ny;
  const double dx = a.dx, dy = a.dy;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int split, rb;
  if (wmax) wmax += (int64_t)bz * gy * gx * 4;
  const int slot = wave_slot(bx, by, gx);
  if (!split_tile(bx, (int)(Tp / 256), nsplit, &split, &rb)) {
    if (wmax && lane == 0) wmax[slot] = 0.f;
    return;
  }
  const int64_t row0 = (int64_t)rb * 256 + wave * 64;
  const int g0 = by * GW;
  const int NGP = NCP / 16;
  const int pz = bz;  // problem
  pmono += pz * Tp * 12;
  dwq += (int64_t)pz * Rp;
  ddw += (int64_t)pz * Rp;
  zs += (int64_t)pz * Rp * NGP * 16;
  part += pz * nsplit * Tp * NCP * 2;
  double P[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) P[m] = pmono[(row0 + lane) * 12 + m];
  const double tt = pmono[(row0 + lane) * 12 + 10];
  const float tf = (float)tt;
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
  for (int r = r0; r < r1; r += 16) {
    const int yi = r / nxq, xi = r % nxq + 8;
    const double ym = (yi - 0.5 * ny) * dy, xc = (xi - 0.5 * nx) * dx;
    const double a0 = P[0] + ym * (P[2] + ym * (P[5] + ym * P[9]));
    const double a1 = P[1] + ym * (P[4] + ym * P[8]);
    const double a2 = P[3] + ym * P[7];
    const double a3 = P[6];
    const double phc = fma(tt, dwq[r + 8], a0 + xc * (a1 + xc * (a2 + xc * a3)));
    const float an = (float)__builtin_amdgcn_fract(phc);
    const float d1 = (float)((a1 + xc * (2.0 * a2 + 3.0 * a3 * xc)) * dx);
    const float d2 = (float)((a2 + 3.0 * a3 * xc) * dx2);
    const float d3 = (float)(a3 * dx3);
    // p(k) = an + d1 k + d2 k^2 + d3 k^3 at k = j - 8: the even part
    // an + d2 k^2 and the odd factor d1 + d3 k^2 are shared by k and -k
    float ph[16];
    ph[8] = an;
#pragma unroll
    for (int m = 1; m < 8; ++m) {
      const float k = (float)m, k2 = (float)(m * m);
      const float ev = fmaf(d2, k2, an), od = fmaf(d3, k2, d1);
      ph[8 + m] = fmaf(od, k, ev);
      ph[8 - m] = fmaf(od, -k, ev);
    }
    ph[0] = fmaf(fmaf(fmaf(d3, -8.f, d2), -8.f, d1), -8.f, an);
    float c[16], sn[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const float f = __builtin_amdgcn_fractf(fmaf(tf, ddw[r + j], ph[j]));
      c[j] = __builtin_amdgcn_cosf(f);
      sn[j] = __builtin_amdgcn_sinf(f);
    }
    u32x4 A[2][4];
    pack_tile16<BF>(c, sn, A);
#pragma unroll
    for (int g = 0; g < GW; ++g) {
      const u32x4 *zq = zs + ((int64_t)(r >> 4) * NGP + (g0 + g)) * 256 + lane;
      const u32x4 b[4] = {zq[0], zq[64], zq[128], zq[192]};
      acc[0][g] = step6<BF>(A[0], b, acc[0][g]);
      acc[1][g] = step6<BF>(A[1], b, acc[1][g]);
    }
  }
  store_partials<GW>(part + (int64_t)split * Tp * NCP * 2, row0, NCP, g0, lane, acc, wmax, slot);
}

template <int GW, bool BF>
__global__ __launch_bounds__(256) void k_fwd_split_sh(FwdShArgs a) {
  fwd_split_sh_body<GW, BF>(a, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, gridDim.y);
}

// One launch for several problem groups of one shape class (same GW and
// number format): the workgroups of every group's grid are numbered group by
// group (x fastest) and the launch has one workgroup per tile.  Every group's
// x extent is a multiple of eight, so a tile runs on the XCD its index
// assigns it and split_tile's L2 locality holds.  (A persistent form, a
// grid of the resident workgroups walking the tiles with its stride, was
// slower: its loop raised the adjoint's registers to two waves per SIMD.)
template <int GW, bool BF>
__global__ __launch_bounds__(256) void k_fwd_split_sh_grouped(GroupedLaunch<FwdShArgs> G) {
  {
    const int64_t t = blockIdx.x;
    if (t >= G.off[G.ng]) return;
    int g = 0;
    while (g + 1 < G.ng && t >= G.off[g + 1]) ++g;
    const int64_t l = t - G.off[g];
    const int gx = G.gx[g], gy = G.gy[g];
    const int64_t q = l / gx;
    fwd_split_sh_body<GW, BF>(G.a[g], (int)(l - q * gx), (int)(q % gy), (int)(q / gy), gx, gy);
  }
}

// ---------------------------------------------------------------------------
// Operand packing.  Record (step q, group g, lane l): 8 reduction indices
// 16q + 8*(l/32) + i, column col = 16g + l%16, part = (l/16)&1.
//   forward:  b1 = part ? Zi : Zr,   b2 = part ? Zr : -Zi
//   adjoint:  b1 = part ? Yi : Yr,   b2 = part ? -Yr : Yi
// ---------------------------------------------------------------------------

template <bool BF>
__device__ inline void write_record(u32x4 *out, int64_t q, int g, int NGP, int lane, const float (&b1)[8],
                                    const float (&b2)[8]) {
  uint32_t h1[4], l1[4], h2[4], l2[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    split_pair<BF>(b1[2 * m], b1[2 * m + 1], h1[m], l1[m]);
    split_pair<BF>(b2[2 * m], b2[2 * m + 1], h2[m], l2[m]);
  }
  u32x4 *o = out + (q * NGP + g) * 256 + lane;
  o[0] = u32x4{h1[0], h1[1], h1[2], h1[3]};
  o[64] = u32x4{l1[0], l1[1], l1[2], l1[3]};
  o[128] = u32x4{h2[0], h2[1], h2[2], h2[3]};
  o[192] = u32x4{l2[0], l2[1], l2[2], l2[3]};
}

// ---------------------------------------------------------------------------
// Operand scaling of the fp16 form.  An fp16 hi/lo pair represents |v| up to
// 65504 and keeps its ~22-bit precision only while the lo half is normal,
// i.e. for |v| above ~2^-3.  The fp16 form therefore multiplies each packed
// operand by a power of two s = 2^(14 - e), where M < 2^e bounds the
// operand's magnitudes, so that every value lies below 2^14 and values down
// to 2^-17 of the largest keep full precision; the reductions that read the
// contraction's output divide s out again (exact for powers of two).
// M comes from a pre-pass over the operand (image operand, or data given at
// the boundary) or from the forward contraction's per-wave output maxima
// (the residual operand, summed over nsplit partial sums).
// ---------------------------------------------------------------------------

__device__ inline float pow2_scale(float m) {
  if (!(m > 0.f) || !(m <= 3.0e38f)) return 1.f;  // zero, NaN or infinite: unscaled
  int e;
  (void)frexpf(m, &e);
  return ldexpf(1.f, min(126, max(-126, 14 - e)));
}

// Max of v[0..n) over a 256-thread workgroup; every thread returns it.
__device__ inline float block_max(const float *__restrict__ v, int n) {
  __shared__ float wm[4];
  float m = 0.f;
  int i = threadIdx.x;
  for (; i + 768 < n; i += 1024) {  // four independent loads in flight
    const float a = v[i], b = v[i + 256], c = v[i + 512], d = v[i + 768];
    m = fmaxf(m, fmaxf(fmaxf(a, b), fmaxf(c, d)));
  }
  for (; i < n; i += 256) m = fmaxf(m, v[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  __syncthreads();  // an earlier call's readers are done with wm
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  return fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
}

__device__ inline void write_block_max(float m, float *__restrict__ out) {
  __shared__ float wm[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
}

// Pre-pass of the image operand: per-workgroup max of |Re u| + |Im u| over
// the encoded pixels and images, u = x - xsub.  With the same bound of the
// coil maps (taken once per preparation), their product bounds the
// components of Z = S u.  Grid (kAmaxBlocks, P), 256 threads.
__global__ __launch_bounds__(256) void k_amax_z(const float2 *__restrict__ x, const float2 *__restrict__ xsub,
                                                int64_t x_stride, int x_row_stride, int nx, int ny, int B,
                                                int64_t x_pstride, float *__restrict__ amax) {
  const int pz = blockIdx.y;
  const int R = nx * ny;
  x += pz * x_pstride;
  if (xsub) xsub += pz * x_pstride;
  float m = 0.f;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < R; r += gridDim.x * 256) {
    const int yy = r / nx, xx = r % nx;
    for (int b = 0; b < B; ++b) {
      const int64_t o = b * x_stride + (int64_t)yy * x_row_stride + xx;
      float2 u = x[o];
      if (xsub) {
        u.x -= xsub[o].x;
        u.y -= xsub[o].y;
      }
      m = fmaxf(m, fabsf(u.x) + fabsf(u.y));
    }
  }
  write_block_max(m, amax + pz * kAmaxBlocks + blockIdx.x);
}

// Pre-pass of the coil maps [P][n]: per-workgroup max of |Re S| + |Im S|.
__global__ __launch_bounds__(256) void k_amax_l1(const float2 *__restrict__ v, int64_t n, float *__restrict__ amax) {
  const int pz = blockIdx.y;
  v += pz * n;
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float2 a = v[i];
    m = fmaxf(m, fabsf(a.x) + fabsf(a.y));
  }
  write_block_max(m, amax + pz * kAmaxBlocks + blockIdx.x);
}

// Pre-pass of a complex array [P][n] (stride pstride): per-workgroup max of
// the component magnitudes.  Grid (kAmaxBlocks, P), 256 threads.
__global__ __launch_bounds__(256) void k_amax_c(const float2 *__restrict__ v, int64_t n, int64_t pstride,
                                                float *__restrict__ amax) {
  const int pz = blockIdx.y;
  v += pz * pstride;
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float2 a = v[i];
    m = fmaxf(m, fmaxf(fabsf(a.x), fabsf(a.y)));
  }
  write_block_max(m, amax + pz * kAmaxBlocks + blockIdx.x);
}

template <bool BF>
__global__ __launch_bounds__(256) void k_build_z_split(const float2 *__restrict__ smaps, const float2 *__restrict__ x,
                                const float2 *__restrict__ xsub, int64_t x_stride, int x_row_stride, int nx, int ny,
                                int nxq, int Rp, int C, int NC, int NGP, u32x4 *__restrict__ zs, int64_t x_pstride,
                                const float2 *__restrict__ sq, const float *__restrict__ amax,
                                float *__restrict__ scl) {
  const int R = nx * ny;
  const int pz = blockIdx.y;  // problem
  // scaled form: every workgroup derives the same power of two from the pre-pass
  float sc = 1.f;
  if (scl) {
    const int P = gridDim.y;
    const float mu = block_max(amax + pz * kAmaxBlocks, kAmaxBlocks);
    const float ms = block_max(amax + (2 * P + pz) * kAmaxBlocks, kAmaxBlocks);
    sc = pow2_scale(mu * ms);
    if (blockIdx.x == 0 && threadIdx.x == 0) scl[2 * pz] = sc;
  }
  smaps += (int64_t)pz * C * R;
  if (sq) sq += (int64_t)pz * Rp * NGP * 16;
  x += pz * x_pstride;
  if (xsub) xsub += pz * x_pstride;
  zs += (int64_t)pz * Rp * NGP * 16;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)(Rp / 16) * NGP * 64) return;
  const int lane = (int)(id & 63);
  const int g = (int)((id >> 6) % NGP);
  const int64_t q = (id >> 6) / NGP;
  const int col = 16 * g + (lane & 15);
  const int im = (lane >> 4) & 1;
  // the 8 pixels of this lane: every load is issued before the arithmetic
  // (outside pixels and columns read an in-bounds element and give 0)
  const int rq0 = (int)(16 * q + 8 * (lane >> 5));
  int yy = rq0 / nxq, xx = rq0 - yy * nxq;
  const bool colok = col < NC;
  const int b = colok ? col / C : 0, c = colok ? col % C : 0;
  float2 u[8], w[8], sv[8];
  bool ok[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    ok[i] = yy < ny && xx < nx && colok;
    const int yc = ok[i] ? yy : 0, xc = ok[i] ? xx : 0;
    const int64_t o = b * x_stride + (int64_t)yc * x_row_stride + xc;
    u[i] = x[o];
    w[i] = xsub ? xsub[o] : make_float2(0.f, 0.f);
    // (the S table, when given, holds the same value in row-major order)
    sv[i] = sq ? sq[(int64_t)(rq0 + i) * NGP * 16 + col] : smaps[(int64_t)c * R + yc * nx + xc];
    if (++xx == nxq) {
      xx = 0;
      ++yy;
    }
  }
  float b1[8], b2[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    float2 uu = u[i];
    if (xsub) {
      uu.x -= w[i].x;
      uu.y -= w[i].y;
    }
    const float2 s = sv[i];
    const float2 z = ok[i] ? make_float2((s.x * uu.x - s.y * uu.y) * sc, (s.x * uu.y + s.y * uu.x) * sc)
                           : make_float2(0.f, 0.f);
    b1[i] = im ? z.y : z.x;
    b2[i] = im ? z.x : -z.y;
  }
  write_record<BF>(zs, q, g, NGP, lane, b1, b2);
}

// Adjoint operand from y [B][T][C] (src_abi) or from forward partials minus
// y_meas (src_part, nsplit partial arrays in [Tp][NCP] layout).
// With perm, K index 8h + i of a step holds sample 8(i/4) + 4h + i%4 of its
// 16 (the order in which the polynomial adjoint produces its phase tile).
template <bool BF>
__global__ __launch_bounds__(256) void k_pack_y_split(const float2 *__restrict__ src_abi,
                                                      const float2 *__restrict__ src_part, int nsplit,
                                                      const float2 *__restrict__ y_meas, int64_t T, int64_t Tp, int C,
                                                      int NC, int NCP, u32x4 *__restrict__ ys, int perm,
                                                      const float *__restrict__ bnd, int nbnd,
                                                      const float *__restrict__ bnd_meas, float *__restrict__ scl) {
  const int NGP = NCP / 16;
  const int pz = blockIdx.y;  // problem
  // scaled form: the bound of the operand is max(bnd) (src_abi: its pre-pass;
  // src_part: the forward's per-wave maxima, in units of the forward operand's
  // scale, times nsplit) plus max(bnd_meas) (the pre-pass of y_meas, if any)
  float sc = 1.f, inv_z = 1.f;
  if (scl) {
    float m = block_max(bnd + (int64_t)pz * nbnd, nbnd);
    if (src_part) {
      inv_z = 1.f / scl[2 * pz];
      m = m * (float)nsplit * inv_z;
    }
    if (bnd_meas) m += block_max(bnd_meas + pz * kAmaxBlocks, kAmaxBlocks);
    sc = pow2_scale(m);
    if (blockIdx.x == 0 && threadIdx.x == 0) scl[2 * pz + 1] = sc;
  }
  if (src_abi) src_abi += pz * T * NC;
  if (src_part) src_part += pz * nsplit * Tp * NCP;
  if (y_meas) y_meas += pz * T * NC;
  ys += pz * Tp * NGP * 16;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (Tp / 16) * NGP * 64) return;
  const int lane = (int)(id & 63);
  const int g = (int)((id >> 6) % NGP);
  const int64_t q = (id >> 6) / NGP;
  const int col = 16 * g + (lane & 15);
  const int im = (lane >> 4) & 1;
  const int b = col / C, c = col % C;
  int64_t t[8];
  bool ok[8];
  float2 y[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    t[i] = 16 * q + (perm ? 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3) : 8 * (lane >> 5) + i);
    ok[i] = t[i] < T && col < NC;
    y[i] = make_float2(0.f, 0.f);
  }
  if (src_abi) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (ok[i]) y[i] = src_abi[((int64_t)b * T + t[i]) * C + c];
  } else {
    // split order per sample as in a plain loop; the loads of four splits x
    // eight samples are independent and issue together
    int k = 0;
    for (; k + 4 <= nsplit; k += 4) {
      float2 v[4][8];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 8; ++i)
          v[u][i] = ok[i] ? src_part[((int64_t)(k + u) * Tp + t[i]) * NCP + col] : make_float2(0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          y[i].x += v[u][i].x;
          y[i].y += v[u][i].y;
        }
    }
    for (; k < nsplit; ++k) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (ok[i]) {
          const float2 v = src_part[((int64_t)k * Tp + t[i]) * NCP + col];
          y[i].x += v.x;
          y[i].y += v.y;
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      y[i].x *= inv_z;
      y[i].y *= inv_z;
    }
    if (y_meas) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (ok[i]) {
          const float2 m = y_meas[((int64_t)b * T + t[i]) * C + c];
          y[i].x -= m.x;
          y[i].y -= m.y;
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    y[i].x *= sc;
    y[i].y *= sc;
  }
  float b1[8], b2[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    b1[i] = im ? y[i].y : y[i].x;
    b2[i] = im ? -y[i].x : y[i].y;
  }
  write_record<BF>(ys, q, g, NGP, lane, b1, b2);
}

// Per-tile differences d[16q + j][k] = (float)(src[16q + j][k] - src[16q + 8][k]).
__global__ void k_tile_diff(const double *__restrict__ src, float *__restrict__ d, int64_t rows, int NT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * NT) return;
  src += blockIdx.y * rows * NT;  // problem
  d += blockIdx.y * rows * NT;
  const int64_t r = i / NT;
  const int k = (int)(i % NT);
  const int64_t centre = (r & ~int64_t(15)) + 8;
  d[i] = (float)(src[r * NT + k] - src[centre * NT + k]);
}

// Monomial coefficients of the solid harmonics at fixed z (rows l, columns
// m over 1, x, y, x^2, xy, y^2, x^3, x^2 y, x y^2, y^3).
struct MonoMatrix {
  double m[16][10];
};

__host__ __device__ inline MonoMatrix mono_matrix(double z) {
  MonoMatrix M{};
  auto &m = M.m;
  m[0][0] = 1;
  m[1][1] = 1;
  m[2][2] = 1;
  m[3][0] = z;
  m[4][4] = 1;
  m[5][2] = z;
  m[6][0] = 2 * z * z, m[6][3] = -1, m[6][5] = -1;
  m[7][1] = z;
  m[8][3] = 1, m[8][5] = -1;
  m[9][7] = 3, m[9][9] = -1;
  m[10][4] = z;
  m[11][2] = 4 * z * z, m[11][7] = -1, m[11][9] = -1;
  m[12][0] = 2 * z * z * z, m[12][3] = -3 * z, m[12][5] = -3 * z;
  m[13][1] = 4 * z * z, m[13][6] = -1, m[13][8] = -1;
  m[14][3] = z, m[14][5] = -z;
  m[15][6] = 1, m[15][8] = -3;
  return M;
}

// pmono[t][m] = sum_l kap[t][l] M[l][m] (m < 10), pmono[t][10] = t; the
// monomial matrix M comes from the problem's slice position (z0s[p], or M0).
__global__ void k_prep_pmono(const double *__restrict__ kap, int NT, int L, int64_t Tp, MonoMatrix M0,
                             const double *__restrict__ z0s, double *__restrict__ pmono) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Tp) return;
  const int pz = blockIdx.y;
  kap += pz * Tp * NT;
  pmono += pz * Tp * 12;
  MonoMatrix M = z0s ? mono_matrix(z0s[pz]) : M0;
  double out[12];
  for (int m = 0; m < 12; ++m) out[m] = 0.0;
  for (int l = 0; l < L; ++l) {
    const double k = kap[t * NT + l];
    for (int m = 0; m < 10; ++m) out[m] = fma(k, M.m[l][m], out[m]);
  }
  out[10] = kap[t * NT + L];
  for (int m = 0; m < 12; ++m) pmono[t * 12 + m] = out[m];
}

// A operand of the adjoint's phase-increment product, in lane order.  For the
// 32-sample tile q and lane l (sample t = 32q + l%32, half hl = l/32), with
// d_m = pmono[t][m] - pmono[32q + 16][m] (monomials in pmono order), the
// increment at a pixel of image row y is the cubic in x
//   C_0 + C_1 x + C_2 x^2 + C_3 x^3 + d10 dw0,
//   C_0 = d0 + d2 y + d5 y^2 + d9 y^3,  C_1 = d1 + d4 y + d8 y^2,
//   C_2 = d3 + d7 y,                    C_3 = d6,
// and lane l holds the coefficients the adjoint evaluates at a block's row:
// [0..3] the cubic in y of C_hl, [4..5] the linear one of C_{2+hl}, [6] d10
// (hl = 0, the dw0 term) or 1 (hl = 1, the anchor term).
__global__ void k_prep_dpa(const double *__restrict__ pmono, int64_t Tp, float *__restrict__ dpa) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Tp / 32 * 64) return;
  pmono += blockIdx.y * Tp * 12;  // problem
  dpa += blockIdx.y * Tp * 16;
  const int64_t q = i >> 6;
  const int l = (int)(i & 63);
  const int64_t t = 32 * q + (l & 31), ta = 32 * q + 16;
  double d[11];
  for (int m = 0; m <= 10; ++m) d[m] = pmono[t * 12 + m] - pmono[ta * 12 + m];
  const bool hl = (l >> 5) != 0;
  const double c[7] = {hl ? d[1] : d[0], hl ? d[4] : d[2], hl ? d[8] : d[5], hl ? 0.0 : d[9],
                       hl ? d[6] : d[3], hl ? 0.0 : d[7], hl ? 1.0 : d[10]};
  float v[8];
  for (int j = 0; j < 7; ++j) v[j] = (float)c[j];
  v[7] = 0.f;
  float4 *o = reinterpret_cast<float4 *>(dpa + i * 8);
  o[0] = make_float4(v[0], v[1], v[2], v[3]);
  o[1] = make_float4(v[4], v[5], v[6], v[7]);
}

// Anchors of the polynomial split adjoint: for the 32-sample tile q and the
// row-padded pixel rq, the phase of the tile's centre sample 32q + 16 at that
// pixel, sum_m P_m(t) mono_m(x, y) + t dw0(r)/2pi, evaluated in FP64 (nested
// in y, then in x) and reduced to turns in [0, 1).  The adjoint adds its FP32
// phase increments within the tile to it.
__global__ void k_prep_anchor(const double *__restrict__ pmono, const double *__restrict__ dwq, int64_t Tp, int Rp,
                              int nxq, int nx, int ny, double dx, double dy, float *__restrict__ anc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Tp / 32 * Rp) return;
  const int pz = blockIdx.y;  // problem
  pmono += pz * Tp * 12;
  dwq += (int64_t)pz * Rp;
  anc += (int64_t)pz * (Tp / 32) * Rp;
  const int64_t q = i / Rp;
  const int rq = (int)(i - q * Rp);
  const double x = (rq % nxq - 0.5 * nx) * dx, y = (rq / nxq - 0.5 * ny) * dy, w = dwq[rq];
  const double *pc = pmono + (32 * q + 16) * 12;
  // monomial order of pmono: 1, x, y, x^2, xy, y^2, x^3, x^2 y, x y^2, y^3
  const double a0 = fma(y, fma(y, fma(y, pc[9], pc[5]), pc[2]), pc[0]);
  const double a1 = fma(y, fma(y, pc[8], pc[4]), pc[1]);
  const double a2 = fma(y, pc[7], pc[3]);
  const double pa = fma(pc[10], w, fma(x, fma(x, fma(x, pc[6], a2), a1), a0));
  anc[i] = (float)__builtin_amdgcn_fract(pa);
}

// dwq[r'] = dw0(r)/2pi in the row-padded pixel layout.
__global__ void k_prep_dwq(const double *__restrict__ dw0, int nx, int ny, int nxq, int Rp, double *__restrict__ dwq) {
  const int rq = blockIdx.x * blockDim.x + threadIdx.x;
  if (rq >= Rp) return;
  if (dw0) dw0 += (int64_t)blockIdx.y * nx * ny;  // problem
  dwq += (int64_t)blockIdx.y * Rp;
  const int yy = rq / nxq, xx = rq % nxq;
  double v = 0.0;
  if (dw0 && yy < ny && xx < nx) v = dw0[yy * nx + xx] * 0.15915494309189533576888376337251436;
  dwq[rq] = v;
}

// sq[row][col] = S_col(r) at pixel r = (row / nxq) * nx + row % nxq (the
// adjoint partial-sum layout), zero on padding rows and columns.
__global__ void k_prep_sq(const float2 *__restrict__ smaps, int nx, int ny, int nxq, int Rp, int C, int NCP,
                          float2 *__restrict__ sq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Rp * NCP) return;
  const int pz = blockIdx.y;  // problem
  const int R = nx * ny;
  const int row = (int)(i / NCP), col = (int)(i % NCP);
  const int yy = row / nxq, xx = row % nxq;
  float2 v = make_float2(0.f, 0.f);
  if (col < C && xx < nx && yy < ny) v = smaps[((int64_t)pz * C + col) * R + yy * nx + xx];
  sq[(int64_t)pz * Rp * NCP + i] = v;
}

int sh_prepare(const EncPlan &p, const expenc_op *op, const EncBuffers &b, hipStream_t s) {
  auto gp = [&](int64_t n) { return dim3((unsigned)ceil_div(n, 256), (unsigned)p.P); };
  k_prep_pmono<<<gp(p.Tp), 256, 0, s>>>(b.kap, p.NT, p.L, p.Tp, mono_matrix(p.z0), p.z0s, b.pmono);
  EX_LAUNCHED("monomial coefficients");
  if (p.prec != EXPENC_FP32) {
    k_prep_dpa<<<gp(p.Tp / 32 * 64), 256, 0, s>>>(b.pmono, p.Tp, b.dpa);
    EX_LAUNCHED("increment table (samples)");
  }
  k_prep_dwq<<<gp(p.Rp), 256, 0, s>>>(op->dw0, p.nx, p.ny, p.nxq, p.Rp, b.dwq);
  EX_LAUNCHED("off-resonance layout");
  if (p.adj_anc) {
    if (!b.anc) return fail(EXPENC_EINVAL, "anchor table of a split plan is not carved");
    k_prep_anchor<<<gp(p.Tp / 32 * p.Rp), 256, 0, s>>>(b.pmono, b.dwq, p.Tp, p.Rp, p.nxq, p.nx, p.ny, p.dx, p.dy,
                                                        b.anc);
    EX_LAUNCHED("adjoint anchors");
  }
  k_tile_diff<<<gp(p.Rp), 256, 0, s>>>(b.dwq, b.ddw, p.Rp, 1);
  EX_LAUNCHED("tile differences (pixels)");
  return EXPENC_OK;
}

int split_prepare(const EncPlan &p, const expenc_op *op, const EncBuffers &b, hipStream_t s) {
  auto gp = [&](int64_t n) { return dim3((unsigned)ceil_div(n, 256), (unsigned)p.P); };
  if (p.scaled) {
    // bound of the coil maps for the fp16 operand scaling (third amax section)
    if (!b.scl || !b.amax || !b.wmax) return fail(EXPENC_EINVAL, "scale buffers of an fp16 plan are not carved");
    k_amax_l1<<<dim3(kAmaxBlocks, (unsigned)p.P), 256, 0, s>>>(reinterpret_cast<const float2 *>(op->smaps),
                                                               (int64_t)p.C * p.R, b.amax + (size_t)2 * p.P * kAmaxBlocks);
    EX_LAUNCHED("coil-map bound");
  }
  if (p.comb) {
    if (!b.sq) return fail(EXPENC_EINVAL, "coil table of a single-image split plan is not carved");
    k_prep_sq<<<gp((int64_t)p.Rp * p.NCP), 256, 0, s>>>(reinterpret_cast<const float2 *>(op->smaps), p.nx, p.ny,
                                                          p.nxq, p.Rp, p.C, p.NCP, b.sq);
    EX_LAUNCHED("coil table");
  }
  if (p.sh) return sh_prepare(p, op, b, s);
  k_tile_diff<<<gp((int64_t)p.Rp * p.NT), 256, 0, s>>>(b.bet, b.dbet, p.Rp, p.NT);
  EX_LAUNCHED("tile differences (pixels)");
  k_tile_diff<<<gp(p.Tp * p.NT), 256, 0, s>>>(b.kap, b.dkap, p.Tp, p.NT);
  EX_LAUNCHED("tile differences (samples)");
  return EXPENC_OK;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int NT, bool BF>
static void launch_fwd_split(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid(p.Tp / 256 * p.fwd_split), (unsigned)p.NGY, (unsigned)p.P);
  float *part = reinterpret_cast<float *>(b.part);
  const u32x4 *zs = reinterpret_cast<const u32x4 *>(b.zs);
  if (p.GW == 2)
    k_fwd_split<NT, 2, BF><<<grid, 256, 0, s>>>(b.kap, b.bet, b.dbet, zs, part, p.Tp, p.Rp, p.NCP, p.fwd_chunk,
                                                p.fwd_split);
  else
    k_fwd_split<NT, 1, BF><<<grid, 256, 0, s>>>(b.kap, b.bet, b.dbet, zs, part, p.Tp, p.Rp, p.NCP, p.fwd_chunk,
                                                p.fwd_split);
}

template <int NT, bool BF>
static void launch_adj_split(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid((int64_t)p.Rp / 256 * p.adj_split), (unsigned)p.NGY, (unsigned)p.P);
  float *part = reinterpret_cast<float *>(b.part);
  const u32x4 *ys = reinterpret_cast<const u32x4 *>(b.ys);
  const float2 *sm = p.comb ? b.sq : nullptr;
  if (p.GW == 2)
    k_adj_split<NT, 2, BF><<<grid, 256, 0, s>>>(b.kap, b.bet, b.dkap, ys, part, p.Rp, p.Tp, p.NCP, p.adj_chunk,
                                                p.adj_split, sm);
  else
    k_adj_split<NT, 1, BF><<<grid, 256, 0, s>>>(b.kap, b.bet, b.dkap, ys, part, p.Rp, p.Tp, p.NCP, p.adj_chunk,
                                                p.adj_split, sm);
}

template <bool BF>
static void fwd_split_nt(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  switch (p.NT) {
    case 4: launch_fwd_split<4, BF>(p, b, s); break;
    case 10: launch_fwd_split<10, BF>(p, b, s); break;
    default: launch_fwd_split<17, BF>(p, b, s); break;
  }
}

template <bool BF>
static void adj_split_nt(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  switch (p.NT) {
    case 4: launch_adj_split<4, BF>(p, b, s); break;
    case 10: launch_adj_split<10, BF>(p, b, s); break;
    default: launch_adj_split<17, BF>(p, b, s); break;
  }
}

static FwdShArgs fwd_sh_args(const EncPlan &p, const EncBuffers &b) {
  return FwdShArgs{b.pmono, b.dwq, b.ddw, reinterpret_cast<const u32x4 *>(b.zs), reinterpret_cast<float *>(b.part),
                   p.scaled ? b.wmax : nullptr, p.Tp, p.Rp, p.NCP, p.fwd_chunk, p.fwd_split, p.nxq, p.nx, p.ny,
                   p.dx, p.dy};
}

template <bool BF>
static void fwd_split_sh(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid(p.Tp / 256 * p.fwd_split), (unsigned)p.NGY, (unsigned)p.P);
  const FwdShArgs a = fwd_sh_args(p, b);
  if (p.GW == 2)
    k_fwd_split_sh<2, BF><<<grid, 256, 0, s>>>(a);
  else
    k_fwd_split_sh<1, BF><<<grid, 256, 0, s>>>(a);
}

bool split_groupable(const EncPlan &a, const EncPlan &b) {
  return a.sh && b.sh && a.prec == b.prec && a.prec != EXPENC_FP32 && a.GW == b.GW && a.comb == b.comb &&
         a.scaled == b.scaled;
}

template <int GW, bool BF>
static int fwd_grouped(const EncPlan *const *p, const EncBuffers *const *b, int n, hipStream_t s) {
  GroupedLaunch<FwdShArgs> G{};
  G.ng = n;
  G.off[0] = 0;
  for (int g = 0; g < n; ++g) {
    G.a[g] = fwd_sh_args(*p[g], *b[g]);
    G.gx[g] = (int)split_grid(p[g]->Tp / 256 * p[g]->fwd_split);
    G.gy[g] = p[g]->NGY;
    G.off[g + 1] = G.off[g] + (int64_t)G.gx[g] * G.gy[g] * p[g]->P;
  }
  if (G.off[n] > INT32_MAX) return fail(EXPENC_EUNSUPPORTED, "grouped launch larger than 2^31 workgroups");
  k_fwd_split_sh_grouped<GW, BF><<<(unsigned)G.off[n], 256, 0, s>>>(G);
  EX_LAUNCHED("grouped forward contraction");
  return EXPENC_OK;
}

int split_forward_grouped(const EncPlan *const *p, const EncBuffers *const *b, int n, hipStream_t s) {
  for (int i = 0; i < n; i += kMaxGrouped) {
    const int m = std::min(kMaxGrouped, n - i);
    for (int g = i; g < i + m; ++g)
      if (!split_groupable(*p[i], *p[g])) return fail(EXPENC_EINVAL, "plans of a grouped launch differ in shape");
    const bool bf = p[i]->prec == EXPENC_BF16_SPLIT;
    int rc;
    if (p[i]->GW == 2) rc = bf ? fwd_grouped<2, true>(p + i, b + i, m, s) : fwd_grouped<2, false>(p + i, b + i, m, s);
    else rc = bf ? fwd_grouped<1, true>(p + i, b + i, m, s) : fwd_grouped<1, false>(p + i, b + i, m, s);
    EX_TRY(rc);
  }
  return EXPENC_OK;
}

void split_forward_launch(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  const bool bf = p.prec == EXPENC_BF16_SPLIT;
  if (p.sh) {
    if (bf) fwd_split_sh<true>(p, b, s);
    else fwd_split_sh<false>(p, b, s);
  } else {
    if (bf) fwd_split_nt<true>(p, b, s);
    else fwd_split_nt<false>(p, b, s);
  }
}

void split_adjoint_launch(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  const bool bf = p.prec == EXPENC_BF16_SPLIT;
  if (p.sh) {
    split_adjoint_sh_launch(p, b, s);
  } else {
    if (bf) adj_split_nt<true>(p, b, s);
    else adj_split_nt<false>(p, b, s);
  }
}

int split_build_z(const EncPlan &p, const float *smaps, const float2 *x, const float2 *xsub, int64_t x_stride,
                  int32_t x_row_stride, const EncBuffers &b, hipStream_t s, int64_t x_pstride) {
  const int NGP = p.NCP / 16;
  const int64_t n = (int64_t)(p.Rp / 16) * NGP * 64;
  const dim3 nb((unsigned)ceil_div(n, 256), (unsigned)p.P);
  const float2 *sm = reinterpret_cast<const float2 *>(smaps);
  u32x4 *zs = reinterpret_cast<u32x4 *>(b.zs);
  if (p.scaled) {
    if (!b.scl || !b.amax || !b.wmax) return fail(EXPENC_EINVAL, "scale buffers of an fp16 plan are not carved");
    k_amax_z<<<dim3(kAmaxBlocks, (unsigned)p.P), 256, 0, s>>>(x, xsub, x_stride, x_row_stride, p.nx, p.ny, p.B,
                                                              x_pstride, b.amax);
    EX_LAUNCHED("operand bound");
  }
  float *scl = p.scaled ? b.scl : nullptr;
  if (p.prec == EXPENC_BF16_SPLIT)
    k_build_z_split<true><<<nb, 256, 0, s>>>(sm, x, xsub, x_stride, x_row_stride, p.nx, p.ny, p.nxq, p.Rp, p.C,
                                             p.NC, NGP, zs, x_pstride, p.comb ? b.sq : nullptr, b.amax, scl);
  else
    k_build_z_split<false><<<nb, 256, 0, s>>>(sm, x, xsub, x_stride, x_row_stride, p.nx, p.ny, p.nxq, p.Rp, p.C,
                                              p.NC, NGP, zs, x_pstride, p.comb ? b.sq : nullptr, b.amax, scl);
  EX_LAUNCHED("build_z split");
  return EXPENC_OK;
}

int split_pack_y(const EncPlan &p, const float2 *y_abi, bool from_partials, const float2 *y_meas,
                 const EncBuffers &b, hipStream_t s) {
  const int NGP = p.NCP / 16;
  const int64_t n = (p.Tp / 16) * NGP * 64;
  const dim3 nb((unsigned)ceil_div(n, 256), (unsigned)p.P);
  u32x4 *ys = reinterpret_cast<u32x4 *>(b.ys);
  const float2 *part = from_partials ? b.part : nullptr;
  const float *bnd = nullptr, *bnd_meas = nullptr;
  int nbnd = 0;
  if (p.scaled) {
    if (!b.scl || !b.amax || !b.wmax) return fail(EXPENC_EINVAL, "scale buffers of an fp16 plan are not carved");
    const dim3 ng(kAmaxBlocks, (unsigned)p.P);
    const int64_t ny_el = p.T * p.NC;  // [B][T][C] per problem
    if (!from_partials) {
      k_amax_c<<<ng, 256, 0, s>>>(y_abi, ny_el, ny_el, b.amax);
      EX_LAUNCHED("operand bound");
      bnd = b.amax;
      nbnd = kAmaxBlocks;
    } else {
      if (p.sh) {
        // the polynomial forward writes its per-wave output maxima
        bnd = b.wmax;
        nbnd = p.nwmax;
      } else {
        // (the maps-kind forward does not: a pre-pass over its partial sums)
        const int64_t np = (int64_t)p.fwd_split * p.Tp * p.NCP;
        k_amax_c<<<ng, 256, 0, s>>>(b.part, np, np, b.amax);
        EX_LAUNCHED("operand bound");
        bnd = b.amax;
        nbnd = kAmaxBlocks;
      }
      if (y_meas) {
        float *am = b.amax + (size_t)p.P * kAmaxBlocks;
        k_amax_c<<<ng, 256, 0, s>>>(y_meas, ny_el, ny_el, am);
        EX_LAUNCHED("operand bound");
        bnd_meas = am;
      }
    }
  }
  float *scl = p.scaled ? b.scl : nullptr;
  if (p.prec == EXPENC_BF16_SPLIT)
    k_pack_y_split<true><<<nb, 256, 0, s>>>(y_abi, part, p.fwd_split, y_meas, p.T, p.Tp, p.C, p.NC, p.NCP, ys,
                                            p.sh ? 1 : 0, bnd, nbnd, bnd_meas, scl);
  else
    k_pack_y_split<false><<<nb, 256, 0, s>>>(y_abi, part, p.fwd_split, y_meas, p.T, p.Tp, p.C, p.NC, p.NCP, ys,
                                             p.sh ? 1 : 0, bnd, nbnd, bnd_meas, scl);
  EX_LAUNCHED("pack_y split");
  return EXPENC_OK;
}

}  // namespace expenc
