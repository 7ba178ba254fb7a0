// The split adjoint contraction with the solid-harmonic basis in
// polynomial form (the polynomial forms and the split arithmetic are
// described in split.hip).  It sits in a translation unit of its own so that
// it can be built with its own code-generation options.
#include <vector>

#include "internal.h"
#include "split_dev.h"

namespace expenc {

// Arguments of one problem group's adjoint launch.
struct AdjShArgs {
  const float *anc;
  const float *dpa;
  const double *dwq;
  const u32x4 *ys;
  float *part;
  const float2 *sq;
  int64_t Tp;
  int Rp, NCP, chunk, nsplit, nxq, nx, ny;
  double dx, dy;
  Bf16Masks mk;
};

// One workgroup of the adjoint (workgroup bx, by, bz of a grid with gy
// column groups).
//
// Phase of a 32-sample x 32-pixel block: the FP64 anchor of the tile's centre
// sample at each pixel (table anc) plus the increment over the tile.  With
// the pixels of the block in one image row y the increment is a cubic in x,
// sum_k C_k(t, y) x^k + d10(t) dw0, whose coefficients are polynomials in y
// (k_prep_dpa): a rank-6 product, three v_mfma_f32_32x32x2_f32 with terms
// (1 | x), (x^2 | x^3), (dw0 | anchor) against (C_0 | C_1), (C_2 | C_3),
// (d10 | 1) evaluated at the block's row.  A block that continues into the
// next row (when the padded row length nxq is not a multiple of 32) adds,
// for its pixels in that row only, the change of the coefficients between
// the two rows: E_k = C_k(t, y1) - C_k(t, y0) against (1 | x), (x^2 | 0) on
// those pixels and 0 on the others (E_3 = 0: C_3 does not depend on y), two
// more products; CROSS instantiates that case (nxq not a multiple of 32).
template <int GW, bool BF, bool CROSS>
__device__ inline void adj_split_sh_body(const AdjShArgs &a, int bx, int by, int bz, int gy) {
  const float *__restrict__ anc = a.anc;
  const float *__restrict__ dpa = a.dpa;
  const double *__restrict__ dwq = a.dwq;
  const u32x4 *__restrict__ ys = a.ys;
  float *__restrict__ part = a.part;
  const float2 *__restrict__ sq = a.sq;
  const int64_t Tp = a.Tp;
  const int Rp = a.Rp, NCP = a.NCP, chunk = a.chunk, nsplit = a.nsplit, nxq = a.nxq, nx = a.nx, ny = a.ny;
  const double dx = a.dx, dy = a.dy;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int hl = lane >> 5, jl = lane & 31;
  int split, rb;
  if (!(sq ? split_tile_rows(bx, Rp / 256, nsplit, &split, &rb) : split_tile(bx, Rp / 256, nsplit, &split, &rb))) return;
  const int64_t row0 = (int64_t)rb * 256 + wave * 64;
  const int g0 = by * GW;
  const int NGP = NCP / 16;
  const int pz = bz;  // problem
  anc += pz * (Tp / 32) * Rp;
  dpa += pz * Tp * 16;
  dwq += (int64_t)pz * Rp;
  ys += pz * Tp * NGP * 16;
  // this lane's pixel in each 32-pixel block and its B operands: terms
  // 2J + hl of the row product, and of the next-row correction
  float bm[2][3], bd[2][2];
  float y0[2], y1[2];  // image rows of the block's first and last pixel
  bool two[2];         // the block continues into the next row (uniform)
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const int rs = (int)(row0 + 32 * blk), rq = rs + jl;
    const int r0 = rs / nxq, r1 = (rs + 31) / nxq;
    const double x = (rq % nxq - 0.5 * nx) * dx, w = dwq[rq];
    y0[blk] = (float)((r0 - 0.5 * ny) * dy);
    y1[blk] = (float)((r1 - 0.5 * ny) * dy);
    two[blk] = r1 != r0;
    const bool next = rq / nxq != r0;
    bm[blk][0] = (float)(hl ? x : 1.0);
    bm[blk][1] = (float)(hl ? x * x * x : x * x);
    bm[blk][2] = (float)w;  // lanes 32..63 replace it by the anchor per step
    bd[blk][0] = next ? bm[blk][0] : 0.f;
    bd[blk][1] = next && !hl ? bm[blk][1] : 0.f;
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
  for (int64_t t = t0; t < t1; t += 32) {
    // this lane's sample: the coefficients of C_hl(y) (cubic) and
    // C_{2+hl}(y) (linear), then d10 or 1
    const float4 *ap = reinterpret_cast<const float4 *>(dpa + ((t >> 5) * 64 + lane) * 8);
    const float4 a03 = ap[0], a47 = ap[1];
    // anchor: FP64 phase of the tile's centre sample at this lane's pixels
    // in turns (from the table); it enters the product with A = 1
    const float *ap2 = anc + (t >> 5) * Rp + row0 + jl;
    const float an[2] = {ap2[0], ap2[32]};
    f32x16 ph[2];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const float ya = y0[blk];
      const float c0 = fmaf(ya, fmaf(ya, fmaf(ya, a03.w, a03.z), a03.y), a03.x);
      const float c1 = fmaf(ya, a47.y, a47.x);
#pragma unroll
      for (int v = 0; v < 16; ++v) ph[blk][v] = 0.f;
      ph[blk] = __builtin_amdgcn_mfma_f32_32x32x2f32(c0, bm[blk][0], ph[blk], 0, 0, 0);
      ph[blk] = __builtin_amdgcn_mfma_f32_32x32x2f32(c1, bm[blk][1], ph[blk], 0, 0, 0);
      ph[blk] = __builtin_amdgcn_mfma_f32_32x32x2f32(a47.z, hl ? an[blk] : bm[blk][2], ph[blk], 0, 0, 0);
      if (CROSS && two[blk]) {
        const float yb = y1[blk];
        const float e0 = fmaf(yb, fmaf(yb, fmaf(yb, a03.w, a03.z), a03.y), a03.x) - c0;
        const float e1 = fmaf(yb, a47.y, a47.x) - c1;
        ph[blk] = __builtin_amdgcn_mfma_f32_32x32x2f32(e0, bd[blk][0], ph[blk], 0, 0, 0);
        ph[blk] = __builtin_amdgcn_mfma_f32_32x32x2f32(e1, bd[blk][1], ph[blk], 0, 0, 0);
      }
    }
    // two contraction steps of 16 samples; ph[blk][8h + i] is sample
    // 16h + 8(i/4) + 4hl + i%4 of pixel jl, which is K index 8hl + i of
    // step h in the permuted sample order of the adjoint records
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u32x4 b[GW][4];
#pragma unroll
      for (int g = 0; g < GW; ++g) {
        const u32x4 *yq = ys + (((t >> 4) + h) * NGP + (g0 + g)) * 256 + lane;
        b[g][0] = yq[0];
        b[g][1] = yq[64];
        b[g][2] = yq[128];
        b[g][3] = yq[192];
      }
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        uint32_t w[4][4];  // [kind: c hi, c lo, s hi, s lo][word]
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          float c2[2], s2[2];
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const float f = __builtin_amdgcn_fractf(ph[blk][8 * h + 2 * m + e]);
            c2[e] = __builtin_amdgcn_cosf(f);
            s2[e] = __builtin_amdgcn_sinf(f);
          }
          split_pair<BF>(c2[0], c2[1], w[0][m], w[1][m], a.mk);
          split_pair<BF>(s2[0], s2[1], w[2][m], w[3][m], a.mk);
        }
        const u32x4 A[4] = {u32x4{w[0][0], w[0][1], w[0][2], w[0][3]}, u32x4{w[1][0], w[1][1], w[1][2], w[1][3]},
                            u32x4{w[2][0], w[2][1], w[2][2], w[2][3]}, u32x4{w[3][0], w[3][1], w[3][2], w[3][3]}};
#pragma unroll
        for (int g = 0; g < GW; ++g) acc[blk][g] = step6<BF>(A, b[g], acc[blk][g]);
      }
    }
  }
  adj_epilogue<GW>(part, sq, Rp, NCP, nsplit, split, pz, by, gy, row0, g0, lane, acc);
}

// The bf16 build is held to three waves per SIMD: left to itself the
// compiler may take a few more registers than that allows, and two waves
// per SIMD measured 3 % slower.
template <int GW, bool BF, bool CROSS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BF ? 3 : 1))) void k_adj_split_sh(AdjShArgs a) {
  adj_split_sh_body<GW, BF, CROSS>(a, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.y);
}

// One launch over several problem groups, one workgroup per tile (the
// forward's grouped kernel in split.hip describes the numbering and why the
// XCD mapping holds).
template <int GW, bool BF, bool CROSS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BF ? 3 : 1))) void k_adj_split_sh_grouped(
    GroupedLaunch<AdjShArgs> G) {
  {
    const int64_t t = blockIdx.x;
    if (t >= G.off[G.ng]) return;
    int g = 0;
    while (g + 1 < G.ng && t >= G.off[g + 1]) ++g;
    const int64_t l = t - G.off[g];
    const int gx = G.gx[g], gy = G.gy[g];
    const int64_t q = l / gx;
    adj_split_sh_body<GW, BF, CROSS>(G.a[g], (int)(l - q * gx), (int)(q % gy), (int)(q / gy), gy);
  }
}

static AdjShArgs adj_sh_args(const EncPlan &p, const EncBuffers &b) {
  return AdjShArgs{b.anc, b.dpa, b.dwq, reinterpret_cast<const u32x4 *>(b.ys), reinterpret_cast<float *>(b.part),
                   p.comb ? b.sq : nullptr, p.Tp, p.Rp, p.NCP, p.adj_chunk, p.adj_split, p.nxq, p.nx, p.ny, p.dx,
                   p.dy, bf16_masks()};
}

// Blocks of 32 pixels continue into the next image row unless the padded row
// length is a multiple of 32.
static bool adj_cross(const EncPlan &p) { return p.nxq % 32 != 0; }

template <bool BF, bool CROSS>
static void adj_split_sh(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid((int64_t)p.Rp / 256 * p.adj_split), (unsigned)p.NGY, (unsigned)p.P);
  const AdjShArgs a = adj_sh_args(p, b);
  if (p.GW == 2)
    k_adj_split_sh<2, BF, CROSS><<<grid, 256, 0, s>>>(a);
  else
    k_adj_split_sh<1, BF, CROSS><<<grid, 256, 0, s>>>(a);
}

template <int GW, bool BF, bool CROSS>
static int adj_grouped(const EncPlan *const *p, const EncBuffers *const *b, int n, hipStream_t s) {
  GroupedLaunch<AdjShArgs> G{};
  G.ng = n;
  G.off[0] = 0;
  for (int g = 0; g < n; ++g) {
    G.a[g] = adj_sh_args(*p[g], *b[g]);
    G.gx[g] = (int)split_grid((int64_t)p[g]->Rp / 256 * p[g]->adj_split);
    G.gy[g] = p[g]->NGY;
    G.off[g + 1] = G.off[g] + (int64_t)G.gx[g] * G.gy[g] * p[g]->P;
  }
  if (G.off[n] > INT32_MAX) return fail(EXPENC_EUNSUPPORTED, "grouped launch larger than 2^31 workgroups");
  k_adj_split_sh_grouped<GW, BF, CROSS><<<(unsigned)G.off[n], 256, 0, s>>>(G);
  EX_LAUNCHED("grouped adjoint contraction");
  return EXPENC_OK;
}

// Grouped launches (chunks of kMaxGrouped) of plans of one kernel variant.
template <bool CROSS>
static int adj_grouped_class(const EncPlan *const *p, const EncBuffers *const *b, int n, hipStream_t s) {
  for (int i = 0; i < n; i += kMaxGrouped) {
    const int m = std::min(kMaxGrouped, n - i);
    const bool bf = p[i]->prec == EXPENC_BF16_SPLIT;
    int rc;
    if (p[i]->GW == 2)
      rc = bf ? adj_grouped<2, true, CROSS>(p + i, b + i, m, s) : adj_grouped<2, false, CROSS>(p + i, b + i, m, s);
    else
      rc = bf ? adj_grouped<1, true, CROSS>(p + i, b + i, m, s) : adj_grouped<1, false, CROSS>(p + i, b + i, m, s);
    EX_TRY(rc);
  }
  return EXPENC_OK;
}

int split_adjoint_grouped(const EncPlan *const *p, const EncBuffers *const *b, int n, hipStream_t s) {
  // groups whose pixel blocks stay inside image rows and the others take
  // kernel variants of their own
  std::vector<const EncPlan *> pv[2];
  std::vector<const EncBuffers *> bv[2];
  for (int g = 0; g < n; ++g) {
    if (!split_groupable(*p[0], *p[g])) return fail(EXPENC_EINVAL, "plans of a grouped launch differ in shape");
    pv[adj_cross(*p[g])].push_back(p[g]);
    bv[adj_cross(*p[g])].push_back(b[g]);
  }
  EX_TRY(adj_grouped_class<false>(pv[0].data(), bv[0].data(), (int)pv[0].size(), s));
  return adj_grouped_class<true>(pv[1].data(), bv[1].data(), (int)pv[1].size(), s);
}

void split_adjoint_sh_launch(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  const bool bf = p.prec == EXPENC_BF16_SPLIT;
  if (adj_cross(p))
    bf ? adj_split_sh<true, true>(p, b, s) : adj_split_sh<false, true>(p, b, s);
  else
    bf ? adj_split_sh<true, false>(p, b, s) : adj_split_sh<false, false>(p, b, s);
}

}  // namespace expenc
