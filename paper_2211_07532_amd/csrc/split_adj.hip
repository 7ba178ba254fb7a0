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
// column groups).  ROWS: every 32-pixel block lies in one image row and the
// increment product has rank 6 (the row layout of dpa, see k_prep_dpa).
template <int GW, bool BF, bool ROWS>
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
  // this lane's pixel in each 32-row block, and its B operand of the
  // increment product: the monomial (or dw0) of term 2J + hl
  constexpr int NJ = ROWS ? 3 : 6;  // term pairs
  float bm[2][NJ];
  float yb[2];  // ROWS: the block's image row y
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const int rq = (int)(row0 + 32 * blk + jl);
    const double x = (rq % nxq - 0.5 * nx) * dx, y = (rq / nxq - 0.5 * ny) * dy, w = dwq[rq];
    yb[blk] = (float)y;
    if constexpr (ROWS) {
      // terms 0..5: 1, x, x^2, x^3, dw0, anchor
      bm[blk][0] = (float)(hl ? x : 1.0);
      bm[blk][1] = (float)(hl ? x * x * x : x * x);
    } else {
      // terms 0..11: 1, x, y, x^2, xy, y^2, x^3, x^2 y, x y^2, y^3, dw0, anchor
      bm[blk][0] = (float)(hl ? x : 1.0);
      bm[blk][1] = (float)(hl ? x * x : y);
      bm[blk][2] = (float)(hl ? y * y : x * y);
      bm[blk][3] = (float)(hl ? x * x * y : x * x * x);
      bm[blk][4] = (float)(hl ? y * y * y : x * y * y);
    }
    bm[blk][NJ - 1] = (float)w;  // lanes 32..63 replace it by the anchor per step
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
    // A operand of the increment product (this lane's sample, terms 2J + hl)
    const float4 *ap = reinterpret_cast<const float4 *>(dpa + ((t >> 5) * 64 + lane) * 8);
    const float4 a03 = ap[0], a47 = ap[1];
    float av[2][NJ];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      if constexpr (ROWS) {
        // C_hl and C_{2+hl} at the block's row, then d10 or 1
        const float y = yb[blk];
        av[blk][0] = fmaf(y, fmaf(y, fmaf(y, a03.w, a03.z), a03.y), a03.x);
        av[blk][1] = fmaf(y, a47.y, a47.x);
        av[blk][2] = a47.z;
      } else {
        const float v[6] = {a03.x, a03.y, a03.z, a03.w, a47.x, a47.y};
#pragma unroll
        for (int J = 0; J < 6; ++J) av[blk][J] = v[J];
      }
    }
    // anchor: FP64 phase of the tile's centre sample at this lane's pixels
    // in turns (from the table); it enters the product as term 11 (A = 1)
    const float *ap2 = anc + (t >> 5) * Rp + row0 + jl;
    const float an[2] = {ap2[0], ap2[32]};
    f32x16 ph[2];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const float bl = hl ? an[blk] : bm[blk][NJ - 1];
#pragma unroll
      for (int v = 0; v < 16; ++v) ph[blk][v] = 0.f;
#pragma unroll
      for (int J = 0; J < NJ - 1; ++J)
        ph[blk] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[blk][J], bm[blk][J], ph[blk], 0, 0, 0);
      ph[blk] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[blk][NJ - 1], bl, ph[blk], 0, 0, 0);
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
template <int GW, bool BF, bool ROWS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BF ? 3 : 1))) void k_adj_split_sh(AdjShArgs a) {
  adj_split_sh_body<GW, BF, ROWS>(a, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.y);
}

// Persistent form over several problem groups (the forward's grouped kernel
// in split.hip describes the numbering and why the XCD mapping holds).
template <int GW, bool BF, bool ROWS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BF ? 3 : 1))) void k_adj_split_sh_grouped(
    GroupedLaunch<AdjShArgs> G) {
  for (int64_t t = blockIdx.x; t < G.off[G.ng]; t += gridDim.x) {
    int g = 0;
    while (g + 1 < G.ng && t >= G.off[g + 1]) ++g;
    const int64_t l = t - G.off[g];
    const int gx = G.gx[g], gy = G.gy[g];
    const int64_t q = l / gx;
    adj_split_sh_body<GW, BF, ROWS>(G.a[g], (int)(l - q * gx), (int)(q % gy), (int)(q / gy), gy);
  }
}

static AdjShArgs adj_sh_args(const EncPlan &p, const EncBuffers &b) {
  return AdjShArgs{b.anc, b.dpa, b.dwq, reinterpret_cast<const u32x4 *>(b.ys), reinterpret_cast<float *>(b.part),
                   p.comb ? b.sq : nullptr, p.Tp, p.Rp, p.NCP, p.adj_chunk, p.adj_split, p.nxq, p.nx, p.ny, p.dx,
                   p.dy, bf16_masks()};
}

template <bool BF, bool ROWS>
static void adj_split_sh(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid((int64_t)p.Rp / 256 * p.adj_split), (unsigned)p.NGY, (unsigned)p.P);
  const AdjShArgs a = adj_sh_args(p, b);
  if (p.GW == 2)
    k_adj_split_sh<2, BF, ROWS><<<grid, 256, 0, s>>>(a);
  else
    k_adj_split_sh<1, BF, ROWS><<<grid, 256, 0, s>>>(a);
}

template <int GW, bool BF, bool ROWS>
static int adj_grouped(const EncPlan *const *p, const EncBuffers *const *b, int n, hipStream_t s) {
  const void *kern = reinterpret_cast<const void *>(&k_adj_split_sh_grouped<GW, BF, ROWS>);
  GroupedLaunch<AdjShArgs> G{};
  G.ng = n;
  G.off[0] = 0;
  for (int g = 0; g < n; ++g) {
    G.a[g] = adj_sh_args(*p[g], *b[g]);
    G.gx[g] = (int)split_grid((int64_t)p[g]->Rp / 256 * p[g]->adj_split);
    G.gy[g] = p[g]->NGY;
    G.off[g + 1] = G.off[g] + (int64_t)G.gx[g] * G.gy[g] * p[g]->P;
  }
  unsigned grid = 0;
  EX_TRY(persistent_grid(kern, G.off[n], &grid));
  k_adj_split_sh_grouped<GW, BF, ROWS><<<grid, 256, 0, s>>>(G);
  EX_LAUNCHED("grouped adjoint contraction");
  return EXPENC_OK;
}

// Grouped adjoint launches (chunks of kMaxGrouped) of plans that share the
// row layout flag.
static int adj_grouped_class(const EncPlan *const *p, const EncBuffers *const *b, int n, hipStream_t s) {
  for (int i = 0; i < n; i += kMaxGrouped) {
    const int m = std::min(kMaxGrouped, n - i);
    const bool bf = p[i]->prec == EXPENC_BF16_SPLIT, rows = p[i]->adj_rows;
    int rc;
    if (p[i]->GW == 2) {
      if (rows) rc = bf ? adj_grouped<2, true, true>(p + i, b + i, m, s) : adj_grouped<2, false, true>(p + i, b + i, m, s);
      else rc = bf ? adj_grouped<2, true, false>(p + i, b + i, m, s) : adj_grouped<2, false, false>(p + i, b + i, m, s);
    } else {
      if (rows) rc = bf ? adj_grouped<1, true, true>(p + i, b + i, m, s) : adj_grouped<1, false, true>(p + i, b + i, m, s);
      else rc = bf ? adj_grouped<1, true, false>(p + i, b + i, m, s) : adj_grouped<1, false, false>(p + i, b + i, m, s);
    }
    EX_TRY(rc);
  }
  return EXPENC_OK;
}

int split_adjoint_grouped(const EncPlan *const *pall, const EncBuffers *const *ball, int nall, hipStream_t s) {
  // the row-layout groups and the others take kernels of their own
  std::vector<const EncPlan *> pv[2];
  std::vector<const EncBuffers *> bv[2];
  for (int g = 0; g < nall; ++g) {
    if (!split_groupable(*pall[0], *pall[g])) return fail(EXPENC_EINVAL, "plans of a grouped launch differ in shape");
    pv[pall[g]->adj_rows].push_back(pall[g]);
    bv[pall[g]->adj_rows].push_back(ball[g]);
  }
  for (int cls = 0; cls < 2; ++cls) EX_TRY(adj_grouped_class(pv[cls].data(), bv[cls].data(), (int)pv[cls].size(), s));
  return EXPENC_OK;
}

void split_adjoint_sh_launch(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  const bool bf = p.prec == EXPENC_BF16_SPLIT;
  if (p.adj_rows)
    bf ? adj_split_sh<true, true>(p, b, s) : adj_split_sh<false, true>(p, b, s);
  else
    bf ? adj_split_sh<true, false>(p, b, s) : adj_split_sh<false, false>(p, b, s);
}

}  // namespace expenc
