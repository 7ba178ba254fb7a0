// The split adjoint contraction with the solid-harmonic basis in
// polynomial form (the polynomial forms and the split arithmetic are
// described in split.hip).  It sits in a translation unit of its own so that
// it can be built with its own code-generation options.
#include "internal.h"
#include "split_dev.h"

namespace expenc {

template <int GW, bool BF>
__global__ __launch_bounds__(256) void k_adj_split_sh(const double *__restrict__ pmono, const float *__restrict__ dpa,
                                                      const double *__restrict__ dwq, const u32x4 *__restrict__ ys,
                                                      float *__restrict__ part, int Rp, int64_t Tp, int NCP, int chunk,
                                                      int nsplit, int nxq, int nx, int ny, double dx, double dy,
                                                      const float2 *__restrict__ sq) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int hl = lane >> 5, jl = lane & 31;
  int split, rb;
  if (!(sq ? split_tile_rows(Rp / 256, nsplit, &split, &rb) : split_tile(Rp / 256, nsplit, &split, &rb))) return;
  const int64_t row0 = (int64_t)rb * 256 + wave * 64;
  const int g0 = blockIdx.y * GW;
  const int NGP = NCP / 16;
  const int pz = blockIdx.z;  // problem
  pmono += pz * Tp * 12;
  dpa += pz * Tp * 16;
  dwq += (int64_t)pz * Rp;
  ys += pz * Tp * NGP * 16;
  // this lane's pixel in each 32-row block, and its B operand of the
  // increment product: the monomial (or dw0) of term 2J + hl
  double xg[2], yg[2], wg[2];
  float bm[2][6];
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const int rq = (int)(row0 + 32 * blk + jl);
    const double x = (rq % nxq - 0.5 * nx) * dx, y = (rq / nxq - 0.5 * ny) * dy, w = dwq[rq];
    xg[blk] = x;
    yg[blk] = y;
    wg[blk] = w;
    // terms 0..11: 1, x, y, x^2, xy, y^2, x^3, x^2 y, x y^2, y^3, dw0, anchor
    bm[blk][0] = (float)(hl ? x : 1.0);
    bm[blk][1] = (float)(hl ? x * x : y);
    bm[blk][2] = (float)(hl ? y * y : x * y);
    bm[blk][3] = (float)(hl ? x * x * y : x * x * x);
    bm[blk][4] = (float)(hl ? y * y * y : x * y * y);
    bm[blk][5] = (float)w;  // lanes 32..63 replace it by the anchor per step
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
    const float av[6] = {a03.x, a03.y, a03.z, a03.w, a47.x, a47.y};
    // anchor: FP64 phase of the tile's centre sample at this lane's pixels,
    // reduced to turns; it enters the product as term 11 (A = 1)
    const double *pc = pmono + (t + 16) * 12;
    f32x16 ph[2];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const double y = yg[blk], x = xg[blk];
      const double a0 = pc[0] + y * (pc[2] + y * (pc[5] + y * pc[9]));
      const double a1 = pc[1] + y * (pc[4] + y * pc[8]);
      const double a2 = pc[3] + y * pc[7];
      const double pa = fma(pc[10], wg[blk], a0 + x * (a1 + x * (a2 + x * pc[6])));
      const float anc = (float)__builtin_amdgcn_fract(pa);
      const float b5 = hl ? anc : bm[blk][5];
#pragma unroll
      for (int v = 0; v < 16; ++v) ph[blk][v] = 0.f;
#pragma unroll
      for (int J = 0; J < 5; ++J) ph[blk] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[J], bm[blk][J], ph[blk], 0, 0, 0);
      ph[blk] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[5], b5, ph[blk], 0, 0, 0);
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
          split_pair<BF>(c2[0], c2[1], w[0][m], w[1][m]);
          split_pair<BF>(s2[0], s2[1], w[2][m], w[3][m]);
        }
        const u32x4 A[4] = {u32x4{w[0][0], w[0][1], w[0][2], w[0][3]}, u32x4{w[1][0], w[1][1], w[1][2], w[1][3]},
                            u32x4{w[2][0], w[2][1], w[2][2], w[2][3]}, u32x4{w[3][0], w[3][1], w[3][2], w[3][3]}};
#pragma unroll
        for (int g = 0; g < GW; ++g) acc[blk][g] = step6<BF>(A, b[g], acc[blk][g]);
      }
    }
  }
  adj_epilogue<GW>(part, sq, Rp, NCP, nsplit, split, pz, row0, g0, lane, acc);
}

template <bool BF>
static void adj_split_sh(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  dim3 grid(split_grid((int64_t)p.Rp / 256 * p.adj_split), (unsigned)p.NGY, (unsigned)p.P);
  float *part = reinterpret_cast<float *>(b.part);
  const u32x4 *ys = reinterpret_cast<const u32x4 *>(b.ys);
  const float2 *sm = p.comb ? b.sq : nullptr;
  if (p.GW == 2)
    k_adj_split_sh<2, BF><<<grid, 256, 0, s>>>(b.pmono, b.dpa, b.dwq, ys, part, p.Rp, p.Tp, p.NCP, p.adj_chunk,
                                               p.adj_split, p.nxq, p.nx, p.ny, p.dx, p.dy, sm);
  else
    k_adj_split_sh<1, BF><<<grid, 256, 0, s>>>(b.pmono, b.dpa, b.dwq, ys, part, p.Rp, p.Tp, p.NCP, p.adj_chunk,
                                               p.adj_split, p.nxq, p.nx, p.ny, p.dx, p.dy, sm);
}

void split_adjoint_sh_launch(const EncPlan &p, const EncBuffers &b, hipStream_t s) {
  if (p.prec == EXPENC_BF16_SPLIT)
    adj_split_sh<true>(p, b, s);
  else
    adj_split_sh<false>(p, b, s);
}

}  // namespace expenc
