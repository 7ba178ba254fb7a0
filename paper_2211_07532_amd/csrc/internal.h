// Internal helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>

#include <cstddef>
#include <cstdint>

#include "expenc.h"

namespace expenc {

void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define EX_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::expenc::fail(EXPENC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define EX_LAUNCHED(name)                                                              \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess)                                                              \
      return ::expenc::fail(EXPENC_EHIP, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
  } while (0)

#define EX_TRY(expr)              \
  do {                            \
    int s_ = (expr);              \
    if (s_ != EXPENC_OK) return s_; \
  } while (0)

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
inline int64_t ceil_div(int64_t v, int64_t m) { return (v + m - 1) / m; }

// Bump allocator over the caller's workspace (256-byte aligned slices).
struct Arena {
  char *base = nullptr;
  size_t size = 0;
  size_t used = 0;
  template <class T>
  T *take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return (base && used <= size) ? reinterpret_cast<T *>(base + off) : nullptr;
  }
  bool ok() const { return used <= size; }
};

// Status block at the start of every solver and coil workspace: one 32-bit
// word of flags that kernels set (atomicOr) when they see a failure, cleared
// at the start of each call, read back by expenc_solve_status.
constexpr size_t kStatusBytes = 256;
enum : unsigned {
  kStatusNonFinite = 1u,  // an iterate (or a factor) holds NaN or Inf
  kStatusDiverged = 2u    // the objective of eq. 1 rose above its value at x = 0
};
inline unsigned *take_status(Arena &a) { return a.take<unsigned>(kStatusBytes / sizeof(unsigned)); }
// status[0] = 0 (stream-ordered; a fill kernel, so it may also be captured)
int clear_status(unsigned *status, hipStream_t s);
// Flags a non-finite complex value (no-op for a NULL status).
__device__ inline void flag_nonfinite(unsigned *status, float2 v) {
  if (status && !(isfinite(v.x) && isfinite(v.y))) atomicOr(status, kStatusNonFinite);
}

// Geometry of one encoding contraction: a GEMM-shaped sum over pixels
// (forward) or samples (adjoint) with B*C complex columns, padded so that
// the kernels never test bounds inside their loops.
// XCD-aware decomposition of a split-K contraction launch.  Workgroup ids
// go to the eight XCDs in turn (id % 8), each XCD with its own L2.  Id b is
// remapped to b' = (b % 8) * Q + b / 8 (Q = ceil(N / 8), N = row blocks x
// splits) and b' is read split-major, so every XCD works through a
// contiguous range of reduction chunks and the slice of the streamed operand
// it needs stays in its L2.  The grid has 8Q >= N workgroups; the at most 7
// surplus ones return at once.
// (b: the workgroup's index in the launch's x dimension; a grouped launch
// passes the tile's index within its group.)
__device__ inline bool split_tile(int b, int nrb, int nsplit, int *split, int *rb) {
  const int n = nrb * nsplit;
  const int q = (n + 7) >> 3;
  const int bp = (b & 7) * q + (b >> 3);
  if (bp >= n) return false;
  *split = bp / nrb;
  *rb = bp - *split * nrb;
  return true;
}
// Variant for the coil-combining adjoint, whose epilogue also reads a table
// over its pixel rows (the coil sensitivities): XCD x takes the contiguous
// range [xQ, xQ + Q) of the row-major (row block, split) list, about one
// eighth of the row blocks with all of their splits, and walks it
// split-major.  Its slice of the row table then stays in its L2 across the
// splits, and the workgroups in flight on an XCD still share the chunks of a
// few splits of the streamed operand.  Same grid as split_tile.
__device__ inline bool split_tile_rows(int b, int nrb, int nsplit, int *split, int *rb) {
  const int n = nrb * nsplit;
  const int q = (n + 7) >> 3;
  const int j = b >> 3;
  const int lo = (b & 7) * q, hi = min(n, lo + q);
  if (lo + j >= hi) return false;
  // the range holds row block r of split s iff lo <= r * nsplit + s < hi
  int cum = 0;
  for (int s = 0; s < nsplit; ++s) {
    const int r0 = (lo - s + nsplit - 1) / nsplit, r1 = (hi - s + nsplit - 1) / nsplit;
    if (j < cum + r1 - r0) {
      *split = s;
      *rb = r0 + (j - cum);
      return true;
    }
    cum += r1 - r0;
  }
  return false;
}
inline unsigned split_grid(int64_t n) { return (unsigned)((n + 7) / 8 * 8); }

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Coil combination in the epilogue of the split adjoint contractions (single
// image per operator).  The adjoint of the multi-coil encoding ends in
// x(r) = sum_c conj(S_c(r)) u_c(r); a workgroup holds u_c(r) of its sample
// chunk for 256 pixel rows and its 16*GW coil columns in the MFMA output
// layout (lane: column 16g + l%16, part l/16 & 1 = Re/Im; element v of block
// a: row 32a + 8(v/4) + 4(l/32) + v%4).  sq holds S_c(r) in the same
// [row][column] layout (zero on padding rows and columns), so each load
// instruction reads two contiguous 128-byte row segments; a 32-row block's
// loads are all issued before their first use, so the epilogue waits for
// memory twice.  For each 32-row block a lane forms its share of conj(S) u (16 rows
// x Re/Im), then the 32 lanes of each half-wave sum those 32 values by
// recursive halving (xor 16, 8, 4, 2, 1: at each stage a lane keeps one half
// of its values and adds the partner's copy of that half), so that lane l
// ends with part l%2 of row element v = (l%32)/2, and the wave stores its 32
// rows as one contiguous 256-byte segment.
template <int GW>
__device__ inline void store_combined(float *__restrict__ dst, const float2 *__restrict__ sq, int NCP, int64_t row0,
                                      int g0, int lane, f32x16 (&acc)[2][GW]) {
  const int half = lane >> 5, c16 = lane & 15, im = (lane >> 4) & 1;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    float2 sv[2][16][GW];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = row0 + a * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
#pragma unroll
      for (int g = 0; g < GW; ++g) sv[a][v][g] = sq[row * NCP + (g0 + g) * 16 + c16];
    }
    __builtin_amdgcn_sched_barrier(0);
    float val[32];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float re = 0.f, ii = 0.f;
#pragma unroll
      for (int g = 0; g < GW; ++g) {
        const float u = acc[a][g][v];
        // conj(S) u: Re = Sr ur + Si ui, Im = Sr ui - Si ur
        re = fmaf(im ? sv[a][v][g].y : sv[a][v][g].x, u, re);
        ii = fmaf(im ? sv[a][v][g].x : -sv[a][v][g].y, u, ii);
      }
      val[2 * v] = re;
      val[2 * v + 1] = ii;
    }
#pragma unroll
    for (int o = 16, n = 32; o > 0; o >>= 1, n >>= 1) {
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int i = 0; i < n / 2; ++i) {
        const float keep = up ? val[i + n / 2] : val[i];
        const float send = up ? val[i] : val[i + n / 2];
        val[i] = keep + __shfl_xor(send, o);
      }
    }
    const int k = lane & 31, v = k >> 1;
    const int64_t row = row0 + a * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
    dst[row * 2 + (k & 1)] = val[0];
  }
}

// End of an adjoint contraction workgroup: with sq (single image, split
// forms) the coil-combined partial image of (problem pz, split, column block
// gy of ngy) goes to part as float2 [P][nsplit][NGY][Rp]; without, the
// per-coil accumulators go to [P][nsplit][Rp][NCP] complex.
template <int GW>
__device__ inline void adj_epilogue(float *part, const float2 *sq, int Rp, int NCP, int nsplit, int split, int pz,
                                    int gy, int ngy, int64_t row0, int g0, int lane, f32x16 (&acc)[2][GW]) {
  if (sq) {
    const int64_t slice = ((int64_t)pz * nsplit + split) * ngy + gy;
    store_combined<GW>(part + slice * Rp * 2, sq + (int64_t)pz * Rp * NCP, NCP, row0, g0, lane, acc);
    return;
  }
  const int half = lane >> 5, c16 = lane & 15, im = (lane >> 4) & 1;
  float *dst = part + ((int64_t)pz * nsplit + split) * Rp * NCP * 2;
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

// Real solid harmonics up to 3rd order at (x, y, z), in the basis order of
// expenc_sh_basis.
__device__ inline void sh_eval(double x, double y, double z, double (&v)[16]) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
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
}

struct EncPlan {
  int32_t nx = 0, ny = 0, R = 0, Rp = 0;  // pixels, padded to a multiple of 256
  int64_t T = 0, Tp = 0;                  // samples, padded to a multiple of 256
  int32_t C = 0, B = 0, NC = 0;           // coils, batch, columns = B*C
  int32_t G = 0, NCP = 0;                 // 16-column groups, padded columns = 16*GW*NGY
  int32_t GW = 0, NGY = 0;                // groups per wave, grid y = ceil(G/GW)
  int32_t L = 0, NT = 0;                  // basis terms, phase terms per entry (padded L+1)
  int32_t prec = 0;
  int32_t fwd_split = 1, fwd_chunk = 0;   // split-K over pixels
  int32_t adj_split = 1, adj_chunk = 0;   // split-K over samples
  // split forms with a single image (B == 1): the adjoint contraction
  // combines its coils in the epilogue and writes [adj_split][NGY][Rp]
  // partial images instead of [adj_split][Rp][NCP] per-coil partials
  bool comb = false;
  // split forms with the solid-harmonic basis: the adjoint contraction reads
  // its per-tile FP64 phase anchors from a table built at preparation
  // (EncBuffers::anc); off for forward-only plans
  bool adj_anc = false;
  bool has_dw0 = false;
  // Solid-harmonic basis given by grid geometry (EXPENC_BASIS_SH).  Split
  // forms with it lay pixels out row-padded: r' = y*nxq + x, nxq = nx rounded
  // up to 16, so that every 16-pixel step lies inside one image row.
  bool sh = false;
  int32_t nxq = 0;                        // padded row length of the pixel index
  double dx = 0, dy = 0, z0 = 0;          // pixel pitch and slice position (metres)
  // P independent problems of identical shape, each with its own operator
  // data packed contiguously (coef [P][T][L], time [P][T], dw0 [P][R],
  // smaps [P][C][R], basis [P][L][R], y [P][B][T][C]) and its own buffers;
  // every kernel takes the problem index as an extra grid dimension.
  int32_t P = 1;
  const double *z0s = nullptr;            // [P] slice positions (SH basis), or NULL: z0 for all
  // fp16 split form: every packed operand is multiplied by a power of two
  // chosen on the device from a bound on its magnitudes (the fp16 halves
  // overflow above 65504 and lose the lo half's precision below ~2^-3), and
  // the reductions divide it out.  nwmax: per-problem slots of the forward
  // contraction's per-wave output maxima (the residual operand's bound).
  bool scaled = false;
  int32_t nwmax = 0;
};

// Workgroups (per problem) of the magnitude pre-pass of the scaled form.
constexpr int kAmaxBlocks = 64;
// Longest reduction chunk of one workgroup: samples in the split adjoint
// contractions; pixels or samples in the FP32 contractions.
constexpr int32_t kSplitAdjChunkMax = 1024;
constexpr int32_t kF32ChunkMax = 2048;

int make_plan(const expenc_op *op, int32_t batch, int32_t precision, EncPlan *p, int32_t nprob = 1);

// Device buffers of one operator application, carved from the workspace.
struct EncBuffers {
  double *kap = nullptr;   // [Tp][NT] field coefficients in turns (+ time)
  double *bet = nullptr;   // [Rp][NT] basis values (+ dw0 in turns/s)
  float2 *zop = nullptr;   // forward operand: FP32 [Rp][NCP] or packed split
  float2 *yop = nullptr;   // adjoint operand: FP32 [Tp][NCP] or packed split
  float2 *part = nullptr;  // split-K partial sums (max of forward and adjoint)
  void *zs = nullptr;      // split forms: packed hi/lo forward operand [Rp/16][NCP/16][4][64] x 16 B
  void *ys = nullptr;      // split forms: packed hi/lo adjoint operand [Tp/16][NCP/16][4][64] x 16 B
  float *dbet = nullptr;   // split forms: [Rp][NT] bet minus its 16-row tile centre (FP32)
  float *dkap = nullptr;   // split forms: [Tp][NT] kap minus its 16-row tile centre (FP32)
  double *pmono = nullptr; // split + SH: [Tp][12] cubic-monomial phase coefficients (turns) and t
  float *dpa = nullptr;    // split + SH: [Tp/32][64][8] adjoint increment coefficients (FP32, per lane)
  double *dwq = nullptr;   // split + SH: [Rp] dw0/2pi in the row-padded pixel layout
  float *ddw = nullptr;    // split + SH: [Rp] dwq minus its 16-pixel tile centre (FP32)
  float *anc = nullptr;    // split + SH, adj_anc: [Tp/32][Rp] FP64 phase of each 32-sample tile's centre
                           // sample at each pixel, reduced to turns in [0, 1) (the adjoint's anchors)
  float2 *sq = nullptr;    // split, single image: [Rp][NCP] S_c(r) in the partial-sum layout (0 on padding)
  float *scl = nullptr;    // scaled form: [P][2] powers of two of the forward (0) and adjoint (1) operands
  float *amax = nullptr;   // scaled form: [3][P][kAmaxBlocks] per-workgroup bounds of pre-passes (operand,
                           // measured data, coil maps)
  float *wmax = nullptr;   // scaled form: [P][nwmax] per-wave max |partial sum| of the forward contraction
};

size_t enc_operand_bytes(const EncPlan &p);
// Forward-only plan whose buffers (carve_enc) fit in cap bytes: one adjoint
// split, and the forward split lowered from make_plan's as far as needed
// (not below the FP32 chunk cap).  EXPENC_EWORKSPACE if even that is larger.
int plan_forward_within(const expenc_op *op, int32_t batch, int32_t precision, size_t cap, EncPlan *p);
// Split-K partial-sum elements (float2) a plan needs.
size_t enc_part_elems(const EncPlan &p);
// Runs body(stream) captured into a cached HIP graph keyed by `key` (or
// eagerly when graphs are disabled), launched on s.
int run_captured(uint64_t key, hipStream_t s, const std::function<int(hipStream_t)> &body);
uint64_t hash_bytes(uint64_t h, const void *p, size_t n);

// Default anchor cadence of the split forms' anchored gradient.  The error of
// a split difference step scales with the form's product precision times
// ||z - z_ref||, so frequent anchors help, and an anchor formed in the split
// form costs no more than a difference iteration: the split-anchored modes
// refresh every 5 iterations (1.5 mm, 50 iterations: final image 2.8e-6
// fp16, 3.3e-6 bf16 against the FP64 solve, the same with the last anchor
// in FP32).  Anchors all in FP32 cost a
// full FP32 A and A^H each and keep the earlier cadences, which held the
// image within 1e-5 (4.9e-6 fp16 at 25, 6.9e-6 bf16 at 17).
inline int default_refine(int32_t precision, int32_t anchor) {
  if (anchor != EXPENC_ANCHOR_FP32) return 5;
  return precision == EXPENC_FP16_SPLIT ? 25 : 17;
}
// Whether the anchor of iteration k (of K) is formed in FP32.
inline bool anchor_in_fp32(int32_t anchor, int k, int K) {
  return k == 0 || anchor == EXPENC_ANCHOR_FP32 || (anchor == EXPENC_ANCHOR_ENDS && k == K - 1);
}
int set_tuning(const expenc_op *op, int32_t batch, int32_t precision, int32_t fwd_target, int32_t adj_target,
               int32_t col_groups);
uint64_t tuning_generation();
// Carves the buffers of plan p; the partial-sum buffer gets at least
// min_part float2 elements (so a second plan can share it).
int carve_enc(const EncPlan &p, Arena &a, EncBuffers *b, size_t min_part = 0);

// Kernel launchers (stream-ordered, no synchronisation).
int enc_prepare(const EncPlan &p, const expenc_op *op, const EncBuffers &b, hipStream_t s);
// Z[r][b*C+c] = S_c(r) x_b(r) from x [B][R] (x_stride elements between problems);
// for split precisions, pre-split and packed in the MFMA operand order.
// (x_pstride: elements between problems)
int enc_build_z(const EncPlan &p, const float *smaps, const float2 *x, int64_t x_stride,
                int32_t x_row_stride, const EncBuffers &b, hipStream_t s, const float2 *xsub = nullptr,
                int64_t x_pstride = 0);
// (timing = false: never records the profiling events of expenc_kernel_timing)
int enc_forward_partials(const EncPlan &p, const EncBuffers &b, hipStream_t s, bool timing = true);
// y[b][t][c] = sum_split partials (ABI layout)
int enc_forward_reduce_out(const EncPlan &p, const EncBuffers &b, float2 *y, hipStream_t s);
// Y operand from sign * y, y [B][T][C] (sign other than 1: FP32 plans only)
int enc_pack_y(const EncPlan &p, const float2 *y, const EncBuffers &b, hipStream_t s, float sign = 1.f);
int enc_adjoint_partials(const EncPlan &p, const EncBuffers &b, hipStream_t s);
// x_b(r) = alpha * sum_c conj(S_c(r)) sum_split partials (+ add_b(r)),
// written to x [B] with x_stride between problems and row stride
// x_row_stride (pixels); alpha = *alpha_dev (device FP64) or 1 if NULL.
// If base is given (same layout as x) it is added to the sum before scaling:
// x = add + alpha * (base + sum).
// alpha_dev, if given, holds one value per problem.  With pad_nx > 0, x is
// a pad_nx x pad_ny grid (>= nx x ny) whose pixels outside the encoded
// block are set to add (or 0).
int enc_adjoint_reduce_out(const EncPlan &p, const EncBuffers &b, const float *smaps, float2 *x,
                           int64_t x_stride, int32_t x_row_stride, const double *alpha_dev,
                           const float2 *add, hipStream_t s, const float2 *base = nullptr,
                           int64_t x_pstride = 0, int32_t pad_nx = 0, int32_t pad_ny = 0);
// Residual r = A z - y (y_meas [B][T][C], or NULL for r = A z) written
// straight into the adjoint operand.
int enc_forward_residual(const EncPlan &p, const EncBuffers &b, const float2 *y_meas, hipStream_t s);

// Split-precision kernels (split.hip).
int split_prepare(const EncPlan &p, const expenc_op *op, const EncBuffers &b, hipStream_t s);
// Polynomial phase tables of the solid-harmonic kind (pmono, dwq, ddw; dpa
// for the split forms) from kap (split.hip).
int sh_prepare(const EncPlan &p, const expenc_op *op, const EncBuffers &b, hipStream_t s);
void split_forward_launch(const EncPlan &p, const EncBuffers &b, hipStream_t s);
void split_adjoint_launch(const EncPlan &p, const EncBuffers &b, hipStream_t s);
// the polynomial (solid-harmonic) split adjoint, built in split_adj.hip
void split_adjoint_sh_launch(const EncPlan &p, const EncBuffers &b, hipStream_t s);

// One launch of a split contraction over several problem groups (plans of
// one shape class: solid-harmonic kind, same number format and column width
// GW).  Workgroup t of the launch runs workgroup (x, y, z) of group
// g's own grid, where off[g] <= t < off[g+1] and t - off[g] numbers that grid
// x fastest; the launch has one workgroup per t.
constexpr int kMaxGrouped = 8;
template <class Args>
struct GroupedLaunch {
  Args a[kMaxGrouped];
  int64_t off[kMaxGrouped + 1];
  int gx[kMaxGrouped], gy[kMaxGrouped];
  int ng;
};
// Whether two plans can share a grouped launch.
bool split_groupable(const EncPlan &a, const EncPlan &b);
// The forward (adjoint) contractions of n plans, in launches of at most
// kMaxGrouped groups each.
int split_forward_grouped(const EncPlan *const *p, const EncBuffers *const *b, int n, hipStream_t s);
int split_adjoint_grouped(const EncPlan *const *p, const EncBuffers *const *b, int n, hipStream_t s);
int split_build_z(const EncPlan &p, const float *smaps, const float2 *x, const float2 *xsub, int64_t x_stride,
                  int32_t x_row_stride, const EncBuffers &b, hipStream_t s, int64_t x_pstride);
int split_pack_y(const EncPlan &p, const float2 *y_abi, bool from_partials, const float2 *y_meas,
                 const EncBuffers &b, hipStream_t s);

// Per-kernel event timing of the contraction kernels (mode 0 off, 1 on, 2 read).
int kernel_timing(int32_t mode, double *out);

// Daubechies / Haar analysis low-pass filter, derived on the host.
int wavelet_filter(int32_t wavelet, double *h, int *taps);

}  // namespace expenc
