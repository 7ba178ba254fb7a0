// expenc_forward_static: the forward operator of eq. 1 (y = A_exp x) for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops).  Its scratch (tables, packed operands, split-K
// partial sums) lives in a file-scope device array instead of a caller
// workspace.  The array is per device: at the first call on a device (that
// device current) its address is looked up with hipGetSymbolAddress and kept;
// host code uses only that address, never the array's name.  Every call on
// one device shares the array, so calls that overlap on one device race.
// The kernels write every scratch element they later read (tables, operands,
// partial sums of every split), so nothing has to start at zero.
#include <mutex>

#include "internal.h"

namespace expenc {

constexpr size_t kStaticScratchBytes = size_t(128) << 20;  // 128 MiB per device
constexpr int kMaxStaticDevices = 64;

static __device__ __align__(256) char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxStaticDevices] = {};

static int scratch_for_current_device(void **out) {
  int dev = 0;
  EX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxStaticDevices) return fail(EXPENC_EUNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    EX_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(EXPENC_EHIP, "no device address for the static scratch");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return EXPENC_OK;
}

}  // namespace expenc

using namespace expenc;

extern "C" int expenc_forward_static(const expenc_op *op, int32_t batch, int32_t precision, const float *x, float *y,
                                     void *stream) {
  EncPlan p;
  EX_TRY(plan_forward_within(op, batch, precision, kStaticScratchBytes, &p));
  if (!x || !y) return fail(EXPENC_EINVAL, "x or y is NULL");
  void *base = nullptr;
  EX_TRY(scratch_for_current_device(&base));
  Arena a{static_cast<char *>(base), kStaticScratchBytes, 0};
  EncBuffers eb;
  if (carve_enc(p, a, &eb) != EXPENC_OK)
    return fail(EXPENC_EWORKSPACE, "forward scratch of %zu bytes exceeds the static %zu", a.used,
                kStaticScratchBytes);
  hipStream_t s = (hipStream_t)stream;
  EX_TRY(enc_prepare(p, op, eb, s));
  EX_TRY(enc_build_z(p, op->smaps, reinterpret_cast<const float2 *>(x), p.R, p.nx, eb, s));
  EX_TRY(enc_forward_partials(p, eb, s, false));
  return enc_forward_reduce_out(p, eb, reinterpret_cast<float2 *>(y), s);
}
