// Reductions, small vector kernels and solver building blocks shared by the
// entry points (implemented in api.hip and fista.hip).
#pragma once

#include "internal.h"

namespace expenc {

constexpr int kRedBlocks = 256;  // blocks of the first reduction stage

// out[b] = scale * Re sum_i conj(a[b*stride+i]) b[b*stride+i], i < n  (FP64, fixed order)
int reduce_dot(const float2 *a, const float2 *b, int64_t n, int64_t stride, int B, double scale, double *part,
               double *out, hipStream_t s);
// out[b] = scale * max_i |a[b*stride+i]|
int reduce_maxabs(const float2 *a, int64_t n, int64_t stride, int B, double scale, double *part, double *out,
                  hipStream_t s);
// out[b] = scale * sum_k part[b*nblk+k]
int reduce_sum_parts(const double *part, int nblk, int B, double scale, double *out, hipStream_t s);
int scale_rsqrt(float2 *v, int64_t n, int64_t stride, int B, const double *nrm2, hipStream_t s);
int copy_f2(const float2 *in, float2 *out, int64_t n, hipStream_t s);

// u = A^H A v with the batch-1 plan p (v, u: [R]).
int normal_apply(const EncPlan &p, const expenc_op *op, const EncBuffers &eb, const float2 *v, float2 *u,
                 hipStream_t s);
size_t lipschitz_bytes(const EncPlan &p1);
int lipschitz_run(const EncPlan &p1, const expenc_op *op, const EncBuffers &eb, int n_iter, const float *v0,
                  float2 *vec, float2 *tmp, double *dpart, double *dsc, double *L_out, hipStream_t s);

size_t fista_bytes(const expenc_op *op, int32_t batch, int32_t precision, int32_t nx_pad, int32_t ny_pad);
size_t cg_bytes(const expenc_op *op, int32_t batch, int32_t precision);
size_t grad_bytes(const expenc_op *op, int32_t precision);

}  // namespace expenc
