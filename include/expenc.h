/*
 * expenc.h -- C ABI of the MI355X (gfx950) expanded-encoding compressed-sensing
 * reconstruction library (libexpenc.so).
 *
 * The library solves eq. 1 of Varela-Mattatall, Dubovan et al. ("High-resolution
 * single-shot spiral diffusion-weighted imaging at 7T using expanded encoding
 * with compressed sensing"):
 *
 *     x_hat = argmin_x ||A_exp x - y||_2^2 + lambda ||W x||_1
 *
 * where A_exp is the expanded encoding operator.  The paper describes A_exp
 * (Introduction; Methods 2.1) as a signal model that includes a static B0 map,
 * the dynamic field measured by field probes and expanded in spherical
 * harmonics up to 2nd or 3rd order, and the coil sensitivities, for an
 * arbitrary trajectory.  Written out, for coil c, sample t and pixel r:
 *
 *     A[(t,c), r] = S_c(r) * exp(i * phi(t,r)),
 *     phi(t,r)    = sum_{l<L} k_l(t) * b_l(r) + dw0(r) * t.
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers owned by the caller; the library
 *     never allocates, frees or retains caller memory.  Scratch memory is a
 *     caller-provided workspace whose size comes from expenc_workspace_size.
 *   - Complex arrays are interleaved complex64 (re, im as two floats), the
 *     layout of torch.complex64.  Field/geometry arrays are float64.
 *   - Images are row-major [ny][nx] (x fastest); R = nx*ny.  k-space is
 *     sample-major [T][C] (coils fastest); a batch of B problems that share
 *     one operator is stacked in front: x [B][R], y [B][T][C].
 *   - Every call is stream-ordered and asynchronous on `stream` (a
 *     hipStream_t passed as void*; NULL is the default stream).  Argument
 *     validation happens on the host before any HIP call and is reported
 *     synchronously; launch failures are reported as EXPENC_EHIP.
 *   - On a non-OK status, expenc_last_error() returns a thread-local message.
 *   - Calls on distinct workspaces are independent, also when issued from
 *     several host threads at once (the library's graph cache, capture
 *     stream and fork streams are shared and locked; two first calls that
 *     both capture a graph capture one after the other); calls that share a
 *     workspace must be ordered by the caller (same stream).
 */
#ifndef EXPENC_H
#define EXPENC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  EXPENC_OK = 0,
  EXPENC_EINVAL = -1,        /* bad argument (null pointer, size, enum)          */
  EXPENC_EWORKSPACE = -2,    /* workspace missing or smaller than required       */
  EXPENC_EHIP = -3,          /* a HIP runtime call or kernel launch failed       */
  EXPENC_EUNSUPPORTED = -4,  /* valid but unsupported combination                */
  EXPENC_ENONFINITE = -5,    /* a solve produced NaN/Inf (expenc_solve_status)   */
  EXPENC_EDIVERGED = -6      /* a solve's objective diverged (expenc_solve_status) */
};

/* Arithmetic form of the encoding contraction.  The fp16 form multiplies
 * each operand it packs by a power of two chosen on the device from a bound
 * on the operand's magnitudes (one extra pre-pass launch for an image
 * operand or boundary data), and its reductions divide it out, so inputs of
 * any magnitude within the FP32 range keep the form's accuracy; the fp16
 * halves alone cover only ~2^-3 .. 65504 at full pair precision. */
enum {
  EXPENC_FP32 = 0,        /* FP32 phase tile x FP32 operand on FP32 MFMA              */
  EXPENC_BF16_SPLIT = 1,  /* both operands split hi+lo in bf16, 3 MFMA products      */
  EXPENC_FP16_SPLIT = 2   /* both operands split hi+lo in fp16, 3 MFMA products,
                             operands scaled by powers of two (above)               */
};

/* Wavelet families (periodised, orthonormal, separable 2D). */
enum {
  EXPENC_HAAR = 0,        /* h = [1, 1]/sqrt(2)                                    */
  EXPENC_DB4 = 1          /* 8-tap Daubechies, 4 vanishing moments, extremal phase */
};

/* What a workspace query is for. */
enum {
  EXPENC_WS_FORWARD = 0,
  EXPENC_WS_ADJOINT = 1,
  EXPENC_WS_FISTA = 2,
  EXPENC_WS_LIPSCHITZ = 3,
  EXPENC_WS_CG = 4,
  EXPENC_WS_FIELD_GRAD = 5
};

/* How the field basis b_l(r) is given. */
enum {
  EXPENC_BASIS_MAPS = 0,  /* `basis` holds b_l(r) for every pixel (any basis)            */
  EXPENC_BASIS_SH = 1     /* b_l are the real solid harmonics of expenc_sh_basis on the
                             grid (fov_x, fov_y, z0); `basis` is ignored and may be NULL.
                             The split forms then evaluate the phase as a cubic
                             polynomial in (x, y) (same values, fewer operations).      */
};

/*
 * One expanded-encoding operator (the entry formula above).  B problems may
 * share it (same field, same coils), in which case their coil data form the
 * columns of one contraction.
 */
typedef struct expenc_op {
  int32_t nx, ny;          /* image grid; R = nx*ny                                  */
  int32_t ncoils;          /* C >= 1                                                  */
  int32_t nbasis;          /* L in [0, 16]: number of field basis terms              */
  int64_t nsamples;        /* T >= 1                                                  */
  const double *basis;     /* [L][R] b_l(r) (basis units, e.g. m^degree); may be NULL if L == 0 */
  const double *coef;      /* [T][L] k_l(t) in rad per basis unit; may be NULL if L == 0 */
  const double *time;      /* [T] seconds from the first sample                      */
  const double *dw0;       /* [R] off-resonance in rad/s, or NULL for none           */
  const float *smaps;      /* [C][R] complex64 coil sensitivities S_c(r)             */
  int32_t basis_kind;      /* EXPENC_BASIS_MAPS or EXPENC_BASIS_SH                   */
  int32_t reserved;        /* must be 0                                              */
  double fov_x, fov_y, z0; /* EXPENC_BASIS_SH: grid geometry in metres (as expenc_sh_basis) */
} expenc_op;

/*
 * Real solid-harmonic field basis on the pixel grid (Introduction: field
 * dynamics expanded in spherical harmonics up to 2nd or 3rd order).
 * Writes basis[L][R] (float64): pixel centres x_i = (i - nx/2)*fov_x/nx,
 * y_j = (j - ny/2)*fov_y/ny, slice at z = z0 (metres).  Term order:
 * 1; x, y, z; xy, yz, 2z^2-x^2-y^2, xz, x^2-y^2; 3x^2y-y^3, xyz,
 * y(4z^2-x^2-y^2), z(2z^2-3x^2-3y^2), x(4z^2-x^2-y^2), z(x^2-y^2), x^3-3xy^2.
 * nbasis 9 = up to 2nd order, 16 = up to 3rd order.
 */
int expenc_sh_basis(int32_t nx, int32_t ny, double fov_x, double fov_y, double z0,
                    int32_t nbasis, double *basis, void *stream);

/* Bytes of workspace needed by the call `what` for this operator, batch and
 * precision (for EXPENC_WS_FISTA also the wavelet grid nx_pad x ny_pad; pass
 * 0 for the default).  Returns 0 on invalid arguments. */
size_t expenc_workspace_size(const expenc_op *op, int32_t batch, int32_t precision,
                             int32_t what, int32_t nx_pad, int32_t ny_pad);

/*
 * y = A_exp x (eq. 1's encoding operator).  x: [B][R] complex64,
 * y: [B][T][C] complex64 (overwritten).  precision: EXPENC_FP32 or a split form.
 */
int expenc_forward(const expenc_op *op, int32_t batch, int32_t precision,
                   const float *x, float *y, void *ws, size_t ws_bytes, void *stream);

/*
 * x = A_exp^H y, the adjoint (the paper's A^T in W A^T y, Methods 2.1):
 * x[b][r] = sum_c conj(S_c(r)) sum_t exp(-i phi(t,r)) y[b][t][c].
 * y: [B][T][C], x: [B][R] (overwritten).
 */
int expenc_adjoint(const expenc_op *op, int32_t batch, int32_t precision,
                   const float *y, float *x, void *ws, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * y = A_exp x as expenc_forward, with no workspace argument.  Its scratch is
 * a static device array of the library, 128 MiB per device, held from the
 * first call on a device until the process ends; the call itself allocates
 * nothing.  The forward's reduction split is lowered as far as needed to fit
 * (not below the FP32 form's chunk limit, so results may differ from
 * expenc_forward by summation order only); an operator whose forward does not
 * fit returns EXPENC_EWORKSPACE.  All calls on one device share the array:
 * calls that overlap on one device (different streams, other threads) race,
 * and must be ordered by the caller.  x: [B][R], y: [B][T][C] as in
 * expenc_forward.
 */
int expenc_forward_static(const expenc_op *op, int32_t batch, int32_t precision,
                          const float *x, float *y, void *stream);

/*
 * Lipschitz constant of the gradient of ||A x - y||^2: L = 2 lambda_max(A^H A),
 * by n_iter normalised power steps v <- A^H A v / ||A^H A v|| from the
 * caller's start vector v0 [R] complex64, then the Rayleigh quotient
 * 2 <v, A^H A v> / <v, v> (FP64 reductions), with the operators of the given
 * precision.  Writes L to *lipschitz_out (a DEVICE float64 scalar).
 */
int expenc_lipschitz(const expenc_op *op, int32_t precision, int32_t n_iter, const float *v0,
                     double *lipschitz_out, void *ws, size_t ws_bytes, void *stream);

/*
 * Forward 2D wavelet transform W (eq. 1's sparsifying transform), periodised
 * orthonormal separable, `levels` levels, Mallat layout (coarsest LL block at
 * the top-left).  One level on a periodic length-n line v:
 *   a[m] = sum_k h[k] v[(2m+k) mod n],  d[m] = sum_k g[k] v[(2m+k) mod n],
 *   g[k] = (-1)^k h[M-1-k];  rows first, then columns, on the current LL block.
 * x, w: [B][ny][nx] complex64; nx, ny multiples of 2^levels; w may equal x.
 */
int wavelet_fwd(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch,
                const float *x, float *w, void *stream);

/* Inverse (= adjoint) of wavelet_fwd; x may equal w. */
int wavelet_inv(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch,
                const float *w, float *x, void *stream);

/*
 * Proximal map of tau * sum_detail |w_i| (the l1 term of eq. 1 in the wavelet
 * domain, complex modulus): every detail coefficient becomes
 * w * max(0, 1 - tau/|w|); the coarsest LL block (ny>>levels x nx>>levels)
 * passes through.  w_in, w_out: [B][ny][nx]; w_out may equal w_in.
 */
int soft_threshold(int32_t nx, int32_t ny, int32_t levels, int32_t batch, const float *w_in,
                   float *w_out, float tau, void *stream);

/*
 * One proximal step of the l1 term of eq. 1 with the FISTA momentum (the
 * iteration's wavelet part, Methods 2.1): x = W^H S_tau(W v) and
 * z = x + beta (x - x_prev), for batch images of nx x ny (nx, ny multiples of
 * 2^levels; all arrays [B][ny][nx] complex64 on the device).  S_tau is the
 * soft_threshold above with tau[b] (device float64 [B]) for image b.  w
 * receives the thresholded coefficients (Mallat layout).  v is overwritten:
 * it and x carry the transform's intermediate low-pass blocks, so the call
 * needs no workspace; x_prev and z must be other buffers than v, w and x.
 * One launch per level and direction (rows and columns fused).
 */
int wavelet_prox(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch, float *v, float *w,
                 float *x, const float *x_prev, float *z, double beta, const double *tau, void *stream);

/*
 * Vector-Jacobian product of the soft-threshold (for differentiating through
 * the prox of eq. 1's l1 term).  With u = w/|w|, a = 1 - tau/|w|, b = tau/|w|,
 * the real-linear derivative of S_tau at |w| > tau is dw -> a dw + b u Re(conj(u) dw)
 * (symmetric), so grad_in = a g + b u Re(conj(u) g); grad_in = 0 where
 * |w| <= tau, and grad_in = g on the coarsest LL block.  Upstream g and the
 * result use the convention grad = dL/dRe + i dL/dIm.  All [B][ny][nx].
 */
int soft_threshold_vjp(int32_t nx, int32_t ny, int32_t levels, int32_t batch, const float *w_in, const float *g,
                       float *grad_in, float tau, void *stream);

/*
 * Field-parameter gradients of the encoding operator (differentiation of
 * A(theta) with theta = (k_l(t), dw0(r))).  Using dA/dk_l(t) = i b_l(r) A and
 * dA/d dw0(r) = i t A, for a real loss and upstream gradients in the
 * convention grad = dL/dRe + i dL/dIm:
 *   for y = A x with upstream g:     call with (w, kk) = (x, g);
 *   for x = A^H y with upstream gx:  call with (w, kk) = (gx, y);
 * then
 *   grad_coef[t][l] = -Im sum_c conj(kk[t][c]) [A (b_l w)](t, c)     (float64 [T][L])
 *   grad_dw0[r]     = -Im( w(r) conj([A^H (t kk)](r)) )              (float64 [R])
 * Either output may be NULL to skip it.  w: [R], kk: [T][C] complex64.
 * precision must be EXPENC_FP32.  The L basis-weighted products run as one
 * batched forward contraction (every phase tile is shared by the L terms).
 */
int expenc_field_grad(const expenc_op *op, int32_t precision, const float *w, const float *kk,
                      double *grad_coef, double *grad_dw0, void *ws, size_t ws_bytes, void *stream);

/*
 * out = a x + b y over n complex64 values, a and b real (FP32 arithmetic).
 * The linear steps of a FISTA iteration on eq. 1 (Methods 2.1) as a
 * separate call, for differentiating through unrolled iterations: the
 * residual A z - y (a = 1, b = -1), the gradient step z - (2/L) grad
 * (b = -2/L) and the momentum (1 + beta) x_k - beta x_{k-1}.  out may equal
 * x or y.
 */
int expenc_axpby(int64_t n, double a, const float *x, double b, const float *y, float *out, void *stream);

/* Options of fista_solve / cg_solve. */
typedef struct expenc_fista_opts {
  int32_t n_iter;          /* iterations K (Methods 2.1 uses 100)                    */
  int32_t precision;       /* EXPENC_FP32 / EXPENC_BF16_SPLIT / EXPENC_FP16_SPLIT    */
  int32_t wavelet;         /* EXPENC_HAAR / EXPENC_DB4                               */
  int32_t levels;          /* J >= 1                                                 */
  int32_t nx_pad, ny_pad;  /* wavelet grid (>= nx, ny, multiples of 2^J); 0 = round up */
  int32_t ista;            /* 1: momentum off (t_k = 1), monotone ISTA               */
  int32_t refine_every;    /* split forms: anchor cadence m (0 = the anchor mode's default) */
  int32_t n_power;         /* power steps when lipschitz <= 0 (in the solve's
                              precision when batch == 1, else FP32)                  */
  int32_t batch_launch;    /* fista_solve_batched: EXPENC_BATCH_FORKED or
                              EXPENC_BATCH_GROUPED (ignored by fista_solve)         */
  double lipschitz;        /* > 0: L to use; <= 0: estimate from power_v0            */
  double lambda;           /* >= 0: lambda to use; < 0: lambda_factor * max|A^H y|
                              (A^H y in FP32; it also gives the first iteration's
                              gradient)                                              */
  double lambda_factor;    /* used when lambda < 0 (e.g. 1e-3)                       */
  const float *power_v0;   /* device [R] complex64 power-iteration start (lipschitz <= 0) */
  double *objective;       /* device [B][n_iter] float64 objective trace, or NULL    */
  double *scalars;         /* device [2 + 2B] float64: L, tau(b=0), lambda[B], ..., or NULL */
  int32_t anchor;          /* split forms: precision of the anchors, EXPENC_ANCHOR_*  */
  int32_t reserved;        /* must be 0                                              */
} expenc_fista_opts;

/* Anchors of the split forms' gradient (expenc_fista_opts.anchor and
 * expenc_balanced_opts.anchor).  Every refine_every-th iteration, and the
 * last, recomputes the gradient at z_ref = z_k and later iterations add the
 * split operators' A^H A (z_k - z_ref) to it.
 *   SPLIT (default, 0; cadence 5): every anchor but the first in the
 *     iteration's split form;
 *   FP32 (cadence 25 fp16, 17 bf16): every anchor in FP32, so the solve
 *     converges to the FP32 operator's solution (the choice for problems
 *     whose solution is sensitive to the operator's last digits);
 *   ENDS (cadence 5): as SPLIT, with the last iteration's anchor in FP32.
 * The first iteration's gradient is FP32 in every mode (z_0 = 0, so it is
 * -A^H y, which the lambda rule also uses). */
enum { EXPENC_ANCHOR_SPLIT = 0, EXPENC_ANCHOR_FP32 = 1, EXPENC_ANCHOR_ENDS = 2 };

/*
 * CS reconstruction: FISTA on eq. 1 exactly as written (no 1/2 on the data
 * term), Methods 2.1.  With f(x) = ||A crop(x) - y||^2, L the Lipschitz
 * constant of grad f and tau = lambda/L, from x_0 = z_1 = 0, t_1 = 1:
 *   x_k     = W^H S_tau( W (z_k - grad f(z_k)/L) )
 *   t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
 *   z_{k+1} = x_k + (t_k - 1)/t_{k+1} (x_k - x_{k-1})
 * for exactly n_iter iterations.  The image lives on an nx_pad x ny_pad grid
 * whose top-left nx x ny block is encoded.  y: [B][T][C]; x: [B][ny][nx]
 * (crop of x_K, overwritten).  The iteration loop is captured once into a
 * HIP graph and replayed on `stream`; L, lambda and tau stay on the device.
 * Split precisions use an anchored gradient: the gradient at z_ref is
 * recomputed every refine_every iterations (in FP32 or the split form, see
 * EXPENC_ANCHOR_*) and the split operators only apply A^H A to z_k - z_ref.
 */
int fista_solve(const expenc_op *op, int32_t batch, const float *y, float *x,
                const expenc_fista_opts *opts, void *ws, size_t ws_bytes, void *stream);

/*
 * Many independent reconstructions in one call (the batch of slices and
 * diffusion directions of Methods 2.1 and Fig. 5, each solved as by
 * fista_solve).  ops[i], y[i] ([B][T][C] device) and x[i] ([B][ny][nx]
 * device, overwritten) describe problem i; B = batch for every problem.
 * Problems may differ in grid, samples, fields, coil maps and slice
 * position z0; those with equal (nx, ny, ncoils, nbasis, nsamples,
 * basis_kind, fov, presence of dw0) are solved together, one launch per pass
 * for the whole group, and all groups' iteration loops run inside one
 * captured HIP graph.  Every problem uses opts (K, precision, wavelet,
 * levels, lambda rule); each gets its own L, lambda and tau.  The wavelet
 * grid is each problem's rounded up to 2^levels (nx_pad, ny_pad must be 0);
 * objective and scalars must be NULL.  With lipschitz <= 0, power_v0 holds
 * at least max_i R_i complex values and problem i starts from its first
 * R_i.  The inputs are copied into the workspace at the start of the call.
 */
/* Launch pattern of a batched solve (expenc_fista_opts.batch_launch).
 * FORKED: every group runs its own iteration loop (one launch per pass for
 * the group's problems) on a stream forked inside the captured graph.
 * GROUPED: the groups advance in lock step and each split-difference
 * iteration's forward and adjoint contractions run as one launch each over
 * the (problem, row block, split) tiles of every group, one workgroup per tile
 * (split precisions with EXPENC_BASIS_SH and one column width for every
 * group, else EXPENC_EUNSUPPORTED).  Both give bit-identical results. */
enum { EXPENC_BATCH_FORKED = 0, EXPENC_BATCH_GROUPED = 1 };
size_t fista_batched_workspace_size(int32_t nprob, const expenc_op *ops, int32_t batch,
                                    const expenc_fista_opts *opts);
int fista_solve_batched(int32_t nprob, const expenc_op *ops, int32_t batch, const float *const *y,
                        float *const *x, const expenc_fista_opts *opts, void *ws, size_t ws_bytes,
                        void *stream);

/*
 * The paper's regulariser (Methods 2.1; Supporting Information S1):
 * undecimated wavelet transform, sigma/2 weights per level, balanced FISTA.
 *
 * swt_fwd / swt_inv: undecimated ("a trous") periodised separable 2D
 * transform with J = levels (1..8) on any nx x ny grid, and its adjoint.
 * Level j (step d = 2^j) applies the 1D filters
 * f(u)[i] = 2^-1/2 sum_k f[k] u[(i + d k) mod n] (low pass h, high pass g of
 * the chosen wavelet) along x and y; coefficients w [B][3J+1][ny][nx] hold
 * level j in bands 3j (high x, low y), 3j+1 (low x, high y), 3j+2 (high,
 * high) and the final low pass in band 3J.  With orthonormal filters this
 * is a tight frame: swt_inv(swt_fwd(x)) = x.  Workspace: for levels > 1,
 * expenc_swt_workspace_size() bytes of device scratch (NULL allowed at one
 * level).
 *
 * expenc_sigma_weights: weights lam [B][3J+1] (device, float64) from the
 * coefficients w (e.g. of A^H y): per image and level, the magnitudes |w| of
 * the level's three high-pass bands are counted in 256 equal bins over
 * [0, 4 mean|w|) (larger values are not counted); sigma = the centre of the
 * fullest bin (lowest bin on ties) and the level's weight is
 * scale * sigma / 2; the low-pass band gets 0.  counts [B][J][256]
 * (uint32, device) receives the histograms if not NULL.
 *
 * fista_balanced_solve: balanced FISTA (Methods 2.1) on the coefficients
 * alpha of the undecimated frame:
 *   F(alpha) = ||A W^H alpha - y||^2 + kappa/2 ||(I - W W^H) alpha||^2
 *              + sum_b lambda_b ||alpha_b||_1,
 * from alpha = 0 for exactly n_iter iterations with step 1/L,
 * L = L_A + kappa, L_A = 2 lambda_max(A^H A), gradient
 * 2 W A^H (A W^H beta - y) + kappa (beta - W W^H beta), per-band soft
 * threshold tau_b = lambda_b / L and the FISTA momentum; x = W^H alpha_K
 * ([B][ny][nx]).  Weights: opts->lambda ([B][3J+1] device) or, when NULL,
 * lambda_scale * sigma/2 from W A^H y (FP32 operators).  Split precisions use
 * the anchored gradient of fista_solve (the gradient recomputed every
 * refine_every-th and at the last iteration, see EXPENC_ANCHOR_*).  The loop is captured into a cached HIP graph.
 * scalars (device, optional): [L_A, kappa, L, lambda[B][3J+1], tau[B][3J+1]].
 */
typedef struct expenc_balanced_opts {
  int32_t n_iter;        /* iterations K                                           */
  int32_t precision;     /* EXPENC_FP32 / EXPENC_BF16_SPLIT / EXPENC_FP16_SPLIT    */
  int32_t wavelet;       /* EXPENC_HAAR / EXPENC_DB4                               */
  int32_t levels;        /* J in [1, 8] (the paper: 1)                             */
  int32_t refine_every;  /* split forms: anchor cadence (0 = the anchor mode's default) */
  int32_t n_power;       /* power steps when lipschitz <= 0 (solve's precision at
                            batch 1, else FP32)                                      */
  int32_t ista;          /* 1: momentum off                                        */
  int32_t anchor;        /* split forms: precision of the anchors, EXPENC_ANCHOR_*  */
  double lipschitz;      /* > 0: L_A to use; <= 0: power iteration from power_v0   */
  double kappa;          /* >= 0: balance weight; < 0: kappa = L_A                 */
  double lambda_scale;   /* factor on the sigma/2 rule (1 = the paper's)           */
  const float *power_v0; /* device [R] complex64 power-iteration start             */
  const double *lambda;  /* device [B][3J+1] weights, or NULL for the sigma/2 rule */
  double *scalars;       /* device output (see above), or NULL                     */
} expenc_balanced_opts;

size_t expenc_swt_workspace_size(int32_t nx, int32_t ny, int32_t levels, int32_t batch);
int swt_fwd(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch, const float *x, float *w,
            void *ws, size_t ws_bytes, void *stream);
int swt_inv(int32_t nx, int32_t ny, int32_t levels, int32_t wavelet, int32_t batch, const float *w, float *x,
            void *ws, size_t ws_bytes, void *stream);
size_t expenc_sigma_workspace_size(int32_t nx, int32_t ny, int32_t levels, int32_t batch);
int expenc_sigma_weights(int32_t nx, int32_t ny, int32_t levels, int32_t batch, const float *w, double scale,
                         double *lam, unsigned *counts, void *ws, size_t ws_bytes, void *stream);
size_t fista_balanced_workspace_size(const expenc_op *op, int32_t batch, const expenc_balanced_opts *opts);
int fista_balanced_solve(const expenc_op *op, int32_t batch, const float *y, float *x,
                         const expenc_balanced_opts *opts, void *ws, size_t ws_bytes, void *stream);

/*
 * Least-squares reconstruction by conjugate gradients on A^H A x = A^H y
 * from x = 0, stopped after n_iter iterations (Methods 2.1: early stopping
 * at 20 iterations as implicit regularisation).  Uses opts->n_iter and
 * opts->precision only.  y: [B][T][C]; x: [B][R].
 */
int cg_solve(const expenc_op *op, int32_t batch, const float *y, float *x,
             const expenc_fista_opts *opts, void *ws, size_t ws_bytes, void *stream);

/*
 * Receiver pre-whitening and coil compression (Methods 2.2.1: noise
 * correlation between receivers corrected by pre-whitening; k-space data
 * compressed to virtual coils to speed up the reconstruction).  C = ncoils in
 * [1, 64].  Workspace (device, caller-owned) from expenc_coil_workspace_size
 * (ncoils, nsamples); 0 for invalid sizes.
 *
 * expenc_prewhiten: psi [C][C] complex128 (interleaved FP64), the receivers'
 * Hermitian positive-definite noise covariance, factored as psi = L L^H
 * (Cholesky, FP64).  In place, every coil vector becomes L^{-1} v: the data
 * y [nsamples][C] (one vector per sample; pass B*T samples for a batch) and
 * the maps smaps [C][npix] (one vector per pixel).  Either may be skipped with
 * a zero size.  A psi that is not positive definite yields NaN outputs.
 *
 * expenc_coil_compress: G = Y^H Y over the nsamples rows of y [nsamples][C]
 * (FP64 sums), its eigenvectors V (columns, eigenvalues descending) by a
 * cyclic Jacobi method; with V_k = the first k = nvirtual columns:
 * y_out [nsamples][k] = Y V_k, smaps_out [k][npix] with
 * smaps_out[j] = sum_c V[c][j] smaps[c], so that y_out follows the encoding
 * model with the virtual maps.  eigvec ([C][C] complex128, row-major, column j
 * = eigenvector j) and eigval ([C] float64) receive the full decomposition if
 * not NULL; y_out may be NULL (maps only), npix may be 0 (data only).
 * Eigenvectors are unique up to a phase per column (and within degenerate
 * eigenvalues); the compressed subspace is what is determined.
 */
size_t expenc_coil_workspace_size(int32_t ncoils, int64_t nsamples);
int expenc_prewhiten(int32_t ncoils, const double *psi, int64_t nsamples, float *y, int32_t npix, float *smaps,
                     void *ws, size_t ws_bytes, void *stream);
int expenc_coil_compress(int32_t ncoils, int32_t nvirtual, int64_t nsamples, const float *y, int32_t npix,
                         const float *smaps, float *y_out, float *smaps_out, double *eigvec, double *eigval,
                         void *ws, size_t ws_bytes, void *stream);

/*
 * Launch-shape tuning (not part of the method).  The contraction kernels
 * split their reduction (pixels for A, samples for A^H) so that one launch
 * has about `target` workgroups (default 2048, or the EXPENC_TARGET_WG
 * environment variable).  expenc_set_tuning sets the forward and adjoint
 * targets for every later plan of op's geometry (nx, ny, ncoils, nbasis,
 * nsamples, basis_kind) at this batch and precision; 0 restores the default
 * for that direction, both 0 remove the entry.  A batched solve of P such
 * problems uses the same totals across its P problems.  Whatever the target,
 * one workgroup's reduction chunk is capped (1024 samples in the split
 * adjoints, 2048 pixels or samples in the FP32 contractions): the error of a
 * long sum on the matrix cores grows with its length, so a launch may have
 * more workgroups than its target.  Later calls plan
 * with the new targets (workspace sizes may change: query them again).
 * Process-wide and thread-safe; changing it while a call is being issued on
 * another thread leaves that call on either setting.
 */
int expenc_set_tuning(const expenc_op *op, int32_t batch, int32_t precision, int32_t fwd_target,
                      int32_t adj_target);

/*
 * The launch shape a call would use for nprob problems of op's geometry:
 * out[0] = forward split, out[1] = adjoint split, out[2] / out[3] = forward /
 * adjoint workgroups per launch, out[4] / out[5] = largest forward / adjoint
 * split (host array of 6).
 */
int expenc_plan_info(const expenc_op *op, int32_t batch, int32_t precision, int32_t nprob, int64_t *out);

/*
 * expenc_set_tuning with the contractions' column width as well:
 * col_groups = 16-column groups of the B*C coil columns that one wave
 * carries (1 or 2; 0 = the default, 2 when there are at least two groups).
 * Two share every phase tile between 32 columns; one halves the
 * accumulator registers and puts the groups in separate workgroups.  The
 * operand layouts follow the width, so later plans (and workspace sizes)
 * change with it.  Other properties as for expenc_set_tuning; all three
 * values 0 remove the entry.
 */
int expenc_set_launch_shape(const expenc_op *op, int32_t batch, int32_t precision, int32_t fwd_target,
                            int32_t adj_target, int32_t col_groups);

/*
 * expenc_plan_info writing min(n_out, 7) values: out[0..5] as there and
 * out[6] = the column width in 16-column groups per wave.
 */
int expenc_plan_info_ex(const expenc_op *op, int32_t batch, int32_t precision, int32_t nprob, int64_t *out,
                        int32_t n_out);

/*
 * Profiling aid (not part of the method): per-kernel timing of the two
 * contraction kernels with HIP events recorded on their launch stream around
 * every eager launch (launches captured into a graph are not timed).
 * mode 0: off and clear; 1: on and clear; 2: wait for the recorded events
 * and write out[0] = total forward-contraction ms, out[1] = forward launches,
 * out[2] = total adjoint-contraction ms, out[3] = adjoint launches (host array).
 */
int expenc_kernel_timing(int32_t mode, double *out);

/*
 * Outcome of the last call that used the workspace ws (the iterations of
 * eq. 1 by FISTA or CG, Methods 2.1; also the coil calls).  The solvers
 * (fista_solve, fista_solve_batched, fista_balanced_solve, cg_solve) and the
 * coil calls (expenc_prewhiten, expenc_coil_compress) keep a status word in
 * the first 256 bytes of their workspace: it is cleared at the start of each
 * call and set on the device when
 *   - an iterate x_k of a solve (any problem of a batched call), the
 *     Cholesky factor of expenc_prewhiten (a noise covariance that is not
 *     positive definite) or an eigenvalue of expenc_coil_compress holds NaN
 *     or Inf -> EXPENC_ENONFINITE;
 *   - with an objective trace requested (fista_solve), F(x_k) of eq. 1 rises
 *     above F(0) = ||y||^2, the value at the zero start image, at any
 *     iteration (e.g. an underestimated Lipschitz constant) -> EXPENC_EDIVERGED.
 * Non-finite takes precedence.  This call waits for `stream` (the stream of
 * the call that used ws) and returns EXPENC_OK, EXPENC_ENONFINITE or
 * EXPENC_EDIVERGED (with a message in expenc_last_error), or EXPENC_EINVAL /
 * EXPENC_EHIP.  ws is the caller's device workspace of that call.
 */
int expenc_solve_status(const void *ws, void *stream);

/* Thread-local text of the last non-OK status of this thread. */
const char *expenc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EXPENC_H */
