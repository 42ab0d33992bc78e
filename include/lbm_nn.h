/*
 * C-ABI of the convolutional surrogate kernels in liblbm.so.
 *
 * The surrogate is a 3-D encoder-decoder that maps a pore-space mask to the
 * steady single-phase velocity and pressure fields; its prediction
 * warm-starts the solver (f = f^eq(rho_pred, u_pred - a/2), formed on the
 * device by lbm_nn_warm_fields) when computing permeability from Darcy's
 * law, the workflow the paper runs with a cold start (Sec. 3.4.1, 50,000
 * steps to steady state).  These are its training and inference kernels.
 *
 * Conventions
 *   - Activations are FP32 device arrays [C][D][H][W] (W fastest).
 *   - Every convolution is 3x3x3, stride 1, with periodic wrap (the pore
 *     geometries are periodic), computed on MFMA matrix cores: BF16 inputs
 *     with FP32 accumulation (prec = LBM_NN_BF16) or FP32 inputs
 *     (prec = LBM_NN_FP32).
 *   - Weights are FP32 [C_out][C_in][27] with tap t = 9 dz + 3 dy + dx
 *     (dz, dy, dx in 0..2, offset -1); they are packed once per update with
 *     lbm_nn_pack before use.
 *   - All work is enqueued on the given hipStream_t (asynchronous); pointers
 *     are device pointers owned by the caller.  Returns 0 or LBM_ERR_ARG /
 *     LBM_ERR_HIP (include/lbm.h).
 */
#ifndef PAPER_2506_17713_LBM_NN_H
#define PAPER_2506_17713_LBM_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LBM_NN_BF16 = 0, LBM_NN_FP32 = 1 };

/* Number of 32-bit words of the packed weights of a (c_out, c_in) layer. */
size_t lbm_nn_packed_words(int c_out, int c_in);

/* Pack W [c_out][c_in][27] for lbm_nn_conv.  transpose = 1 packs the weights
 * of the data-gradient convolution (channels swapped, taps mirrored), so that
 * lbm_nn_conv(dY, packed_T) gives dL/dX. */
int lbm_nn_pack(const float* W, int c_out, int c_in, int transpose, int prec, uint32_t* packed, void* stream);

/* Y[co] = act(bias[co] + sum_ci sum_t W[co][ci][t] X[ci][p + off(t)]) + skip[co]
 * act = max(0, .) when relu != 0; bias and skip may be NULL.  work: device
 * buffer of lbm_nn_conv_work_bytes() bytes, which receives X converted to
 * BF16 with channels innermost (BF16 only; FP32 takes NULL).
 * Errors: LBM_ERR_ARG (bad sizes, P max(c_in, c_out) >= 2^31, no work for BF16), LBM_ERR_HIP. */
size_t lbm_nn_conv_work_bytes(int c_in, int D, int H, int W, int prec);
int lbm_nn_conv(const float* X, int c_in, const uint32_t* packed, const float* bias, const float* skip,
                float* Y, int c_out, int D, int H, int W, int relu, int prec, void* work, void* stream);

/* lbm_nn_conv in BF16 for chains of convolutions (inference): the input is
 * either X (FP32, converted into work as lbm_nn_conv does) or xb, already in
 * the work layout (BF16 [P][c_in padded to 16], channels innermost: the
 * yb_next of the producing call); the output goes to Y (FP32) and / or
 * yb_next, the same values in the work layout of a c_out-channel input
 * (lbm_nn_conv_work_bytes(c_out, D, H, W, LBM_NN_BF16) bytes, padding
 * channels zero), so the next convolution skips the conversion and no FP32
 * tensor needs to exist between two convolutions.  X or xb, and Y or
 * yb_next, must be given; work is needed only with X.
 * Errors: LBM_ERR_ARG, LBM_ERR_HIP. */
int lbm_nn_conv_x(const float* X, const void* xb, int c_in, const uint32_t* packed, const float* bias,
                  const float* skip, float* Y, void* yb_next, int c_out, int D, int H, int W, int relu, void* work,
                  void* stream);

/* dW[co][ci][t] = sum_p dY[co][p] X[ci][p + off(t)] (overwrites dW).
 * partial: device scratch of lbm_nn_wgrad_partial_words(c_out, c_in, D, H, W) floats (tile partials, and
 * for BF16 the operands converted once). */
size_t lbm_nn_wgrad_partial_words(int c_out, int c_in, int D, int H, int W);
int lbm_nn_wgrad(const float* X, int c_in, const float* dY, int c_out, int D, int H, int W, float* dW,
                 float* partial, int prec, void* stream);

/* db[c] = sum_p dY[c][p] (overwrites), summed in double in a fixed order
 * (64 chunks per channel, then the chunk sums in order).  scratch: device
 * double[64 c].  Errors: LBM_ERR_ARG (c < 1, c > 65535, P < 1, NULL), LBM_ERR_HIP. */
int lbm_nn_bias_grad(const float* dY, int c, int64_t P, float* db, double* scratch, void* stream);
/* lbm_nn_bias_grad without the scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid allocation).  The chunk partials live
 * in a library-owned device array of 64 x 1024 doubles (512 KiB), one per
 * device, held until the process ends; the call itself allocates nothing.
 * Same result, bit for bit, as lbm_nn_bias_grad.  c must be <= 1024
 * (LBM_ERR_ARG otherwise).  All calls on one device share that array: calls
 * that overlap in time on one device (different streams or threads) race;
 * calls ordered on one stream do not.  Each call rewrites every partial it
 * reads, so nothing carries over between calls.
 * Errors: LBM_ERR_ARG (c < 1, c > 1024, P < 1, NULL), LBM_ERR_HIP. */
int lbm_nn_bias_grad_noalloc(const float* dY, int c, int64_t P, float* db, void* stream);
/* dY[i] *= (Y[i] > 0) */
int lbm_nn_relu_bwd(const float* Y, float* dY, int64_t n, void* stream);
/* y[i] += x[i] */
int lbm_nn_add(float* y, const float* x, int64_t n, void* stream);
/* 2x2x2 average pooling of X [c][D][H][W] into Y [c][D/2][H/2][W/2] and its
 * adjoint dX = dY / 8 spread over the children (accumulate: dX += ...). */
int lbm_nn_pool(const float* X, int c, int D, int H, int W, float* Y, void* stream);
int lbm_nn_pool_bwd(const float* dY, int c, int D, int H, int W, float* dX, int accumulate, void* stream);
/* Nearest 2x upsampling of X [c][D][H][W] into Y [c][2D][2H][2W] and its
 * adjoint dX = sum over the 8 children of dY. */
int lbm_nn_up(const float* X, int c, int D, int H, int W, float* Y, void* stream);
int lbm_nn_up_bwd(const float* dY, int c, int D, int H, int W, float* dX, void* stream);
/* The same pooling and upsampling written straight into the BF16 work layout
 * of a convolution's input ([output positions][c padded to 16], channels
 * innermost, padding zero; lbm_nn_conv_work_bytes(c, output D, H, W, LBM_NN_BF16)
 * bytes), for lbm_nn_conv_x(xb = ...) in an inference chain: bitwise the
 * values that lbm_nn_conv would convert from lbm_nn_pool / lbm_nn_up.
 * Errors: LBM_ERR_ARG, LBM_ERR_HIP. */
int lbm_nn_pool_x(const float* X, int c, int D, int H, int W, void* xb, void* stream);
int lbm_nn_up_x(const float* X, int c, int D, int H, int W, void* xb, void* stream);
/* Masked mean squared error over c channels: L = sum_{c,p} mask[p] (Y - T)^2 / (c sum_p mask[p]).
 * loss: device double[2 + 512]; loss[0] = L, loss[1] = sum_p mask[p], the rest
 * is scratch.  dY = dL/dY (may be NULL). */
int lbm_nn_mse(const float* Y, const float* T, const float* mask, int c, int64_t P, double* loss, float* dY,
               void* stream);
/* Symmetry transform of a field for training-set augmentation, written by the
 * callers that build training sets from solver output:
 *   Y[k](r) = sign[k] * X[src[k]](g^-1 r),  X, Y device float [c][D][H][W], c <= 8,
 * with g = periodic shift (host int shift[3] along D, H, W) o axis flips (host
 * int flip[3], nonzero = reverse that axis) o exchange of the D and H axes when
 * swap != 0 (needs D == H).  src/sign (host, c entries) permute and negate the
 * channels, as vector components require.  Y must not alias X.
 * Errors: LBM_ERR_ARG, LBM_ERR_HIP. */
int lbm_nn_augment(const float* X, float* Y, int c, int D, int H, int W, const int* shift, const int* flip,
                   int swap, const int* src, const float* sign, void* stream);
/* Initial fields of a warm-started flow solve from the network output, for
 * the callers that start lbm_reset from a prediction.  With Y device float
 * [4][P] (u_x, u_y, u_z, pressure channel), mask device float [P] (nonzero at
 * pore voxels), c host double[4] and <Y3> the pore mean of channel 3:
 *   pore voxels:  rho0[p] = 1 + c[3] (Y[3][p] - <Y3>),
 *                 u0[d][p] = c[d] Y[d][p] - (d == 0 ? shift_x : 0)
 *   solid voxels: rho0[p] = 1, u0[d][p] = 0
 * rho0 [P] and u0 [3][P] are device arrays of double (real_bytes 8) or float
 * (real_bytes 4), evaluated in double precision; the pore mean is summed in a
 * fixed order.  scratch: device double[2 + 512] (scratch[0] = sum over pores
 * of Y3, scratch[1] = pore count).  Errors: LBM_ERR_ARG, LBM_ERR_HIP. */
int lbm_nn_warm_fields(const float* Y, const float* mask, int64_t P, const double* c, double shift_x,
                       int real_bytes, void* rho0, void* u0, double* scratch, void* stream);
/* Adam update (Kingma & Ba) of n parameters at step t >= 1. */
int lbm_nn_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                float eps, int t, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_2506_17713_LBM_NN_H */
