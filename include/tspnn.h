/*
 * tspnn.h -- companions of the spherical-grid projector on MI355X (gfx950):
 * the regulariser and optimiser of differentiable reconstruction, and the
 * layers of a small 3-D CNN on the (r, e, a) grid.  C ABI.
 *
 * Differentiable reconstruction minimises ||y - F rho||^2 + lambda TV(rho)
 * (TomoSphero Sec. 4.5, Eq. 6-7, with a total-variation regulariser) with the
 * Adam optimiser (Listing 7); F and F^T come from tsp.h.
 *
 * The CNN maps a few-iteration reconstruction to a warm start for iterative
 * reconstruction.  Its layers are 3x3x3 convolutions on the grid with
 * circular padding along azimuth (the grid is periodic there) and zero
 * padding along r and e.  Layers with 32 input and 32 output channels run on
 * BF16 MFMA with FP32 accumulation; the 1->32 input layer and the 32->1
 * output layer are tiny and run on FP32 vector ALUs.
 *
 * Layouts (all device pointers, contiguous, row-major):
 *   grid volume    [N][D0][D1][D2] with D0 = Nr, D1 = Ne, D2 = Na (azimuth,
 *                  circular), float32 for single-channel tensors;
 *   activations    [N][D0][D1][D2][32] bfloat16 (channels last);
 *   weights 32->32 [27][32 out][32 in] bfloat16, tap t = (dr+1)*9+(de+1)*3+(da+1)
 *                  for offsets (dr, de, da) in {-1,0,1}^3;
 *   weights 1->32  [27][32] float32;  weights 32->1  [27][32] float32;
 *   biases         float32.
 * A layer computes out[p][o] = b[o] + sum_t sum_i w[t][o][i] in[p + off(t)][i]
 * (cross-correlation), with in = 0 outside [0,D0) x [0,D1) and the azimuth
 * index taken modulo D2.
 *
 * Ownership / streams / errors: the caller owns every buffer; outputs are
 * overwritten; work is enqueued on `stream` (hipStream_t, NULL = default);
 * every call returns TSPNN_OK or an error code, with a message from
 * tspnn_last_error().  Reductions (weight and bias gradients, TV value) sum
 * per-block partials in a fixed order: results are bitwise reproducible.
 * The elementwise calls (Adam, bfloat16 conversions, axpy, scale) take
 * arrays of any length: they stride over grids of at most 2^23 workgroups
 * (one dispatch holds fewer than 2^32 work-items), a cap that the
 * environment variable TSP_MAX_BLOCKS lowers for tests.
 */
#ifndef TSPNN_H
#define TSPNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tspnn_status {
    TSPNN_OK = 0,
    TSPNN_E_INVALID = 1,     /* bad argument */
    TSPNN_E_HIP = 3,         /* HIP runtime failure */
    TSPNN_E_UNSUPPORTED = 5  /* shape the kernels do not handle (e.g. D2 % 32 != 0) */
} tspnn_status;

/* ------------------------------------------------------------------ vectors */
/*
 * Per-object vector steps of the solvers (gradient descent, power iteration,
 * the data term and the training loss).  Objects are B rows of n float32 on
 * the device.  Reductions run in a fixed order (blocks of 8192 elements,
 * then the blocks of each row in increasing order): the same inputs give the
 * same bits.  work: tspnn_vec_workspace(B, n) bytes of device memory.
 */
size_t tspnn_vec_workspace(int32_t B, int64_t n);

/*
 * Residual of the data term: diff[o][i] = f[o][i] - y[o][i] (diff may be NULL,
 * or alias f) and res[o] = sum_i diff[o][i]^2, written only for objects with
 * active[o] != 0 (every object when active is NULL; active: device int32 [B]).
 * 1 <= B <= 65535.
 */
tspnn_status tspnn_residual(const float *y, const float *f, int32_t B, int64_t n, float *diff,
                            float *res, const int32_t *active, void *work, void *stream);

/* out[o] = sum_i a[o][i] * b[o][i]  (1 <= B <= 65535) */
tspnn_status tspnn_dot(const float *a, const float *b, int32_t B, int64_t n, float *out,
                       void *work, void *stream);

/* x[o][i] += alpha * a[o][i] for objects with active[o] != 0 (all when NULL) */
tspnn_status tspnn_axpy(float *x, const float *a, float alpha, int32_t B, int64_t n,
                        const int32_t *active, void *stream);

/* dst[i] = alpha * src[i], i < n (dst may alias src) */
tspnn_status tspnn_scale(const float *src, float alpha, int64_t n, float *dst, void *stream);

/* ------------------------------------------------------------------ TV + Adam */

/* Workspace (bytes) that tspnn_tv needs for a batch of B volumes of V voxels. */
size_t tspnn_tv_workspace(int32_t B, int64_t V);

/*
 * Anisotropic smoothed total variation of B volumes [B][D0][D1][D2]:
 *   TV = sum_v sum_{d in r,e,a} sqrt((D_d rho)_v^2 + eps^2)
 * with forward differences; D_r, D_e have no term past the last index,
 * D_a is circular.  value: device float32 [B] (overwritten); grad: device
 * float32 like rho, receives dTV/drho (may be NULL); work: tspnn_tv_workspace
 * bytes of device memory.
 */
tspnn_status tspnn_tv(const float *rho, int32_t B, int32_t D0, int32_t D1, int32_t D2, float eps,
                      float *value, float *grad, void *work, void *stream);

/*
 * One Adam step on n parameters (PyTorch semantics, L2 weight decay added to
 * the gradient): g' = g + wd p; m = b1 m + (1-b1) g'; v = b2 v + (1-b2) g'^2;
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).  step t >= 1.
 * When p_bf16 is not NULL it also receives p rounded to bfloat16.
 */
tspnn_status tspnn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                        float beta1, float beta2, float eps, float weight_decay, int32_t step,
                        uint16_t *p_bf16, void *stream);

/* ------------------------------------------------------------------ CNN layers */

/* Workspace (bytes) for the gradient reductions of a layer over N volumes. */
size_t tspnn_conv_workspace(int32_t N, int32_t D0, int32_t D1, int32_t D2);

/* 1 -> 32 input layer: y = relu(conv(x) + b).  x float32 [N][D0][D1][D2];
 * w float32 [27][32]; y bfloat16 [..][32]. */
tspnn_status tspnn_conv_in_fwd(const float *x, int32_t N, int32_t D0, int32_t D1, int32_t D2,
                               const float *w, const float *b, uint16_t *y, void *stream);

/* 32 -> 32 layer on MFMA: y = relu(conv(x) + b), x, y bfloat16 [..][32],
 * w bfloat16 [27][32][32] (out, in), b float32 [32].  D2 % 32 == 0, D2 <= 128.
 * The bfloat16 arrays of the 32 -> 32 layers (here and in the two backward
 * calls below) are read and written in 8- and 16-byte pieces and must be
 * 16-byte aligned (TSPNN_E_INVALID otherwise). */
tspnn_status tspnn_conv_fwd(const uint16_t *x, int32_t N, int32_t D0, int32_t D1, int32_t D2,
                            const uint16_t *w, const float *b, uint16_t *y, void *stream);

/* 32 -> 1 output layer with residual: out = res + conv(x) + b.  x bfloat16
 * [..][32]; w float32 [27][32]; res, out float32 [N][D0][D1][D2]; res may be
 * NULL (no residual). */
tspnn_status tspnn_conv_out_fwd(const uint16_t *x, int32_t N, int32_t D0, int32_t D1, int32_t D2,
                                const float *w, const float *b, const float *res, float *out,
                                void *stream);

/*
 * Backward of a 32 -> 32 layer with respect to its input, fused with the ReLU
 * of the layer below:  dz_in = (conv^T(dz_out; w)) * (act_in > 0),
 * where conv^T is the adjoint of the layer's convolution.  dz_out, act_in,
 * dz_in bfloat16 [..][32]; w as in tspnn_conv_fwd.  D2 % 32 == 0, D2 <= 128.
 */
tspnn_status tspnn_conv_bwd_data(const uint16_t *dz_out, int32_t N, int32_t D0, int32_t D1,
                                 int32_t D2, const uint16_t *w, const uint16_t *act_in,
                                 uint16_t *dz_in, void *stream);

/* Weight / bias gradients of a 32 -> 32 layer on MFMA:
 * dw[t][o][i] = sum_p dz[p][o] x[p + off(t)][i], db[o] = sum_p dz[p][o].
 * dw float32 [27][32][32]; db float32 [32] (may be NULL).  D2 % 32 == 0, D2 <= 128.
 * work: tspnn_conv_workspace(N, D0, D1, D2) bytes of device memory; work, x
 * and dz 16-byte aligned (TSPNN_E_INVALID otherwise).  The partial sums are added up in a
 * fixed order, so equal inputs give the same bits. */
tspnn_status tspnn_conv_bwd_weight(const uint16_t *x, const uint16_t *dz, int32_t N, int32_t D0,
                                   int32_t D1, int32_t D2, float *dw, float *db, void *work,
                                   void *stream);

/* Input layer gradients: dw[t][o] = sum_p dz[p][o] x[p + off(t)], db[o]. */
tspnn_status tspnn_conv_in_bwd_weight(const float *x, const uint16_t *dz, int32_t N, int32_t D0,
                                      int32_t D1, int32_t D2, float *dw, float *db, void *work,
                                      void *stream);

/* Output layer backward: dw[t][i] = sum_p dout[p] x[p + off(t)][i],
 * db = sum_p dout[p], and dz_in = conv^T(dout; w) * (x > 0) (bfloat16, may be
 * NULL).  dout float32 [N][D0][D1][D2]. */
tspnn_status tspnn_conv_out_bwd(const uint16_t *x, const float *dout, int32_t N, int32_t D0,
                                int32_t D1, int32_t D2, const float *w, float *dw, float *db,
                                uint16_t *dz_in, void *work, void *stream);

/* Reorder 32 -> 32 weights for the input-gradient pass: wt[t][i][o] = w[26 - t][o][i]. */
tspnn_status tspnn_conv_flip_weights(const uint16_t *w, uint16_t *wt, void *stream);

/* float32 <-> bfloat16 conversion (round to nearest even) of n values. */
tspnn_status tspnn_to_bf16(const float *x, uint16_t *y, int64_t n, void *stream);
tspnn_status tspnn_from_bf16(const uint16_t *x, float *y, int64_t n, void *stream);

/* ------------------------------------------------------------------ measurement */
/*
 * Plain HBM streams, for the roofline of the projector kernels (the rate a
 * simple stream reaches on this device next to the published peak): a copy
 * of n float32 from src to dst, and a read of n float32 whose per-block sums
 * land in partial[blocks].  Non-temporal 16-byte loads and stores, a
 * grid-stride loop over `blocks` workgroups of 256 threads, four loads in
 * flight per thread.  n: a positive multiple of 4; src, dst: 16-byte
 * aligned, not overlapping; blocks in [1, TSPNN_STREAM_MAX_BLOCKS].
 * TSPNN_E_INVALID otherwise.
 */
#define TSPNN_STREAM_MAX_BLOCKS 65536
tspnn_status tspnn_stream_copy(const float *src, float *dst, int64_t n, int32_t blocks,
                               void *stream);
tspnn_status tspnn_stream_read(const float *src, int64_t n, int32_t blocks, float *partial,
                               void *stream);

const char *tspnn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TSPNN_H */
