/*
 * gpe_learn.h -- C-ABI of the learned coarse-grid correction of libgpe: a
 * small convolutional network that, after every step of the GPE solver on a
 * grid coarsened by an integer factor, adds a correction to the coarse
 * state, trained on restrictions of the solver's own fine-grid runs.  The
 * network and its training are not part of the paper's method; the paper's
 * Sec. 4 Rayleigh-Taylor set-up supplies the flows it is trained and
 * evaluated on, and the plain fine-grid solver (include/gpe.h) stays the
 * reference and the fallback.
 *
 * Network: three 3 x 3 convolutions, channels 4 -> 32 -> 32 -> 4, ReLU after
 * the first two; x periodic, y zero-padded (walls).  Input channels at cell
 * centres: (u_c, v_c, p, phi) / in_scale, u_c and v_c the means of the two
 * faces of a cell (the face above the top row is a wall face, 0).  Output
 * channels: corrections of (u, v, p, phi) in units of out_scale, applied to
 * the low-face velocities and the centre values of the same cell index.
 *
 * Conventions:
 *  - 2-D states only, FP32 fields of shape (ny, nx), x fastest, as stored by
 *    gpe.h.  A batch of B states is passed as a device array of 4 B device
 *    pointers, (u, v, p, phi) of case 0, then case 1, ...
 *  - Activations are NHWC (case, y, x, channel).  act_type selects their
 *    storage and that of the weight copy the kernels read: GPE_ACT_BF16
 *    (bfloat16 operands, round to nearest even) or GPE_ACT_FP32; every sum
 *    accumulates in FP32.  Master weights, gradients and Adam moments are
 *    FP32.
 *  - Parameters are packed: w1 [32][3][3][4], b1 [32], w2 [32][3][3][32],
 *    b2 [32], w3 [4][3][3][32], b3 [4] (gpe_cnn_param_count floats); a tap
 *    (dy, dx) sits at index (dy + 1, dx + 1) and reads input (y + dy, x + dx).
 *  - The caller owns every buffer (device memory) and the stream; every call
 *    only enqueues kernels, except where noted.  Errors: GPE_OK or a negative
 *    gpe_error (GPE_EINVAL for bad sizes or null pointers, GPE_EHIP).
 */
#ifndef GPE_LEARN_H
#define GPE_LEARN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum gpe_act_type { GPE_ACT_BF16 = 0, GPE_ACT_FP32 = 1 };

/* Number of FP32 parameters of the network (weights and biases, packed). */
size_t gpe_cnn_param_count(void);

/* Bytes of one activation element for act_type (2 or 4; 0 if invalid). */
size_t gpe_cnn_act_bytes(int32_t act_type);

/* Bytes of the scratch buffer gpe_cnn_backward and gpe_cnn_loss need for
 * B states of H x W cells (deterministic two-pass reductions). */
size_t gpe_cnn_scratch_bytes(int32_t B, int32_t H, int32_t W);

/* Restriction of B fine states (ny x nx) to (ny/f) x (nx/f): cell means of
 * p and phi over f x f cells; the coarse low x-face velocity is the mean of
 * the f fine x-faces on it (likewise y).  ny, nx multiples of f; f = 1
 * copies the states. */
int gpe_restrict2d(const float* const* d_fine, float* const* d_coarse, int32_t B, int32_t ny, int32_t nx,
                   int32_t f, void* stream);

/* Training target [B][H][W][4] (FP32): (next - pred) / out_scale per field
 * (u, v, p, phi) and cell, from two tables of B states each. */
int gpe_cnn_target(const float* const* d_next, const float* const* d_pred, int32_t B, int32_t H, int32_t W,
                   const float out_scale[4], float* d_target, void* stream);

/* Network input x0 [B][H][W][4] (act_type) from B coarse states. */
int gpe_cnn_features(const float* const* d_fields, int32_t B, int32_t H, int32_t W, const float in_scale[4],
                     int32_t act_type, void* d_x0, void* stream);

/* Copy of the FP32 master parameters in act_type (what the kernels read). */
int gpe_cnn_convert(const float* d_params, void* d_params_act, int32_t act_type, void* stream);

/* Forward pass: x0 -> a1 = relu(conv1), a2 = relu(conv2) (act_type, kept
 * for the backward pass), out = conv3 [B][H][W][4] (FP32).  Biases come from
 * the FP32 master parameters d_params, weights from d_params_act. */
int gpe_cnn_forward(const float* d_params, const void* d_params_act, const void* d_x0, void* d_a1, void* d_a2,
                    float* d_out, int32_t B, int32_t H, int32_t W, int32_t act_type, void* stream);

/* Loss = mean over the n outputs of (out - target)^2 into d_loss[0] (FP32)
 * and its gradient d_gout = 2 (out - target) / n. */
int gpe_cnn_loss(const float* d_out, const float* d_target, float* d_gout, float* d_loss, int64_t n,
                 void* d_scratch, size_t scratch_bytes, void* stream);

/* Backward pass from d_gout (gradient of the loss w.r.t. out) through the
 * activations of the last forward pass: d_grads (FP32, packed like the
 * parameters) receives the parameter gradients. */
int gpe_cnn_backward(const float* d_params, const void* d_params_act, const void* d_x0, const void* d_a1,
                     const void* d_a2, const float* d_gout, float* d_grads, int32_t B, int32_t H, int32_t W,
                     int32_t act_type, void* d_scratch, size_t scratch_bytes, void* stream);

/* One Adam step on the FP32 master parameters (bias-corrected moments;
 * t = 1 for the first step). */
int gpe_cnn_adam(float* d_params, float* d_m, float* d_v, const float* d_grads, int64_t n, float lr, float beta1,
                 float beta2, float eps, int64_t t, void* stream);

/* Correction of B coarse states by the network output: (u, v, p, phi) +=
 * out_scale * out; the v correction is 0 on the wall row j = 0 and the phi
 * correction has its mean over each state subtracted (phase mass kept).
 * d_scratch holds B floats. */
int gpe_cnn_apply(float* const* d_fields, const float* d_out, int32_t B, int32_t H, int32_t W,
                  const float out_scale[4], float* d_scratch, void* stream);

/* Bytes of the scratch buffer gpe_cnn_infer needs for B states of H x W
 * cells (one float per 32 x 8 tile and one per state); 0 for invalid
 * sizes. */
size_t gpe_cnn_infer_scratch_bytes(int32_t B, int32_t H, int32_t W);

/* Fused inference with BF16 operands: the network input of B coarse states,
 * the three convolutions (all on the matrix cores, FP32 accumulation) and
 * the correction of the states, the same operations as gpe_cnn_features,
 * gpe_cnn_forward and gpe_cnn_apply with GPE_ACT_BF16, in two launches (three
 * when H W < 256 or a state has more than 128 tiles) and without storing
 * activations in device memory (a work-group keeps a 32 x 8
 * tile's activations, with their halos, in LDS).  d_params are the FP32
 * master parameters (biases), d_params_bf16 their GPE_ACT_BF16 copy
 * (gpe_cnn_convert); d_out receives the network output [B][H][W][4] as
 * gpe_cnn_forward writes it.  Every layer uses the double-K MFMA and adds
 * in another order than the unfused kernels (and rounds NaN payloads
 * differently), so results agree with them to FP32 rounding, not bitwise.
 * d_scratch: gpe_cnn_infer_scratch_bytes(B, H, W) bytes. */
int gpe_cnn_infer(float* const* d_fields, const float* d_params, const void* d_params_bf16, int32_t B, int32_t H,
                  int32_t W, const float in_scale[4], const float out_scale[4], float* d_out, void* d_scratch,
                  size_t scratch_bytes, void* stream);

/* Capacity, in floats, of the buffer gpe_cnn_infer_noalloc keeps in device
 * memory (256 KiB on every GPU the library runs on). */
#define GPE_CNN_INFER_STATIC_FLOATS 65536

/* Allocation-free variant of gpe_cnn_infer, for callers that cannot allocate
 * device memory or hand over a scratch buffer: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  The same kernels
 * and arguments without d_scratch / scratch_bytes; results are bitwise those
 * of gpe_cnn_infer.  The per-tile partial sums live in a buffer of
 * GPE_CNN_INFER_STATIC_FLOATS floats that the library holds in the device
 * memory of each GPU it runs on until the process ends; every entry a call
 * reads is written by the same call first, so no clearing is needed.
 *  - Limit: gpe_cnn_infer_scratch_bytes(B, H, W) must not exceed
 *    GPE_CNN_INFER_STATIC_FLOATS * 4 bytes (one float per 32 x 8 tile and one
 *    per state, e.g. B = 1000 states of 64 x 256); larger batches return
 *    GPE_EWORKSPACE and launch nothing.
 *  - Every call on one GPU shares that GPU's buffer: calls that may overlap
 *    in time on one GPU (different streams, or threads) race; the caller
 *    orders them, e.g. on one stream.
 *  - The first call on a device looks the buffer's address up (no
 *    allocation, no stream operation).
 *  - Never calls hipMalloc, hipFree or any allocating routine.
 * Returns GPE_OK, GPE_EINVAL, GPE_EWORKSPACE or GPE_EHIP. */
int gpe_cnn_infer_noalloc(float* const* d_fields, const float* d_params, const void* d_params_bf16, int32_t B,
                          int32_t H, int32_t W, const float in_scale[4], const float out_scale[4], float* d_out,
                          void* stream);

/* Interface position of B states: per column x the outermost phi = 0
 * crossings, the first sign change scanning down from the top row and up
 * from the bottom row, linearly interpolated between cell centres
 * (y = j + 1/2); d_out [B][W][2] = (top, bottom), NaN where none. */
int gpe_interface_position(const float* const* d_phi, int32_t B, int32_t H, int32_t W, float* d_out,
                           void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GPE_LEARN_H */
