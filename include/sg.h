/*
 * sg.h -- C ABI of the surrogate-network kernels for gfx950: a 3D
 * convolutional encoder-decoder that predicts the macroscopic state (phi, u,
 * p) of the coupled phase-field / hydrodynamic LBM K steps ahead, trained on
 * snapshots the solver itself produces.  The network is an addition to the
 * method of Holzer et al. (IJHPCA 2020); the LBM re-relaxes after every
 * jump and remains the reference (lbm.h).
 *
 * Conventions:
 *   - Activations are BF16, channels last: x[((n*D + d)*H + h)*W + w][c].
 *   - Convolutions are 3x3x3, stride 1, zero padding 1.  Weights are BF16
 *     w[t][c_out][c_in], tap t = (a+1)*9 + (b+1)*3 + (c+1) for the offset
 *     (a, b, c) along (d, h, w); bias is FP32.  Products are accumulated in
 *     FP32 on the matrix cores (v_mfma_f32_32x32x16_bf16).
 *   - Shape rules: c_in % 16 == 0, c_out % 32 == 0 (the output may keep only
 *     the first n_store channels), activation and weight pointers 16-byte
 *     aligned.
 *   - Pointers are device pointers owned by the caller; every call enqueues
 *     on hip_stream and returns sg_status; sg_last_error() has the text.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SG_OK = 0, SG_EARG = -1, SG_EHIP = -2, SG_ESIZE = -3 } sg_status;

/* y = act(conv(x, w) + bias), act = leaky ReLU with `slope` if act != 0.
 * y is BF16 with n_store channels per voxel if y_f32 == 0, else FP32. */
sg_status sg_conv3d_fwd(const void *x, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c_in,
                        const void *wt, const float *bias, int32_t c_out, int32_t n_store, int32_t act,
                        float slope, void *y, int32_t y_f32, void *hip_stream);

/* sg_conv3d_fwd of the channel concatenation [up2(xa), xb] without forming
 * it (the U-Net decoder's input): xa holds ca channels at half resolution,
 * (n, d/2, h/2, w/2, ca), and is upsampled by nearest 2x (as sg_up2_fwd);
 * xb holds cb channels at full resolution, (n, d, h, w, cb); the weights wt
 * have c_in = ca + cb input channels in that order.  The same staging and
 * products as sg_conv3d_fwd on the concatenated tensor, so the output is
 * bit-identical to it.  ca, cb positive multiples of 16; d, h, w even. */
sg_status sg_conv3d_fwd_up_cat(const void *xa, int32_t ca, const void *xb, int32_t cb, int32_t n, int32_t d,
                               int32_t h, int32_t w, const void *wt, const float *bias, int32_t c_out,
                               int32_t n_store, int32_t act, float slope, void *y, int32_t y_f32,
                               void *hip_stream);

/* Weights of the input gradient: wm[26 - t][ci][co] = wt[t][co][ci] (BF16).
 * sg_conv3d_fwd(dy, wm, bias = NULL) then gives dx[v][ci] =
 * sum_t sum_co dy[v - offset(t)][co] wt[t][co][ci]. */
sg_status sg_weight_mirror(const void *wt, int32_t c_out, int32_t c_in, void *wm, void *hip_stream);

/* Input gradient of sg_conv3d_fwd: dx[v][ci] = sum_t sum_co dy[v - offset(t)][co]
 * wt[t][co][ci] (BF16 output dx with c_in channels, FP32 accumulation).  It
 * is the forward convolution of dy with the mirrored, transposed weights,
 * which are written to `workspace` first (27 c_in c_out BF16 values,
 * 16-byte aligned, as sg_weight_mirror writes them).  c_out % 16 == 0,
 * c_in % 32 == 0; SG_ESIZE if workspace_bytes is too small. */
sg_status sg_conv3d_bwd_data(const void *dy, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c_out,
                             const void *wt, int32_t c_in, void *dx, void *workspace, size_t workspace_bytes,
                             void *hip_stream);

/* sg_conv3d_bwd_data without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as
 * sg_conv3d_bwd_data; the mirrored weights go to a fixed 4 MiB device array
 * that the library holds on each GPU it runs on until the process ends, so
 * 27 * c_in * c_out * 2 bytes must not exceed 4 MiB (SG_ESIZE otherwise).
 * Nothing is allocated.  hip_stream must belong to the current device.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams or from different threads) race and must be serialised
 * by the caller. */
sg_status sg_conv3d_bwd_data_noalloc(const void *dy, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c_out,
                                     const void *wt, int32_t c_in, void *dx, void *hip_stream);

/* Bytes of FP32 scratch sg_conv3d_bwd_weight needs for this shape. */
size_t sg_bwd_weight_workspace(int32_t n, int32_t d, int32_t h, int32_t w, int32_t c_in, int32_t c_out);

/* dw[t][co][ci] = sum_v dy[v][co] x[v + offset(t)][ci] and db[co] = sum_v dy[v][co]
 * (FP32 outputs, overwritten), deterministic two-pass reduction through
 * `workspace` (sg_bwd_weight_workspace bytes; 0 for an invalid shape).  x and
 * dy 16-byte aligned; db may be NULL. */
sg_status sg_conv3d_bwd_weight(const void *x, const void *dy, int32_t n, int32_t d, int32_t h, int32_t w,
                               int32_t c_in, int32_t c_out, float *dw, float *db, void *workspace,
                               size_t workspace_bytes, void *hip_stream);

/* Elementwise leaky-ReLU backward from the layer output: dpre = dy * (y > 0 ? 1 : slope). */
sg_status sg_leaky_bwd(const void *y, const void *dy, void *dpre, size_t count, float slope, void *hip_stream);

/* 2x average pooling (d, h, w even) and its backward (dx = dy / 8 spread). */
sg_status sg_pool2_fwd(const void *x, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, void *y,
                       void *hip_stream);
sg_status sg_pool2_bwd(const void *dy, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, void *dx,
                       void *hip_stream);

/* 2x nearest upsampling of a (n, d, h, w, c) tensor and its backward (sum of
 * the 8 children). */
sg_status sg_up2_fwd(const void *x, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, void *y,
                     void *hip_stream);
sg_status sg_up2_bwd(const void *dy, int32_t n, int32_t d, int32_t h, int32_t w, int32_t c, void *dx,
                     void *hip_stream);

/* Channel concatenation y = [a | b] (ca + cb channels) and its split. */
sg_status sg_concat(const void *a, int32_t ca, const void *b, int32_t cb, int64_t voxels, void *y,
                    void *hip_stream);
sg_status sg_split(const void *y, int32_t ca, int32_t cb, int64_t voxels, void *a, void *b, void *hip_stream);

/* Mean squared error over `count` FP32 values: loss (device FP32 scalar,
 * deterministic fixed-order reduction through `scratch`, 1024 floats) and
 * the BF16 gradient 2 (pred - target) / count. */
sg_status sg_mse(const float *pred, const float *target, int64_t count, float *loss, void *grad_bf16,
                 float *scratch, void *hip_stream);

/* One Adam step (Kingma and Ba) on FP32 master weights p with FP32 moments m, v
 * and gradient g; also writes the BF16 copy wt of p.  step >= 1. */
sg_status sg_adam(float *p, const float *g, float *m, float *v, void *wt_bf16, int64_t count, float lr,
                  float beta1, float beta2, float eps, int32_t step, void *hip_stream);

/* FP32 -> BF16 and BF16 -> FP32 conversions (round to nearest even). */
sg_status sg_to_bf16(const float *x, void *y, int64_t count, void *hip_stream);
sg_status sg_to_f32(const void *x, float *y, int64_t count, void *hip_stream);

/* y = a + b elementwise (BF16), used to join gradients of a skip connection. */
sg_status sg_add(const void *a, const void *b, void *y, int64_t count, void *hip_stream);

/* ---- between the LBM fields and the network ------------------------------------
 * Fields are FP32 planes of an nx * ny * nz grid, x fastest (phi, u as 3
 * planes, p); a box is (x0, y0, z0, bx, by, bz), wrapped periodically in x
 * and z; y must lie inside [0, ny).  A box becomes one network sample with
 * D = bz, H = by, W = bx.  `box` (6 int32) and the per-channel scales (5
 * floats) are HOST arrays read during the call. */

/* Network input of a box: channels (phi, u_x, u_y, u_z, p) / scale_in, then
 * zeros up to c_in (>= 5) channels, BF16; optionally the raw FP32 state
 * (5 channels per voxel) into `state` (may be NULL). */
sg_status sg_fields_to_input(const float *phi, const float *u, const float *p, int32_t nx, int32_t ny,
                             int32_t nz, const int32_t *box, const float *scale_in, int32_t c_in, void *x_bf16,
                             float *state, void *hip_stream);

/* Network input of raw states stored channels last (5 FP32 channels per
 * voxel, as written by sg_fields_to_input): state / scale_in, zero-padded to
 * c_in channels, BF16. */
sg_status sg_state_to_input(const float *state, int64_t voxels, const float *scale_in, int32_t c_in, void *x_bf16,
                            void *hip_stream);

/* Training target of a pair of raw states: (s1 - s0) / scale_out in the first
 * 5 of c_out channels, zeros in the rest (FP32). */
sg_status sg_make_target(const float *s0, const float *s1, int64_t voxels, const float *scale_out,
                         int32_t c_out, float *target, void *hip_stream);

/* Applies a predicted increment to the fields of a box: field = base + out * scale_out
 * per channel (out has c_out FP32 channels, the first 5 used; base is a raw
 * state of the box, 5 FP32 channels per voxel, or NULL for the field itself);
 * phi is clipped to [phi_min, phi_max] afterwards (phi_max > phi_min) unless
 * flags & 4 (SG_APPLY_NO_CLIP).  With
 * q = clamp((phi_base - phi_min)/(phi_max - phi_min), 0, 1): flags & 1
 * (SG_APPLY_U_BY_PHASE) weights the velocity increment by q, flags & 2
 * (SG_APPLY_PHI_AT_INTERFACE) weights the phi increment by 4 q (1 - q).
 * Cells of the rows y = 0 and ny-1 are left unchanged if walls_y.  A zero
 * scale leaves that channel at its base. */
enum { SG_APPLY_U_BY_PHASE = 1, SG_APPLY_PHI_AT_INTERFACE = 2, SG_APPLY_NO_CLIP = 4 };
sg_status sg_apply_prediction(const float *out, int32_t c_out, const float *scale_out, const float *base,
                              float *phi, float *u, float *p, int32_t nx, int32_t ny, int32_t nz,
                              const int32_t *box, int32_t walls_y, float phi_min, float phi_max,
                              int32_t flags, void *hip_stream);

/* Physics baseline of a jump of K steps on `count` boxes of raw states
 * (count x bz x by x bx voxels, 5 FP32 channels each, x fastest): phi is
 * transported by the local velocity, phi'(x) = phi(x - K u(x)) with
 * trilinear interpolation and the departure point clamped to the box; u and
 * p are copied.  out must not alias state. */
sg_status sg_advect_phase(const float *state, int64_t count, int32_t bx, int32_t by, int32_t bz, float K,
                          float *out, void *hip_stream);

/* Co-moving baseline of a jump on `count` boxes of raw states (layout as in
 * sg_advect_phase): every channel is translated, out(x) = state(x - d_n)
 * with d_n = (shift[4n], shift[4n+1], shift[4n+2]) in cells, trilinear
 * interpolation, the departure point clamped to the box; the velocity
 * channels are then multiplied by f_n = shift[4n+3].  shift is a DEVICE
 * array of 4 count floats.  A bubble rising at constant speed U is steady
 * in its own frame, so d = K U (f = 1) moves its whole neighbourhood K
 * steps ahead; a slowly accelerating one is followed to first order by
 * d = K U + K^2 a / 2 and f = 1 + K a.U / |U|^2.  out must not alias
 * state. */
sg_status sg_shift_boxes(const float *state, int64_t count, int32_t bx, int32_t by, int32_t bz, const float *shift,
                         float *out, void *hip_stream);

/* Gas-indicator moments of `count` boxes of raw states: with chi =
 * clamp((phi_heavy - phi)/(phi_heavy - phi_light), 0, 1) (the indicator of
 * the statistics in lbm.h), out[8n + k] (DEVICE, 8 count doubles) holds
 * k = 0: sum chi; 1-3: sum chi x, chi y, chi z (box coordinates, x
 * fastest); 4-6: sum chi u_x, chi u_y, chi u_z; 7: 0.  FP64, one block per
 * box, fixed-order reduction (deterministic).  Gives the gas centroid and
 * the gas-weighted velocity of each box. */
sg_status sg_box_moments(const float *state, int64_t count, int32_t bx, int32_t by, int32_t bz, float phi_heavy,
                         float phi_light, double *out, void *hip_stream);

/* Projective time step of field sets (Gear and Kevrekidis, SIAM J. Sci.
 * Comput. 24, 2003): out = s + ratio (s - s_prev) per channel over n points,
 * channels (phi, u_x, u_y, u_z, p); element (i, k) at f[k cs + i vs], either
 * planar (cs = n, vs = 1: the solver's FP32 field planes, phi then u then p
 * as one allocation per argument) or channels last (cs = 1, vs = 5: box
 * states).  phi is clipped to [phi_lo, phi_hi]; with u_by_phase == 1 the
 * velocity increment is weighted by the heavy-phase fraction q of the
 * current phi, with u_by_phase == 2 by clamp(10 q - 9, 0, 1) (the bulk of
 * the heavy phase only);
 * with phi_step == 0 phi is carried over (and clipped), with p_step == 0
 * the pressure.  out may alias s. */
sg_status sg_projective_step(const float *s, const float *s_prev, int64_t n, int64_t cs, int64_t vs, float ratio,
                             float phi_lo, float phi_hi, int32_t u_by_phase, int32_t phi_step, int32_t p_step,
                             float *out, void *hip_stream);

/* Network input of a box state s and the same box m steps earlier (5 FP32
 * channels per voxel each): channels 0-4 = s / scale_in, 5-9 =
 * (s - s_prev) * trend_scale (both HOST arrays of 5 floats), each clipped
 * to [-16, 16], zeros up to c_in (>= 10) channels, BF16. */
sg_status sg_pair_to_input(const float *state, const float *state_prev, int64_t voxels, const float *scale_in,
                           const float *trend_scale, int32_t c_in, void *x_bf16, void *hip_stream);

/* Per-channel sums: out[c] = sum_r a[r][c] and out[8 + c] = sum_r a[r][c]^2
 * in FP64 over a (rows, C) FP32 array, C <= 8 (out has 16 doubles; unused
 * channels are 0); deterministic fixed-order reduction through `scratch`
 * (512 x 16 doubles). */
sg_status sg_channel_moments(const float *a, int64_t rows, int32_t c, double *out, double *scratch,
                             void *hip_stream);

/* Mass projection of a phase field after a jump (the fast-forward's
 * substitute for the exact conservation of sum(phi) by the scheme, Section
 * 3.1): phi is an FP32 field of an nx * ny * nz grid (x fastest); with
 * walls_y the rows y = 0 and ny-1 are solid and take no part.  Over the
 * fluid cells, with q = clamp((phi - phi_min)/(phi_max - phi_min), 0, 1):
 *   phi += c 4 q (1 - q),  c = (target_mass - sum phi) / sum 4 q (1 - q)
 * (c = 0 if no cell lies inside the interface), so the correction stays in
 * the interface and the fluid sum equals target_mass up to the FP32
 * rounding of the stored cells.  Sums are FP64 with a fixed-order reduction
 * through `scratch` (device, 2048 doubles, overwritten).  SG_EARG for
 * phi_max <= phi_min, an empty grid or walls_y with ny < 3. */
sg_status sg_mass_project(float *phi, int32_t nx, int32_t ny, int32_t nz, int32_t walls_y, double target_mass,
                          float phi_min, float phi_max, double *scratch, void *hip_stream);

const char *sg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
