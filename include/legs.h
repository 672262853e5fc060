/*
 * legs.h -- C ABI of the MI355X (gfx950) splatting and decoding library for
 * Language Embedded 3D Gaussians (arXiv 2311.18482).
 *
 * The library renders anisotropic 3D Gaussians that carry RGB, a compact
 * semantic feature s_G and an uncertainty u (Sec. 3.4.1, 3.4.2) through the
 * differentiable rasteriser I = R(p, Sigma, c, alpha; p_cam) of Sec. 3.1,
 * Eq. 1, back-propagates a loss through it, and decodes rendered semantic
 * features into a distribution over the discrete feature space S (Sec. 3.3,
 * Eq. 4; Sec. 3.4.1, Eq. 8; supplementary inference equation).
 *
 * Conventions shared by every call
 *  - Every pointer argument named *_dev or documented as "device" is device
 *    memory of the context's GPU, allocated and owned by the caller. The
 *    library never allocates on the calls below (the context owns nothing but
 *    its error text).
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = legacy default
 *    stream) and is asynchronous unless stated otherwise.
 *  - Return codes: LEGS_OK, or a negative LEGS_ERR_* code. On error nothing is
 *    launched unless stated, and legs_last_error(ctx) holds a message.
 *  - Gaussian parameters are row-major float32: mean [n][3], log_scale [n][3],
 *    quat [n][4] as (w, x, y, z) (normalised inside, need not be unit),
 *    opacity_logit [n] (opacity = sigmoid(logit)), channels [n][C] with
 *    C <= LEGS_MAX_CHANNELS (RGB, s_G and u are ordinary channels).
 *  - Rendered outputs are planar per view, views concatenated in order:
 *    out[C * pixel_offset(v) + c * H_v * W_v + y * W_v + x]; per-pixel
 *    auxiliaries (final transmittance, last contributor) are
 *    [pixel_offset(v) + y * W_v + x].
 *  - Projected records and per-(Gaussian, view) gradients are indexed
 *    gv = v * n + g ("G-view").
 */
#ifndef LEGS_H
#define LEGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LEGS_OK 0
#define LEGS_ERR_ARG (-1)         /* invalid argument; nothing launched */
#define LEGS_ERR_CAPACITY (-2)    /* instance list longer than its buffers */
#define LEGS_ERR_HIP (-3)         /* a HIP runtime call failed */
#define LEGS_ERR_UNSUPPORTED (-4) /* valid request the library does not serve */

#define LEGS_MAX_CHANNELS 64
#define LEGS_MAX_VIEWS 4096

typedef struct legs_ctx legs_ctx;

/* Pinhole camera, OpenCV axes (x right, y down, z forward); world -> camera
 * x_c = R x_w + t; pixel (i, j) has its centre at (i + 1/2, j + 1/2). */
typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double R[9]; /* row-major */
    double t[3];
} legs_camera;

/* One entry of the view table (built on the host by legs_views_build, then
 * copied by the caller into device memory for the calls below). */
typedef struct {
    legs_camera cam;
    int32_t tiles_x, tiles_y;
    int64_t tile_offset;  /* first global tile id of this view */
    int64_t pixel_offset; /* first pixel of this view in the concatenated planes */
} legs_view;

/* Blend kernels as one persistent launch per call over the tiles of every
 * view: the launch first orders all tiles by decreasing list length (the
 * heaviest first), then workgroups take tiles from that queue through an
 * atomic counter in the sort scratch until it is empty, instead of one
 * workgroup per tile. Results are identical. */
#define LEGS_FLAG_PERSISTENT 1
/* Bin with all 8-bit digits of the 64-bit keys sorted over the instances
 * (6 passes at 8160 tiles) instead of the depth-first binning: the G-views
 * sorted by depth, their 8x4-tile super-tile entries sorted by super-tile,
 * and each super-tile's list compacted into its tiles' lists. The lists are
 * identical. The depth-first binning needs capacity + total_tiles < 2^32. */
#define LEGS_FLAG_FULL_SORT 2
/* Blend kernels evaluate alpha at every pixel of each Gaussian's 3-sigma box.
 * By default they skip the pixels outside the bounding box of the ellipse
 * where opacity * exp(power) can reach alpha_min (widened for float32
 * rounding): alpha stays below alpha_min there, so images, T_final, last and
 * gradients are the same either way; only the work differs. */
#define LEGS_FLAG_FULL_BOX 4
/* Depth-first binning writes the per-tile lists of Gaussian ids and the
 * ranges only, not the 64-bit keys (the blend kernels read ids and ranges):
 * bins->keys is left as it was. The lists and ranges are the same. The
 * full-sort binning sorts the keys themselves and ignores this flag. */
#define LEGS_FLAG_IDS_ONLY 8

/* Rasteriser options. Defaults (legs_opts_default): tile 16, lds_batch 256,
 * alpha_max 0.99, alpha_min 1/255, t_min 1e-4, lowpass 0.3 px^2, z_near 0.2,
 * guard 1.3. */
typedef struct {
    int32_t tile;      /* tile edge in pixels: 8, 16 or 32 */
    int32_t lds_batch; /* Gaussians staged in LDS per round: 64, 128 or 256 (the
                          backward with one wave per tile stages at most 128) */
    float alpha_max;   /* alpha = min(alpha_max, opacity * exp(power)) */
    float alpha_min;   /* skip a Gaussian at a pixel when alpha < alpha_min */
    float t_min;       /* stop (without blending) when T * (1 - alpha) < t_min */
    int32_t flags;     /* LEGS_FLAG_* bits */
    double lowpass;    /* added to both diagonal entries of the 2D covariance */
    double z_near;     /* cull Gaussians with camera-space z <= z_near */
    double guard;      /* Jacobian evaluated at x/z clamped to +-guard * W / (2 fx) */
} legs_opts;

/* Per-G-view projected records (device, caller-owned, length n_views * n
 * except block_offsets):
 *   mean2d  [G][2] double  2D mean in pixels (EWA projection of p)
 *   conic   [G][4] float   (A, B, C, opacity): inverse 2D covariance and sigmoid(logit)
 *   box     [G][4] int32   inclusive pixel box (x0, x1, y0, y1): pixels with
 *                          |x + 1/2 - mx| <= r and |y + 1/2 - my| <= r,
 *                          r = ceil(3 sqrt(lambda_max)); x0 > x1 when culled
 *   depth   [G]    float   camera-space z rounded to float (sort key)
 *   ntiles  [G]    uint32  tiles touched by the box (0 when culled)
 *   block_offsets [2 * (legs_projected_blocks(n, n_views) + 1)] uint64 scratch:
 *                          per-block instance counts (written by legs_project),
 *                          then their exclusive scan (written by legs_bin_sort)
 *   order   legs_order_scratch_bytes(n, n_views) bytes of scratch for the depth
 *           order of the G-views used by legs_bin_sort (NULL: the binning
 *           falls back to sorting every key digit over the instances) */
typedef struct {
    double *mean2d;
    float *conic;
    int32_t *box;
    float *depth;
    uint32_t *ntiles;
    uint64_t *block_offsets;
    void *order;
} legs_projected;

/* Tile lists (device, caller-owned). keys/ids hold the sorted instance list on
 * return: key = (global_tile << 32) | bits(depth), sorted ascending, ties in
 * Gaussian order. ranges[2 t], ranges[2 t + 1] = [start, end) of tile t.
 * keys_alt/ids_alt are ping-pong buffers; scratch is legs_sort_scratch_bytes. */
typedef struct {
    uint64_t *keys, *keys_alt;  /* [capacity] */
    uint32_t *ids, *ids_alt;    /* [capacity] */
    uint32_t *ranges;           /* [total_tiles][2] */
    void *scratch;
    uint64_t *count;            /* [1] number of instances (may exceed capacity) */
    int64_t capacity;
} legs_bins;

/* ---- context ------------------------------------------------------------- */

/* Create a context bound to HIP device `device`. Returns LEGS_ERR_ARG for a
 * bad device, LEGS_ERR_UNSUPPORTED if it is not gfx950. */
int32_t legs_create(int32_t device, legs_ctx **out);
int32_t legs_destroy(legs_ctx *ctx);
/* Text of the last error on this context (static storage inside ctx). */
const char *legs_last_error(const legs_ctx *ctx);
int32_t legs_version(void);
void legs_opts_default(legs_opts *o);

/* ---- host-side sizing (no GPU work) --------------------------------------- */

/* Fill the view table for n_views cameras and the chosen tile size; returns
 * the total tile and pixel counts. LEGS_ERR_ARG on bad sizes. */
int32_t legs_views_build(const legs_camera *cams, int32_t n_views, const legs_opts *opts,
                         legs_view *out_host, int64_t *total_tiles, int64_t *total_pixels);
/* Number of 256-entry blocks the projection uses for n Gaussians x n_views. */
int64_t legs_projected_blocks(int64_t n, int32_t n_views);
/* Bytes of legs_projected.order for n Gaussians x n_views. */
int64_t legs_order_scratch_bytes(int64_t n, int32_t n_views);
/* Bytes of legs_bins.scratch for a given instance capacity and tile count. */
int64_t legs_sort_scratch_bytes(int64_t capacity, int64_t total_tiles);
/* Radix passes the sort runs for total_tiles tiles (8-bit digits over the
 * 32 depth bits plus ceil(log2 total_tiles) tile bits). */
int32_t legs_sort_passes(int64_t total_tiles);

/* ---- rasteriser (Sec. 3.1 Eq. 1; Sec. 3.4.1 R_s; Sec. 3.4.2 R_u) ---------- */

/* EWA projection of every (Gaussian, view): camera transform, 3D covariance
 * R S S^T R^T from quaternion and exp(log_scale), 2D covariance
 * J W Sigma W^T J^T + lowpass I with the guard-band clamped Jacobian, conic,
 * 2D mean, 3-sigma integer pixel box, tile count and depth key; also the
 * per-block instance counts in out->block_offsets. Computed in float64.
 * views_dev: device legs_view[n_views]. */
int32_t legs_project(legs_ctx *ctx, const float *mean, const float *log_scale, const float *quat,
                     const float *opacity_logit, int64_t n, const legs_view *views_dev,
                     int32_t n_views, const legs_opts *opts, legs_projected *out, void *stream);

/* Tile binning: one (key, id) per (tile, Gaussian) overlap, sorted by the
 * 64-bit key (global_tile << 32) | bits(depth) with a stable LSD onesweep
 * radix sort, and per-tile [start, end) ranges. By default the depth digits
 * are sorted once per G-view (every instance of a Gaussian in a view shares
 * its depth), the instances are emitted in that order and only the tile
 * digits are sorted over the instances; LEGS_FLAG_FULL_SORT sorts every digit
 * over the instances. Both give the same lists. If host_count != NULL the call waits for the
 * instance total, stores it in *host_count and returns LEGS_ERR_CAPACITY
 * (launching nothing further) when it exceeds bins->capacity. With
 * host_count == NULL nothing waits (graph-capturable): the lists are then
 * truncated to the capacity and *bins->count > capacity signals overflow. */
int32_t legs_bin_sort(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                      const legs_view *views_dev, int32_t n_views, int64_t total_tiles,
                      const legs_opts *opts, legs_bins *bins, int64_t *host_count, void *stream);

/* Front-to-back compositing of all C channels per pixel over its tile list:
 * alpha = min(alpha_max, opacity * exp(power)) inside the Gaussian's box,
 * skipped when alpha < alpha_min, stopped (not blended) when
 * T * (1 - alpha) < t_min; background 0. Writes out (planar, see top),
 * T_final and last = 1 + tile-list position of the last blended Gaussian. */
int32_t legs_render_forward(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                            const legs_bins *bins, const legs_view *views_dev, int32_t n_views,
                            int64_t total_tiles, const float *channels, int32_t C,
                            const legs_opts *opts, float *out, float *T_final, uint32_t *last,
                            void *stream);

/* legs_render_forward that also sets the zero_bytes bytes at zero (device
 * memory, 16-byte aligned, zero_bytes a multiple of 4) to 0 in the same
 * launch: each workgroup stores its share before compositing, so the stores
 * drain while the ALU-bound compositing runs instead of costing a launch and
 * a pass of their own. Meant for the gradient buffers that the following
 * legs_render_backward and legs_project_backward accumulate into; the range
 * must not overlap any buffer the compositing reads or writes (the result is
 * then undefined). LEGS_ERR_ARG for a misaligned pointer or a bad size. */
int32_t legs_render_forward_zero(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                                 const legs_bins *bins, const legs_view *views_dev, int32_t n_views,
                                 int64_t total_tiles, const float *channels, int32_t C,
                                 const legs_opts *opts, float *out, float *T_final, uint32_t *last,
                                 void *zero, int64_t zero_bytes, void *stream);

/* Gradient of a loss with dL/d(out) = d_out (planar like out) through the
 * compositing, replaying each pixel back to front from (T_final, last).
 * Accumulates (+=) into grad2d [G][8] = d(mx, my, A, B, C, opacity, -, -)
 * and d_channels [n][C]; the caller zeroes them first. */
int32_t legs_render_backward(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                             const legs_bins *bins, const legs_view *views_dev, int32_t n_views,
                             int64_t total_tiles, const float *channels, int32_t C,
                             const legs_opts *opts, const float *T_final, const uint32_t *last,
                             const float *d_out, float *grad2d, float *d_channels, void *stream);

/* Work counts of the compositing kernels for the given lists (a statistics
 * pass for roofline reports; it replays the forward decisions). counts [4]
 * uint64 device: alpha evaluations of the forward (entries inside a pixel's
 * box up to and including the stop), blended entries, alpha evaluations of
 * the backward (entries inside the box before `last`), list positions walked
 * by a per-pixel traversal. Overwritten. */
int32_t legs_render_counts(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                           const legs_bins *bins, const legs_view *views_dev, int32_t n_views,
                           int64_t total_tiles, const legs_opts *opts, uint64_t *counts,
                           void *stream);

/* Chain rule from grad2d back to mean, log_scale, (unnormalised) quaternion
 * and opacity logit, summed over views; accumulates (+=) into the outputs. */
int32_t legs_project_backward(legs_ctx *ctx, const float *mean, const float *log_scale,
                              const float *quat, const float *opacity_logit, int64_t n,
                              const legs_view *views_dev, int32_t n_views, const legs_opts *opts,
                              const legs_projected *proj, const float *grad2d, float *d_mean,
                              float *d_log_scale, float *d_quat, float *d_opacity_logit,
                              void *stream);


/* ---- decoding (Sec. 3.3 Eq. 4; Sec. 3.4.1 Eq. 8; supplementary inference) --- */

/* Rendered compact features have LEGS_DECODE_DIN channels. A feature element
 * (pixel p, channel c) is read at feat[c * c_stride + p * p_stride], so the
 * planar maps of legs_render_forward (c_stride = H W, p_stride = 1, starting
 * at the first semantic channel) and row-major [P][8] arrays (c_stride = 1,
 * p_stride = 8) both work without a copy. K (codes) is 32, 64 or 128.
 * probs (nullable) is [P][K] float; top1 is [P] int32, lowest index on ties. */
#define LEGS_DECODE_DIN 8

/* Plain decode: z = P f (proj [D][8], D a multiple of 32 up to 512), cosine
 * scores s_k = <c_k, z> / (|c_k| |z|) against codebook [K][D] (Eq. 4's
 * max-similarity search), softmax over k, argmax. s = 0 when z = 0. */
int32_t legs_decode_plain(legs_ctx *ctx, const float *feat, int64_t P, int64_t c_stride,
                          int64_t p_stride, const float *proj, int32_t D, const float *codebook,
                          int32_t K, float *probs, int32_t *top1, void *stream);

/* Exact algebraic folding of the plain decode: folded [(K + 8) * 8] floats =
 * rows (c_k P) / |c_k| followed by the Gram matrix P^T P (float64 sums). */
int32_t legs_decode_fold(legs_ctx *ctx, const float *proj, int32_t D, const float *codebook,
                         int32_t K, float *folded, void *stream);
/* The plain decode's scores from the folded form: s_k = (M f)_k / sqrt(f^T Q f). */
int32_t legs_decode_folded(legs_ctx *ctx, const float *feat, int64_t P, int64_t c_stride,
                           int64_t p_stride, const float *folded, int32_t K, float *probs,
                           int32_t *top1, void *stream);

/* Learned decode softmax(D_MLP(R_s)) of Sec. 3.4.1, Eq. 8 (and the
 * supplementary inference equation), D_MLP = 8 -> 64 -> 64 -> K per-pixel
 * linear layers with ReLU (1x1 convolutions, the pattern of Table 3). params
 * are float32 masters packed W1 [64][8], b1 [64], W2 [64][64], b2 [64],
 * W3 [K][64], b3 [K]; weights, input and hidden activations are rounded to
 * bf16 (nearest even), accumulation and biases are float32.
 * mlp_flags: LEGS_MLP_NORMALIZE_INPUT feeds the decoder the feature divided
 * by its Euclidean norm (a zero feature stays zero) instead of the feature
 * itself: the plain decode's codes (Eq. 4's cosine search) depend only on the
 * feature's direction, and a decoder given the direction reaches 99 % top-1
 * agreement with them where one given the raw feature does not (this is a
 * reading beyond Eq. 8, which applies the decoder to R_s directly). Every
 * call that runs the decoder (decode, gradient, training step, semantic loss)
 * takes the same flags, and the same parameters must be used with the same
 * flags. Unknown bits: LEGS_ERR_ARG. With probs == NULL only top1 is written
 * (a kernel that never holds all K logits). */
#define LEGS_MLP_NORMALIZE_INPUT 1
int64_t legs_mlp_param_count(int32_t K);
int32_t legs_decode_mlp(legs_ctx *ctx, const float *feat, int64_t P, int64_t c_stride,
                        int64_t p_stride, const float *params, int32_t K, int32_t mlp_flags,
                        float *probs, int32_t *top1, void *stream);

/* Decoder of Table 3 (supplementary implementation details): D_MLP = 1x1
 * convolutions 8 -> 128 -> 256 -> N with ReLU between them, N (the size of
 * the discrete feature space) 32, 64 or 128; M_infer = softmax(D_MLP(R_s))
 * per pixel (supplementary inference equation). params: float32 masters
 * [legs_dmlp_param_count(N)] packed W1 [128][8], b1 [128], W2 [256][128],
 * b2 [256], W3 [N][256], b3 [N]; weights, input and hidden activations are
 * rounded to bf16 (nearest even), biases and accumulation are float32.
 * feat is read as in legs_decode_mlp; mlp_flags as there (0 = Eq. 8 as
 * written). Outputs (each nullable, at least one): probs [P][N] float32
 * (16-byte aligned), probs_f16 [P][N] IEEE half (16-byte aligned; the same
 * probabilities rounded to nearest, the input of legs_language_features),
 * top1 [P] int32 (lowest index on ties). With only top1 requested the kernel
 * never holds all N logits. */
int64_t legs_dmlp_param_count(int32_t N);
int32_t legs_decode_dmlp(legs_ctx *ctx, const float *feat, int64_t P, int64_t c_stride, int64_t p_stride,
                         const float *params, int32_t N, int32_t mlp_flags, float *probs, uint16_t *probs_f16,
                         int32_t *top1, void *stream);

/* Language feature map F = M_infer S (supplementary inference equation):
 * probs_f16 [P][N] the half-precision distribution from legs_decode_dmlp
 * (16-byte aligned), S [N][d] float32 the quantised language features (the
 * discrete feature space), d a multiple of 32 up to 4096. F is written planar,
 * F[c * P + p] for feature dimension c and pixel p, as float32 (out_f16 = 0)
 * or IEEE half (out_f16 = 1). S is rounded to half inside (|S| < 65504);
 * products are accumulated in float32 on FP16 MFMA. */
int32_t legs_language_features(legs_ctx *ctx, const uint16_t *probs_f16, int64_t P, int32_t N,
                               const float *S, int32_t d, int32_t out_f16, void *F, void *stream);

/* Quantisation of K hybrid language features into the discrete feature space
 * S (Sec. 3.3) and its optimisation objective:
 *   D_ij = cos(F_i^CLIP, f_j^CLIP) + lambda_dino cos(F_i^DINO, f_j^DINO)  (Eq. 4)
 *   index_i = argmax_j D_ij (lowest j on ties); F^_i = f_index_i         (Eq. 5)
 *   L_cos = mean_i [(1 - cos(F_i^C, F^_i^C)) + lambda_dino (1 - cos(F_i^D, F^_i^D))]  (Eq. 6)
 *   r = histogram(index) / K, p = mean_i softmax_j(D_ij), L_lb = sum_j r_j p_j
 *                                            (Eq. 7, supplementary load balancing)
 *   L_q = lambda_cos L_cos + lambda_lb L_lb
 * feat [K][d] IEEE half (16-byte aligned, K >= 1), columns [0, d_clip) the CLIP part
 * and [d_clip, d) the DINO part; S [N][d] float32 (16-byte aligned), rounded
 * to half for every use; N 32, 64 or 128; d and d_clip multiples of 128
 * (d <= 8192). Outputs (overwritten): index [K] int32, counts [N] uint32 (the
 * histogram, r = counts / K), prob_mean [N] float32 (p; nullable), losses [3]
 * float32 = (L_cos, L_lb, L_q) (nullable), grad [N][d] float32 = dL_q/dS
 * (nullable: no gradient pass), straight through the half rounding of S;
 * the index and r are piecewise constant (no gradient). A zero part of a
 * feature or code has cosine 0. workspace: legs_quantize_workspace_bytes(K,
 * N, d) bytes (16-byte aligned). Dot products accumulate in float32 on FP16
 * MFMA; features whose two best distances lie within float32 rounding of each
 * other may take either index. */
int64_t legs_quantize_workspace_bytes(int64_t K, int32_t N, int32_t d);
int32_t legs_quantize(legs_ctx *ctx, const uint16_t *feat, int64_t K, int32_t d, int32_t d_clip,
                      const float *S, int32_t N, float lambda_dino, float lambda_cos, float lambda_lb,
                      void *workspace, int32_t *index, uint32_t *counts, float *prob_mean, float *losses,
                      float *grad, void *stream);

/* Adaptive spatial smoothing of the semantic features (Sec. 3.4.2, Eqs.
 * 13-14, Table 4): s_MLP = MLP(PE(p)) with PE configuration 0 (the position
 * itself) and MLP 3 -> 128 -> 128 -> 128 -> 8 (ReLU after the first three
 * layers), and
 *   L_smo = lambda_smo mean_g [ |s_MLP - s_G*| + max(u_G*, w_s) |s_MLP* - s_G| ]
 * (unsquared Euclidean norms, * = stop gradient). mean [n][3] are the
 * Gaussian positions (inputs only: this loss moves no position), channels
 * [n][C] the per-Gaussian channels with s_G at [sem_channel, sem_channel + 8)
 * and u at u_channel. params: float32 masters [legs_smooth_param_count()]
 * packed W1 [128][3], b1 [128], W2 [128][128], b2, W3 [128][128], b3,
 * W4 [8][128], b4 [8]; weights and hidden activations are rounded to bf16,
 * the position enters unrounded, accumulation is float32 (the backward's
 * upstream gradients are carried as two bf16 parts, 16 significant bits).
 * Accumulates (+=): loss [1] += L_smo, grad [legs_smooth_param_count()] +=
 * dL_smo/dparams, d_channels [n][C] += dL_smo/ds_G in the s_G columns (u gets
 * no gradient). A Gaussian with s_MLP = s_G adds nothing. workspace:
 * legs_smooth_workspace_bytes(n) bytes (16-byte aligned), which on return
 * holds the bf16 hidden activations of the forward pass: with Gp = n rounded
 * up to a multiple of 64, a 16-row input plane (16 Gp bf16) and then the
 * planes of h1, h2 and h3 (128 Gp bf16 each), followed by the backward's
 * pre-activation gradients of layers 1-3 and of the output layer, each as a
 * hi and a lo bf16 plane. A plane of R rows is in MFMA operand order:
 * [Gp / 16][ceil(R / 32)][2][min(R, 32)][8], i.e. Gaussian g, row r at
 * (g / 16, r / 32, (g / 8) % 2, r % 32, g % 8); the padding Gaussians are
 * zero in the input and hidden planes. */
int64_t legs_smooth_param_count(void);
int64_t legs_smooth_workspace_bytes(int64_t n);
int32_t legs_smooth_loss_grad(legs_ctx *ctx, const float *mean, const float *channels, int32_t C,
                              int32_t sem_channel, int32_t u_channel, int64_t n, const float *params,
                              float w_s, float lambda_smo, void *workspace, float *grad, float *d_channels,
                              float *loss, void *stream);

/* Gradient of the mean cross-entropy (Eq. 9) of B pixels against labels
 * [B] int32 in [0, K): grad [legs_mlp_param_count(K)] is overwritten, loss [1]
 * receives the mean loss. Straight-through for the bf16 roundings.
 * workspace: legs_mlp_workspace_bytes(B, K) bytes of device memory. */
int64_t legs_mlp_workspace_bytes(int64_t B, int32_t K);
int32_t legs_mlp_grad(legs_ctx *ctx, const float *feat, int64_t B, int64_t c_stride,
                      int64_t p_stride, const int32_t *labels, int32_t K, int32_t mlp_flags,
                      const float *params, void *workspace, float *grad, float *loss, void *stream);

/* Semantic loss of Sec. 3.4.2 over the P pixels of one view (Eqs. 10-12):
 *   L_CE = sum_px CE(softmax(D_MLP(R_s)), M) (1 - R_u) / (H W),
 *   L_u  = sum_px R_u / (H W),   L_s = lambda_CE L_CE + lambda_u L_u,
 * with D_MLP the decoder of legs_decode_mlp (same params and mlp_flags),
 * labels = M [P] int32 in [0, K) and inv_hw = 1 / (H W). feat = R_s is read
 * like the decode calls (c_stride, p_stride); ru [P] = R_u (contiguous, e.g.
 * the uncertainty plane of legs_render_forward's output). Writes
 * d_feat = dL_s/dR_s (element (p, c) at d_feat[c * d_c_stride + p * d_p_stride],
 * e.g. into the semantic planes of the d_out handed to legs_render_backward)
 * and d_ru [P] = dL_s/dR_u = (lambda_u - lambda_CE CE_p) / (H W); accumulates
 * (+=) the decoder's parameter gradient into grad [legs_mlp_param_count(K)]
 * and L_s into loss [1] (the caller zeroes both; one call per view).
 * workspace: legs_mlp_workspace_bytes(P, K) bytes. Straight-through for the
 * bf16 roundings. */
int32_t legs_semantic_loss_grad(legs_ctx *ctx, const float *feat, const float *ru, int64_t P,
                                int64_t c_stride, int64_t p_stride, const int32_t *labels,
                                int32_t K, int32_t mlp_flags, const float *params, float lambda_ce,
                                float lambda_u, float inv_hw, void *workspace, float *grad,
                                float *d_feat, int64_t d_c_stride, int64_t d_p_stride, float *d_ru,
                                float *loss, void *stream);

/* legs_semantic_loss_grad without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). It allocates nothing: its
 * workspace is a fixed array of 21,495,808 bytes inside the library's device
 * code, one per GPU, held from the first legs_create on that GPU until the
 * process ends. P <= LEGS_NOALLOC_MAX_PIXELS, else LEGS_ERR_ARG (nothing
 * launched); the loss and the decoder gradient accumulate, so a larger view
 * is processed in chunks of at most that many pixels, each call given the
 * whole view's inv_hw. All calls on one GPU share the array: calls that
 * overlap in time on one GPU (several streams or threads) race and must be
 * serialised by the caller. Arguments and results as legs_semantic_loss_grad. */
#define LEGS_NOALLOC_MAX_PIXELS 16384
int32_t legs_semantic_loss_grad_noalloc(legs_ctx *ctx, const float *feat, const float *ru, int64_t P,
                                        int64_t c_stride, int64_t p_stride, const int32_t *labels,
                                        int32_t K, int32_t mlp_flags, const float *params,
                                        float lambda_ce, float lambda_u, float inv_hw, float *grad,
                                        float *d_feat, int64_t d_c_stride, int64_t d_p_stride,
                                        float *d_ru, float *loss, void *stream);

/* ---- optimisation (Sec. 4: Adam, lr 1e-3, betas (0.9, 0.999)) ------------- */

/* One parameter group of a fused Adam step (all device pointers, n floats).
 * Elements j with clamp_every > 0 and j % clamp_every == clamp_offset are
 * clamped to [clamp_lo, clamp_hi] after the update (the uncertainty u in [0, 1]
 * of Sec. 3.4.2 stored as a channel column). */
typedef struct {
    float *param;
    const float *grad;
    float *m, *v;
    int64_t n;
    int32_t clamp_every, clamp_offset;
    float clamp_lo, clamp_hi;
} legs_adam_group;
#define LEGS_ADAM_MAX_GROUPS 8

/* m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps); one launch
 * over every group (groups is a host array of n_groups <= 8). The betas are
 * doubles: 1 - b and the bias corrections are formed in double and rounded
 * once to float (so b2 = 0.999 gives 1 - b2 = float(0.001)). */
int32_t legs_adam(legs_ctx *ctx, const legs_adam_group *groups, int32_t n_groups, int32_t step,
                  float lr, double beta1, double beta2, float eps, void *stream);

/* One decoder training step: legs_mlp_grad, then legs_adam on params with
 * moment buffers m, v [legs_mlp_param_count(K)]; grad is scratch. */
int32_t legs_mlp_train_step(legs_ctx *ctx, const float *feat, int64_t B, int64_t c_stride,
                            int64_t p_stride, const int32_t *labels, int32_t K, int32_t mlp_flags,
                            float *params, float *m, float *v, float *grad, int32_t step, float lr,
                            double beta1, double beta2, float eps, void *workspace, float *loss,
                            void *stream);

/* Per view: mean |out - target| over the first n_fit channels (RGB and s_G)
 * plus lambda_u times the mean of the remaining channels (R_u, Eq. 11),
 * summed over views. Writes d_out = dL/d(out) (planar like out) and the loss
 * into loss [1] (overwritten). */
int32_t legs_l1_loss_grad(legs_ctx *ctx, const float *out, const float *target,
                          const legs_view *views_dev, int32_t n_views, int64_t total_pixels,
                          int32_t C, int32_t n_fit, float lambda_u, float *d_out, float *loss,
                          void *stream);

/* Zero `bytes` bytes (a multiple of 4, 4-byte aligned) of device memory with a
 * kernel (a kernel node under graph capture, never a memset node): clears the
 * accumulated (+=) gradient outputs of legs_render_backward and
 * legs_project_backward before a step. LEGS_ERR_ARG on a bad size or
 * pointer. */
int32_t legs_clear(legs_ctx *ctx, void *dev, int64_t bytes, void *stream);

/* ---- runtime: graph capture and autotuning -------------------------------- */

typedef struct legs_graph legs_graph;
/* Begin capturing the work the caller enqueues on `stream` (not the legacy
 * default stream) into a HIP graph. Every call above is capturable when
 * legs_bin_sort runs with host_count == NULL (sizes are then read on device).
 * Buffers referenced during capture must stay allocated while the graph lives. */
int32_t legs_capture_begin(legs_ctx *ctx, void *stream);
/* End the capture and instantiate the graph. */
int32_t legs_capture_end(legs_ctx *ctx, void *stream, legs_graph **out);
int32_t legs_graph_launch(legs_ctx *ctx, legs_graph *graph, void *stream);
int32_t legs_graph_destroy(legs_graph *graph);

/* Time one full step (project, bin/sort, forward, and when d_out != NULL the
 * backward through legs_project_backward) for tile in {8, 16, 32} x
 * lds_batch in {64, 128, 256}, averaged over `reps` after one warm-up, and
 * return the fastest options in *best (other fields copied from *base).
 * ms_table (nullable) receives the nine times, tile-major. Set-up call: it
 * allocates and frees its own device buffers and waits on `stream`. Images are
 * identical for every setting, so only speed depends on the choice. */
int32_t legs_autotune(legs_ctx *ctx, const float *mean, const float *log_scale, const float *quat,
                      const float *opacity_logit, const float *channels, int64_t n, int32_t C,
                      const legs_camera *cams_host, int32_t n_views, const legs_opts *base,
                      const float *d_out, int32_t reps, legs_opts *best, float *ms_table,
                      void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LEGS_H */
