/*
 * r360.h -- C ABI of the MI355X (gfx950) hot path of 360Roam's
 * geometry-aware radiance fields (arXiv 2208.02705).
 *
 * The path: equirect (or pinhole) ray generation (Sec. 3.2, Eq.2/Eq.3) ->
 * sampling of the occupied voxels of an occupancy grid along each ray
 * (Sec. 4.2, Sec. 5) -> routing of each sample to the local radiance field
 * that owns its voxel (Sec. 5, Alg.1 Stage II labels) -> positional encoding
 * plus that field's tiny MLP (Sec. 3.1 Eq.1, App. C) -> alpha compositing
 * (Sec. 3.2, Eq.4/Eq.5); and its backward pass for fine-tuning with an L2
 * photometric loss and Adam (Sec. 4.2, Sec. 6.3).
 *
 * Conventions
 *  - Every pointer argument is a DEVICE pointer unless its name ends in
 *    _host. Arrays are caller-owned; the library never frees or reallocates
 *    them. Ray and per-ray arrays are structure-of-arrays: o and d are [3][N]
 *    (all x, then all y, then all z); rgb is [3][N].
 *  - `stream` is a hipStream_t passed as void*; every call only enqueues work
 *    on it (asynchronous), except where a _host output forces a wait.
 *  - Transient memory is a caller-supplied workspace of at least
 *    r360_workspace_bytes() bytes, 256-byte aligned. A render leaves its sample
 *    lists in the workspace; r360_backward() reads them, so the same
 *    workspace must be passed unchanged between the two.
 *  - The library owns only the opaque objects it creates (scene, equirect
 *    tables); their destroy calls free them.
 *  - Every entry point returns r360_status. Argument checks run before any
 *    launch; a failed check launches nothing. Launch failures return
 *    R360_EHIP and r360_last_error() gives the runtime's text. Nothing aborts
 *    across this boundary.
 *  - Sizes: N <= 2^30 and ceil(N / 64) * 64 * max_samples (the sample slots
 *    of the call) below 2^30 per call (split larger ray sets into chunks);
 *    max_samples is in [1, 256]; n_fields in [1, 16384].
 *  - Calls that share a workspace or a scene must not overlap on different
 *    streams.
 */
#ifndef R360_H
#define R360_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    R360_OK = 0,
    R360_EINVAL = -1,        /* bad argument (null pointer, size out of range, misaligned) */
    R360_ENOMEM = -2,        /* device allocation failed (scene / table creation only) */
    R360_EHIP = -3,          /* a HIP runtime call or launch failed */
    R360_EUNSUPPORTED = -4,  /* valid but unsupported configuration (e.g. encoding length) */
    R360_EWORKSPACE = -5     /* workspace smaller than r360_workspace_bytes() */
} r360_status;

typedef enum {
    R360_FP32 = 0,           /* MLP layers on FP32 MFMA (v_mfma_f32_16x16x4f32) */
    R360_BF16 = 1,           /* MLP layers on BF16 MFMA, FP32 accumulation */
    R360_FP16 = 2,           /* MLP layers on FP16 MFMA, FP32 accumulation */
    R360_FP64_GRADCHECK = 3  /* scalar FP64 kernels; only r360_gradcheck_* accept it */
} r360_precision;

/* Occupancy grid: n[0] x n[1] x n[2] voxels of edge `voxel` (a power of two)
 * from corner lo; voxel (i, j, k) is element i + n0 (j + n1 k) (x fastest);
 * each n[a] in [1, 4096] and fewer than 2^31 voxels in all. A voxel is
 * occupied where its probability is strictly above `threshold` (Sec. 4.1). */
typedef struct {
    int32_t n[3];
    float lo[3];
    float voxel;
    float threshold;
} r360_grid_desc;

/* Local fields (App. C tiny network, widened per the config): per field
 * h1 = relu(W1 g(x) + b1); h2 = relu(W2 h1 + b2); sigma = softplus(ws h2 + bs);
 * f = Wf h2 + bf; h3 = relu(W3 [f ; g(d)] + b3); rgb = sigmoid(W4 h3 + b4),
 * with g the positional encoding of Sec. 3.1 (identity term included, 3 + 6L
 * wide). The encoding input is xhat = (p - center) * (1 / half_extent).
 * Supported: hidden in {32, 64}, L_xyz = 10, L_dir = 4. */
typedef struct {
    int32_t n_fields;
    int32_t hidden;
    int32_t L_xyz;
    int32_t L_dir;
    float center[3];
    float half_extent;
} r360_mlp_desc;

/* Per-call options. Samples lie in [near, far] along unit-length d;
 * far may be +inf. At most max_samples occupied-voxel samples per ray,
 * nearest first. `precision` is an r360_precision. samples_per_voxel k in
 * [0, 64] (0 reads as 1): each occupied segment [t_in, t_out) is cut at
 * b_j = fma(j, (t_out - t_in) / k, t_in), 0 < j < k (b_0 = t_in, b_k =
 * t_out), and every piece gives a sample t_mid = (b_j + b_j+1) / 2, delta =
 * b_j+1 - b_j (FP32, as written); k = 1 is the single midpoint sample. The
 * pieces count against max_samples.
 *
 * Early ray termination (renders only; the tolerance-bounded form of the
 * stopping rule for volume rendering that the related work of Sec. 2 names):
 * term_eps > 0 stops a ray after its first term_after samples when its
 * transmittance exp(-sum sigma delta) there is below term_eps; rays above it
 * continue with their remaining samples, and their result is the same as
 * without termination. A stopped ray differs from the full result by less
 * than term_eps in each colour channel and in opacity (the weights it drops
 * sum to less than its transmittance). term_eps = 0 disables it; otherwise
 * term_eps <= 1 and 1 <= term_after < max_samples. With termination the
 * render runs in two passes and synchronises the stream once between them
 * (to read how many rays continue), so such a render cannot be captured
 * into a HIP graph; training, sampling and the gradient checks reject it. */
typedef struct {
    float near_;
    float far_;
    int32_t max_samples;
    int32_t precision;
    int32_t samples_per_voxel;
    float term_eps;
    int32_t term_after;
} r360_render_opts;

typedef struct r360_scene r360_scene;
typedef struct r360_equirect r360_equirect;

/* Number of FP32 parameters of one local field in canonical order:
 * W1[h x 63], b1[h], W2[h x h], b2[h], ws[1 x h], bs[1], Wf[h x h], bf[h],
 * W3[h x (h + 27)], b3[h], W4[3 x h], b4[3]  (matrices row-major [out x in],
 * W3's input order [f ; g(d)]). 6212 for h = 32 (App. C), 18564 for h = 64. */
int64_t r360_field_params(int32_t hidden, int32_t L_xyz, int32_t L_dir);

/* Create a scene on the current device: takes the occupancy decision and the
 * voxel -> field labels (Sec. 5: each occupied voxel is labelled with its
 * tiny MLP) from occ_prob [n2][n1][n0] and field_map (same layout, -1 = none)
 * into a library-owned label grid, and packs `weights` ([n_fields][P] FP32,
 * canonical order, device) into the per-precision MFMA fragment layouts.
 * The inputs are read during the call (on `stream`) and may be freed after
 * the stream has passed this point. Errors: EINVAL, EUNSUPPORTED, ENOMEM, EHIP. */
r360_status r360_scene_create(const r360_grid_desc* grid, const float* occ_prob, const int32_t* field_map,
                              const r360_mlp_desc* mlp, const float* weights, void* stream, r360_scene** out);

/* Re-pack new FP32 canonical weights (e.g. after an optimizer step). */
r360_status r360_scene_set_weights(r360_scene* scene, const float* weights, void* stream);

/* Replace the occupancy decision and labels (same grid shape). */
r360_status r360_scene_set_grid(r360_scene* scene, const float* occ_prob, const int32_t* field_map, void* stream);

void r360_scene_destroy(r360_scene* scene);

/* Per-resolution sine/cosine tables for equirect rays (Eq.2 inverted at
 * pixel centres, Eq.3): phi = pi a_phi with a_phi = ((2u+1) - W)/W and
 * theta = pi a_theta with a_theta = (H - (2v+1))/(2H), each a correctly
 * rounded FP32 quotient; sin/cos are evaluated in FP64 on the host and
 * rounded once to FP32, then uploaded (synchronous). */
r360_status r360_equirect_create(int32_t W, int32_t H, r360_equirect** out);
void r360_equirect_destroy(r360_equirect* eq);
/* Copy the tables to host arrays (W, W, H, H floats) for inspection. */
r360_status r360_equirect_tables(const r360_equirect* eq, float* sin_phi_host, float* cos_phi_host,
                                 float* sin_theta_host, float* cos_theta_host);

/* Ray directions for pixels of an equirect camera (Eq.3, camera frame
 * x right, y down, z forward), rotated by the 3x4 row-major camera-to-world
 * c2w_host (d = R d_cam as fma(R2, z, fma(R1, y, R0 x))); o = c2w translation.
 * pix: N linear pixel indices v * W + u (int64), or NULL for all W*H pixels
 * in raster order (then N must equal W*H). Outputs o, d: [3][N]. */
r360_status r360_equirect_rays(const r360_equirect* eq, const float c2w_host[12], const int64_t* pix, int64_t N,
                               float* o, float* d, void* stream);

/* Omni-directional stereo (the stereoscopic mode of Sec. 5, for panoramas):
 * the rays of one eye. Directions as r360_equirect_rays; the origin of pixel
 * (u, v) lies on the viewing circle of radius |eye_offset| around the camera
 * centre, across the ray's horizontal heading: camera-frame offset
 * (eye_offset cos(phi), 0, -eye_offset sin(phi)), world o_i = t_i +
 * fma(R_i2, oz, fma(R_i1, oy, R_i0 ox)). eye_offset = +ipd/2 for the right
 * eye, -ipd/2 for the left; 0 gives r360_equirect_rays exactly. */
r360_status r360_ods_rays(const r360_equirect* eq, const float c2w_host[12], float eye_offset, const int64_t* pix,
                          int64_t N, float* o, float* d, void* stream);

/* Pinhole viewport rays (the perspective views of r360_render_pinhole):
 * pixel (u, v) in raster order, x = ((u + 1/2) - W/2) / fx, y = ((v + 1/2) -
 * H/2) / fy, d_cam = (x, y, 1) / n with n the correctly rounded sqrt of
 * fma(x, x, fma(y, y, 1)), rotated by c2w_host as for r360_equirect_rays;
 * o = c2w translation. Outputs o, d: [3][W*H] (device, written). */
r360_status r360_pinhole_rays(int32_t W, int32_t H, float fx, float fy, const float c2w_host[12], float* o,
                              float* d, void* stream);

/* Workspace bytes for r360_render_* / r360_sample_rays / r360_backward over
 * N rays with the given max_samples (the capacity is N * max_samples). */
size_t r360_workspace_bytes(const r360_scene* scene, int64_t n_rays, int32_t max_samples);

/* Occupied-voxel sampling only (Sec. 4.2 dense sampling of occupied voxels,
 * Sec. 5 ray casting): per ray, traverse the voxels between
 * t0 = max(near, box entry) and t1 = min(far, box exit) in FP32 and emit one
 * sample per occupied voxel segment of positive length: t_mid = (t_in +
 * t_out) / 2, delta = t_out - t_in (or samples_per_voxel pieces of it),
 * nearest max_samples first. Outputs in
 * ray-major order; caller arrays hold N * max_samples entries; voxel may be
 * NULL. ray_offset [N+1] (int32) gets the exclusive prefix of per-ray counts.
 * If n_samples_host is not NULL the call waits for the stream and stores the
 * total there. */
r360_status r360_sample_rays(const r360_scene* scene, const float* o, const float* d, int64_t N,
                             const r360_render_opts* opts, int64_t* n_samples_host, float* t_mid, float* delta,
                             int32_t* ray_id, int32_t* field_id, int32_t* voxel, int32_t* ray_offset,
                             void* ws, size_t ws_bytes, void* stream);

/* Full render of N rays: sampling, routing by field, encoding + field MLP in
 * opts->precision, compositing (Eq.4/Eq.5 with log-space FP32 transmittance,
 * no background). Outputs rgb [3][N], depth [N] (sum of w t_mid, not
 * normalised), opacity [N] (sum of w = 1 - T_final). */
r360_status r360_render_rays(const r360_scene* scene, const float* o, const float* d, int64_t N,
                             const r360_render_opts* opts, float* rgb, float* depth, float* opacity,
                             void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): r360_render_rays with its
 * workspace in a library-owned device array of R360_NOALLOC_SCRATCH_BYTES
 * (128 MiB) per GPU instead of a caller workspace. It calls no hipMalloc,
 * hipFree or allocating library routine; the array is set aside when the
 * library's code is loaded on a device and stays there until the process
 * ends. Each call carves it as a render-only workspace:
 * 36 B per sample slot (ceil(N / 64) * 64 * max_samples slots), 28 B per ray,
 * 4 * n_fields * W B of per-wave field counts (W = 8192 for up to 512
 * fields, halved while W * n_fields exceeds 4 Mi and W > 256) and a few KB;
 * a call that needs more returns R360_EWORKSPACE with the bytes it needs
 * (split the rays into smaller calls; the room scene's 141 fields leave
 * room for about 3.4 M slots, e.g. 53,000 rays at max_samples 64). Early ray
 * termination (term_eps > 0) is not offered here: it waits on the stream
 * between its passes (R360_EUNSUPPORTED). Arguments, outputs and errors
 * otherwise as r360_render_rays; the stream must belong to the current
 * device. Every call on one GPU uses that GPU's one array and overwrites
 * what the last call left there: calls that overlap on one GPU (different
 * streams, or host threads without ordering) race and give wrong results;
 * calls in order on one stream do not. */
#define R360_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
r360_status r360_render_rays_noalloc(const r360_scene* scene, const float* o, const float* d, int64_t N,
                                     const r360_render_opts* opts, float* rgb, float* depth, float* opacity,
                                     void* stream);

/* Render a whole equirect view (W*H rays from the table's resolution) from
 * camera c2w_host. Outputs [3][H][W], [H][W], [H][W]. */
r360_status r360_render_equirect(const r360_scene* scene, const r360_equirect* eq, const float c2w_host[12],
                                 const r360_render_opts* opts, float* rgb, float* depth, float* opacity,
                                 void* ws, size_t ws_bytes, void* stream);

/* Render one eye of an omni-directional stereo pair (rays as r360_ods_rays);
 * otherwise as r360_render_equirect. */
r360_status r360_render_ods(const r360_scene* scene, const r360_equirect* eq, const float c2w_host[12],
                            float eye_offset, const r360_render_opts* opts, float* rgb, float* depth,
                            float* opacity, void* ws, size_t ws_bytes, void* stream);

/* Render a pinhole viewport: d_cam = (x, y, 1)/|.| with x = ((u + 1/2) - W/2)/fx,
 * y = ((v + 1/2) - H/2)/fy (correctly rounded sqrt of fma(x,x,fma(y,y,1))). */
r360_status r360_render_pinhole(const r360_scene* scene, int32_t W, int32_t H, float fx, float fy,
                                const float c2w_host[12], const r360_render_opts* opts, float* rgb, float* depth,
                                float* opacity, void* ws, size_t ws_bytes, void* stream);

/* Backward of the most recent r360_render_rays on this workspace (same
 * scene, rays and opts): from dL/dC (grad_rgb [3][N]) recompute per-ray
 * transmittance and partial colours (nothing per-sample is kept from the
 * compositing forward), then dL/dsigma_i = delta_i [T_{i+1} (c_i . g) -
 * ((C - C_{<=i}) . g)] and dL/dc_i = w_i g, then the field MLPs' backward in
 * opts->precision with FP32 accumulation. grad_weights [n_fields][P] (FP32,
 * canonical order) is overwritten. */
r360_status r360_backward(const r360_scene* scene, const float* o, const float* d, int64_t N,
                          const r360_render_opts* opts, const float* grad_rgb, float* grad_weights,
                          void* ws, size_t ws_bytes, void* stream);

/* One fine-tuning step (Sec. 4.2, L2 photometric loss): render the N rays,
 * loss = 1/(3N) sum (C - C*)^2 into loss[0] (device), its gradient w.r.t. all
 * field weights into grad_weights (overwritten); rgb_out [3][N] may be NULL. */
r360_status r360_train_step(const r360_scene* scene, const float* o, const float* d, int64_t N,
                            const float* target_rgb, const r360_render_opts* opts, float* loss,
                            float* grad_weights, float* rgb_out, void* ws, size_t ws_bytes, void* stream);

/* Learning-rate schedule of the fine-tuning (Sec. 6.3: exponential decay
 * from lr0 to lr1): lr0 (lr1 / lr0)^(min(step, total) / max(total, 1)),
 * evaluated in FP64 on the host; lr0, lr1 > 0, step >= 0. Returns the rate to
 * pass to r360_adam_step (NaN for invalid arguments). */
double r360_lr_schedule(int64_t step, int64_t total, double lr0, double lr1);

/* Adam (Sec. 6.3: beta1 0.9, beta2 0.99): m = b1 m + (1-b1) g;
 * v = b2 v + (1-b2) g^2; w -= lr (m/(1-b1^step)) / (sqrt(v/(1-b2^step)) + eps).
 * FP32 master weights, in place. step >= 1. */
r360_status r360_adam_step(float* w, const float* g, float* m, float* v, int64_t n, int64_t step, float lr,
                           float beta1, float beta2, float eps, void* stream);

/* FP64 gradient-check forms (FP64 only here): the same sampling, then scalar
 * FP64 encoding, field MLP and compositing over FP64 canonical weights
 * weights64 [n_fields][P]. Forward writes rgb64 [3][N]; backward takes
 * grad_rgb64 [3][N] and overwrites grad64 [n_fields][P]. The forward leaves
 * its samples in ws for the backward, as r360_render_rays does. */
r360_status r360_gradcheck_forward(const r360_scene* scene, const double* weights64, const float* o,
                                   const float* d, int64_t N, const r360_render_opts* opts, double* rgb64,
                                   void* ws, size_t ws_bytes, void* stream);
r360_status r360_gradcheck_backward(const r360_scene* scene, const double* weights64, const float* o,
                                    const float* d, int64_t N, const r360_render_opts* opts,
                                    const double* grad_rgb64, double* grad64, void* ws, size_t ws_bytes,
                                    void* stream);

/* Global omnidirectional field stage (Sec. 3.2 360NeRF; architecture table
 * of App. C), the density source of Sec. 4.1's occupancy estimation:
 * n_samples samples per ray uniform in inverse depth over [near, far]
 * (t_k = 1 / fma(s_k, 1/far, (1 - s_k)/near), s_k = k/(n_samples - 1);
 * delta_k = t_{k+1} - t_k, the last 0), xhat = (fma(t, d, o) - center) /
 * half_extent, encoding L = 10 / 4, eight ReLU layers of `width` with the
 * encoding concatenated again at the fifth (the eighth linear), sigma =
 * relu(ws h8 + bs), f = relu(Wf h8 + bf), colour sigmoid(W11 relu(W10 [f ;
 * g(d)] + b10) + b11), compositing as Eq.4/Eq.5. Weights: FP32 canonical
 * order W1 b1 ... W8 b8 ws bs Wf bf W10 b10 W11 b11 (W5 input [h4 ; g(x)]).
 * The occupancy grid (grid_n, grid_lo, voxel) receives the per-sample max of
 * sigma over the samples inside each cell. */
typedef struct {
    int32_t width;          /* 256 in the paper's table */
    int32_t color_width;    /* 128 */
    int32_t n_samples;      /* samples per ray, >= 2 */
    float near_, far_;
    float center[3];
    float half_extent;
    int32_t grid_n[3];
    float grid_lo[3];
    float voxel;
} r360_global_desc;

/* Canonical parameter count (595,844 at width 256, colour width 128). */
int64_t r360_global_params(int32_t width, int32_t color_width);
size_t r360_global_workspace_bytes(const r360_global_desc* desc, int64_t n_rays);

/* Forward (BF16 MFMA GEMMs, FP32 accumulation) over N rays [3][N]; writes
 * rgb_out [3][N] and depth_out [N] if not NULL; folds max(sigma) into
 * occ_grid [n2][n1][n0] (FP32, caller-initialised; NULL skips): each cell
 * becomes max(cell, sigma) over the samples whose position lies in it
 * (sigma >= 0 always; a cell may start at any non-NaN value, e.g. 0 or a
 * negative sentinel, and is replaced by the first sample's density). With
 * target_rgb [3][N] also the loss (loss[0], L = 1/(3N) sum (C - C*)^2) and
 * its gradient w.r.t. all weights, grad [P] FP32 (overwritten). Sizes: width
 * and color_width multiples of 32; 1 <= N * n_samples < 2^31. */
r360_status r360_global_field_step(const r360_global_desc* desc, const float* weights, const float* o,
                                   const float* d, int64_t N, const float* target_rgb, float* loss, float* grad,
                                   float* rgb_out, float* depth_out, float* occ_grid, void* ws, size_t ws_bytes,
                                   void* stream);

/* Stage I of Alg.1 (Sec. 4.1): progressive probabilistic occupancy.
 *
 * Measurement of one ray from its samples' Eq.5 weights w_i: opacity A =
 * sum w_i, depth D = sum w_i t_i / A (the Eq.4 depth over normalised
 * weights), uncertainty U = sqrt(sum w_i (t_i - D)^2 / A); A = 0 gives D =
 * U = 0.
 *
 * Update for one sampling position (the logit form of Eq.6, one measurement
 * per voxel per call): each ray with A >= min_opacity and finite D, U >= 0
 * walks its voxels with the sampler's FP32 traversal over [max(near, box
 * entry), min(far, box exit)]. A voxel segment of positive length ending at
 * or before D - U is a free pass; the voxel whose segment [t_in, t_out)
 * holds D is the hit, with logit l_hit / (1 + U / voxel), and ends the walk.
 * Per voxel: l += the largest hit logit of the rays ending in it, else
 * l_miss if a ray passed freely, then clamp to [l_min, l_max] (Sec. 4.1:
 * -2 and 3.5); voxels without a measurement keep their value. Deterministic
 * (independent of ray order). */
typedef struct {
    int32_t n[3];           /* voxels per axis, each in [1, 4096], < 2^31 in total */
    float lo[3];            /* grid lower corner */
    float voxel;            /* voxel edge, a power of two */
    float near_, far_;      /* ray clip, 0 <= near < far (far may be +inf) */
    float l_hit;            /* > 0: logit of a sharp hit (logit(0.7) by default) */
    float l_miss;           /* < 0: logit of a free pass (logit(0.4) by default) */
    float l_min, l_max;     /* clamp, l_min < l_max (-2 and 3.5 in the paper) */
    float min_opacity;      /* rays below this opacity measure nothing */
} r360_occ_desc;

/* Fill an update description from sensor probabilities: l_hit =
 * logit(p_hit), l_miss = logit(p_miss) (logit(p) = log(p / (1 - p)), FP64
 * rounded to FP32), clamp [l_min, l_max] and the other fields as given
 * (n and lo the same on every axis). The customary OctoMap sensor model is
 * p_hit = 0.7, p_miss = 0.4 with the paper's clamp -2, 3.5. Returns
 * R360_EINVAL unless 1/2 < p_hit < 1 and 0 < p_miss < 1/2. */
r360_status r360_occ_desc_init(r360_occ_desc* desc, int32_t n, float lo, float voxel, float near_, float far_,
                               double p_hit, double p_miss, float l_min, float l_max, float min_opacity);

/* Per-ray depth, uncertainty and opacity ([N] each, device, written) from
 * dense samples t, delta, sigma ([N][S] ray-major, device, read). N >= 1,
 * N <= 2^31, S >= 1. */
r360_status r360_depth_uncertainty(const float* t, const float* delta, const float* sigma, int64_t N, int32_t S,
                                   float* depth, float* uncert, float* opacity, void* stream);

/* Device workspace (bytes, 256-byte aligned base) of one update: 5 bytes per
 * voxel, rounded up; 0 for an invalid description. */
size_t r360_occupancy_workspace_bytes(const r360_occ_desc* desc);

/* One pose's update of the FP32 logit grid logit [n2][n1][n0] (device, read
 * and written in place) from N rays o, d [3][N] and their measurement depth,
 * uncert, opacity [N] (device). prob [n2][n1][n0] (device, may be NULL)
 * receives 1 / (1 + exp(-l)) for every voxel, ready for r360_scene_create
 * with threshold 0.97. Caller-owned memory throughout; the workspace holds
 * the per-voxel marks and is overwritten. */
r360_status r360_occupancy_update(const r360_occ_desc* desc, float* logit, float* prob, const float* o,
                                  const float* d, int64_t N, const float* depth, const float* uncert,
                                  const float* opacity, void* ws, size_t ws_bytes, void* stream);

/* The global field's Stage I measurement: its forward over N rays (as
 * r360_global_field_step without a target) followed by the per-ray depth,
 * uncertainty and opacity above ([N] each, device). Workspace as
 * r360_global_workspace_bytes. */
r360_status r360_global_field_measure(const r360_global_desc* desc, const float* weights, const float* o,
                                      const float* d, int64_t N, float* depth, float* uncert, float* opacity,
                                      void* ws, size_t ws_bytes, void* stream);

/* Distillation (Sec. 4.2, Eq.7). The global field's density and colour at
 * M given points x [3][M] with view directions dir [3][M] (device), written
 * to sigma [M] and rgb [3][M] (device): the global forward of
 * r360_global_field_step with one sample per point at the point itself
 * (desc's near, far and n_samples are not used). Workspace:
 * r360_global_points_workspace_bytes. */
size_t r360_global_points_workspace_bytes(const r360_global_desc* desc, int64_t M);
r360_status r360_global_field_points(const r360_global_desc* desc, const float* weights, const float* x,
                                     const float* dir, int64_t M, float* sigma, float* rgb, void* ws,
                                     size_t ws_bytes, void* stream);

/* One distillation step of the local fields: with point i (x, dir [3][M]
 * device) owned by field[i] (int32 [M], device; ids outside [0, n_fields)
 * take no part) and its targets target_sigma [M], target_rgb [3][M] (the
 * global field's values), L = sum_k (1/I_k) sum_{i of field k} [(sigma^k_i -
 * target_sigma_i)^2 + |c^k_i - target_rgb_i|^2], I_k the points of field k.
 * Writes loss[0] and grad_weights [n_fields][P] FP32 (overwritten), on the
 * scene's current weights at opts->precision (FP32, BF16 or FP16; near, far
 * and max_samples are not used). Workspace: r360_workspace_bytes(scene, M,
 * 1). 1 <= M <= 2^30. */
r360_status r360_distill_step(const r360_scene* scene, const float* x, const float* dir, const int32_t* field,
                              int64_t M, const float* target_sigma, const float* target_rgb,
                              const r360_render_opts* opts, float* loss, float* grad_weights, void* ws,
                              size_t ws_bytes, void* stream);

/* Per-field encoding frames (a renderer variant: each local field encodes
 * its own region). r360_field_frames computes, for each field f of
 * field_map [n2][n1][n0] (device int32, grid as `grid`), the box of its
 * voxels: per axis box_lo = fma(imin, voxel, lo), box_hi = fma(imax + 1,
 * voxel, lo); centers [F][3] = (box_lo + box_hi) * 0.5 and half_extents [F]
 * the largest (box_hi - box_lo) * 0.5 over the axes (FP32); a field without
 * voxels gets centre 0 and half extent 1. Workspace:
 * r360_field_frames_workspace_bytes(F). r360_scene_set_frames makes every
 * later render, training, distillation and gradient-check call encode a
 * sample of field f as xhat = (p - c_f) * (1 / h_f) (centers [F][3],
 * half_extents [F] > 0, device); NULL centers restores the scene-wide frame
 * of r360_mlp_desc. The scene keeps its own copy. */
size_t r360_field_frames_workspace_bytes(int32_t n_fields);
r360_status r360_field_frames(const r360_grid_desc* grid, const int32_t* field_map, int32_t n_fields, float* centers,
                              float* half_extents, void* ws, size_t ws_bytes, void* stream);
r360_status r360_scene_set_frames(r360_scene* scene, const float* centers, const float* half_extents, void* stream);

/* Stage II of Alg.1 (Sec. 4.2): adaptive field assignment. Occupied voxels
 * are those with occ > threshold (FP32 compare), S of them; field k (0 <= k <
 * n_fields) receives floor(S / n_fields) + (k < S mod n_fields) voxels. For k
 * = 0, 1, ...: the anchor is the unassigned occupied voxel of smallest linear
 * index (x + n0 (y + n1 z): the minimum coordinate, z then y then x); the
 * field takes the unassigned occupied voxels nearest to the anchor (squared
 * distance between voxel indices, ties to the smaller linear index), the
 * anchor first. Writes field_map [n2][n1][n0] (device, int32, -1 for
 * unoccupied voxels), usable directly by r360_scene_create. Synchronises
 * the stream once (to size the loop by S); S is returned in
 * n_occupied_host (may be NULL). Deterministic. */
size_t r360_assign_workspace_bytes(const int32_t n[3]);
r360_status r360_assign_fields(const int32_t n[3], const float* occ, float threshold, int32_t n_fields,
                               int32_t* field_map, int64_t* n_occupied_host, void* ws, size_t ws_bytes,
                               void* stream);

/* The uniform decomposition (the 360Roam-u variant of Sec. 6): blocks[a]
 * blocks per axis (1 <= blocks[a] <= n[a]), voxel index i in block
 * floor(i * blocks[a] / n[a]); the fields are the blocks holding an occupied
 * voxel, numbered in linear block order (x fastest). Writes field_map as
 * above and the number of fields to n_fields_host (synchronises once). */
size_t r360_assign_uniform_workspace_bytes(const int32_t blocks[3]);
r360_status r360_assign_uniform(const int32_t n[3], const float* occ, float threshold, const int32_t blocks[3],
                                int32_t* field_map, int32_t* n_fields_host, void* ws, size_t ws_bytes,
                                void* stream);

/* Optional per-stage timing for benchmarking: when enabled, every entry
 * point records a HIP event pair around each stage of its launch sequence on
 * the call's own stream. Stages: 0 sampling (traversal + scan + compaction), 1 routing,
 * 2 field-MLP forward, 3 compositing, 4 loss (as a launch of its own; the
 * local training step folds it into stages 3 and 5), 5 compositing backward,
 * 6 field-MLP backward (with the per-field gradient reduction), 7 the whole
 * global-field step, 8 the occupancy update (and depth statistics). */
#define R360_NSTAGES 9
r360_status r360_profile_enable(int32_t on);
/* Waits for the recorded events and returns, per stage, the milliseconds and
 * the number of timed launches since the previous read (arrays of
 * R360_NSTAGES); then forgets them. */
r360_status r360_profile_read(double* ms_host, int32_t* count_host);

/* Status text; for R360_EHIP also the runtime's last error text. */
const char* r360_status_string(int32_t status);
const char* r360_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* R360_H */
