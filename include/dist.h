/*
 * dist.h -- C ABI of the MI355X differentiable sphere tracer.
 *
 * The library renders DeepSDF-style implicit signed distance functions with
 * the differentiable sphere tracing of Liu et al., "DIST: Rendering Deep
 * Implicit Signed Distance Function with Differentiable Sphere Tracing"
 * (CVPR 2020, arXiv 1911.13225), and back-propagates image-space losses to
 * the latent codes and decoder weights with the paper's approximate gradient.
 *
 * Conventions (all entry points):
 *   - Every array argument marked "device" is caller-owned GPU memory
 *     (contiguous, row-major, float32 unless stated).  The library never frees
 *     or retains it beyond the call, except dist_submit (see there).
 *   - "host" arrays are read during the call only.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Render calls are
 *     stream-ordered and do not synchronise the host unless stated.
 *   - Return value: DIST_OK (0) on success, DIST_PENDING (1) from dist_poll
 *     when the request is not finished, a negative DIST_E* code on error.
 *     dist_last_error() returns a message for the last error of the calling
 *     thread.
 *   - A context is used by one host thread at a time for fwd/bwd/eval calls;
 *     dist_submit and dist_poll may be called from any thread.
 */
#ifndef DIST_H_
#define DIST_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------- */
#define DIST_OK           0
#define DIST_PENDING      1
#define DIST_EINVAL      (-1)   /* bad argument, shape or parameter                */
#define DIST_ENOMEM      (-2)   /* request exceeds the context's HBM budget        */
#define DIST_EBUSY       (-3)   /* serving queue full                              */
#define DIST_ENOTFOUND   (-4)   /* unknown ticket                                  */
#define DIST_ECANCELLED  (-5)   /* request cancelled or context shut down          */
#define DIST_EHIP        (-6)   /* HIP runtime error                               */
#define DIST_ENUMERIC    (-7)   /* a non-finite signed distance was produced       */

/* ---- per-pixel ray status (output `status`) ------------------------------
 * Termination cases of sphere tracing (paper Alg. 1 and Sec. 3.2):
 *   HIT          |f| < eps at some query: foreground, depth finite.
 *   MISS         the pixel ray does not meet the unit sphere (Sec. 3.2
 *                "Initialization"): background, no queries.
 *   ESCAPED      the ray left the unit sphere while marching: background.
 *   UNCONVERGED  max_steps reached without convergence: background (the
 *                erosion effect of App. A.2).
 *   ERROR        a query returned a non-finite signed distance (NaN or
 *                infinity: the decoder's weights or codes are not finite):
 *                the ray stops, background, no gradient samples; a served
 *                request with such a ray ends with DIST_ENUMERIC.           */
#define DIST_ACTIVE       0
#define DIST_HIT          1
#define DIST_MISS         2
#define DIST_ESCAPED      3
#define DIST_UNCONVERGED  4
#define DIST_ERROR        5

/* ---- precision ----------------------------------------------------------- */
#define DIST_FP32  0   /* every decoder product in float32                       */
#define DIST_BF16  1   /* hidden-layer products with bfloat16 weights/activations
                          and float32 accumulation; layer-0 and skip point terms,
                          biases, the output layer, t and the convergence test
                          stay float32.  Normal queries and the recompute of the
                          backward use DIST_BF16X3, the VJP itself bfloat16.      */
#define DIST_BF16X3 2  /* split bfloat16: x = hi + lo, products hi*hi + lo*hi +
                          hi*lo with float32 accumulation (about 16 significant
                          bits per product, float32-class decoder values)         */

typedef struct dist_ctx dist_ctx;      /* opaque, library-owned */
typedef struct dist_saved dist_saved;  /* opaque, library-owned forward state  */

/* Pinhole camera (OpenCV axes: x right, y down, z forward).  A pixel (u, v)
 * (u = column) is traced through its centre (u + 1/2, v + 1/2); the ray
 * direction is R_wc * K^-1 (u + 1/2, v + 1/2, 1), normalised, and depth is
 * z_c = d / sqrt(xt^2 + yt^2 + 1) with (xt, yt, 1) = K^-1 (x, y, 1)
 * (paper Sec. 3.3).  The camera centre must lie outside the unit sphere. */
typedef struct {
  float fx, fy, cx, cy;
  float R_wc[9];   /* camera-to-world rotation, row-major */
  float c[3];      /* camera centre in world coordinates   */
  int32_t H, W;
} dist_camera;

/* Tracing parameters (paper Sec. 3.2, App. A, App. B.4).
 *   alpha        aggressive-marching factor: t += alpha * f  (paper: 1.5)
 *   eps          convergence threshold: stop when |f| < eps (paper: 5e-5)
 *   normal_delta central-difference step of the normal (Sec. 3.3)
 *   near_, far_  clip range of t; must satisfy near_ <= |c| - 1 and
 *                far_ >= |c| + 1 for every camera (they then never bind)
 *   max_steps    number of marching steps (1..255), coarse steps included
 *   c2f_levels   coarse-to-fine levels L (0..2): tracing starts at
 *                1/2^L resolution per side and splits every ray into four
 *                after every 3 steps; H and W must be multiples of 2^L and
 *                max_steps > 3 L
 *   k_samples    K (1..4): number of minimum-|f| queries per ray that carry
 *                the depth gradient (Sec. 3.4, App. B.4)
 *   precision    DIST_FP32, DIST_BF16 or DIST_BF16X3
 *   want_normals 1 to compute normals (6 float32 queries per hit)
 *   keep_history 1 to keep, in the saved state of dist_render_fwd, the ray
 *                parameter t of every ray at every marching step, which
 *                dist_render_bwd_unrolled needs (4 bytes x max_steps per ray
 *                slot of device memory); 0 otherwise.  dist_submit ignores it. */
typedef struct {
  float alpha, eps, normal_delta, near_, far_;
  int32_t max_steps, c2f_levels, k_samples, precision, want_normals, keep_history;
} dist_trace_params;

/* DeepSDF-style decoder (paper App. B.1): n_layers fully connected layers;
 * layer 0 reads [z, p] (latent_dim + 3 values), layer `skip_layer` (or -1)
 * reads [h, z, p], hidden layers use ReLU and the last layer has width 1.
 * The signed distance is f(p) = 0.5 (|p| - 0.5) + 0.05 tanh(m(z, p)).  A last
 * layer of width 3 makes a colour network (dist_render_color).
 * out_dims: host array of n_layers output widths (last = 1).  Hidden widths
 * up to 512, latent_dim up to 512, n_layers up to 12. */
typedef struct {
  int32_t n_layers;
  int32_t latent_dim;
  int32_t skip_layer;
  const int32_t* out_dims;
} dist_decoder_desc;

/* Create a context.  W[l] and b[l] (host arrays of n_layers device pointers)
 * hold layer l's weights [out][in] and bias [out] in float32; they are copied
 * into the library's packed layouts and not retained.  hbm_budget_bytes caps
 * the device memory the context allocates (0 = no cap).  stream orders the
 * weight packing.  On success *out owns the context until dist_destroy. */
int dist_create(dist_ctx** out, const dist_decoder_desc* desc,
                const float* const* W, const float* const* b,
                size_t hbm_budget_bytes, void* stream);

/* Replace the decoder weights (same shapes as at creation). */
int dist_set_weights(dist_ctx* ctx, const float* const* W, const float* const* b, void* stream);

/* Destroy a context; stops its serving thread and frees its memory.  Any
 * dist_saved created from it must be freed first. */
int dist_destroy(dist_ctx* ctx);

/* Forward render (paper Sec. 3): sphere-trace n_images images, image i
 * being the pair (view pairs[2i], latent pairs[2i+1]).  pairs may be NULL,
 * meaning all n_views x n_latents pairs with image i = (i / n_latents,
 * i % n_latents).  All views must share H and W; 1 <= n_images <= 65535
 * (an image is one row of the per-image launch grids) and H W <= 2^22.
 *   cams     host [n_views]
 *   z        device [n_latents, latent_dim]
 * Outputs (device, caller-owned, each may be NULL), per image [H, W](x3):
 *   depth    z_c, +inf for background                      (Sec. 3.3)
 *   dist     ray distance d of Eq. 1, +inf for background
 *   normal   [H, W, 3] unit normal from central differences, 0 for background
 *   sil      soft silhouette: min|f| - eps along the pixel's ray, or
 *            (distance of the ray from the origin) - 1 for rays that miss
 *            the unit sphere; negative means foreground (Sec. 3.3, App. A.3)
 *   status   uint8 DIST_HIT / DIST_MISS / DIST_ESCAPED / DIST_UNCONVERGED /
 *            DIST_ERROR (the call stays stream-ordered and returns DIST_OK:
 *            a non-finite query is reported per pixel, here)
 *   nsteps   uint8 number of global marching steps taken (0 for MISS)
 *   queries  device int64 [n_images]: decoder queries spent marching
 * saved: if non-NULL receives the state dist_render_bwd needs; the caller
 *   frees it with dist_saved_free.  z must stay unchanged until then.
 * Errors: DIST_EINVAL for bad shapes/parameters, DIST_ENOMEM beyond the
 * budget, DIST_EHIP for runtime failures. */
int dist_render_fwd(dist_ctx* ctx, const dist_camera* cams, int32_t n_views,
                    const float* z, int32_t n_latents,
                    const int32_t* pairs, int32_t n_images,
                    const dist_trace_params* prm,
                    float* depth, float* dist, float* normal, float* sil,
                    uint8_t* status, uint8_t* nsteps, int64_t* queries,
                    dist_saved** saved, void* stream);

/* Backward of a forward render with the paper's approximate gradient
 * (Sec. 3.4, Eq. 2 first term; App. B.2 recompute): given dL/d(depth),
 * dL/d(normal) and dL/d(sil) (device, shaped like the forward outputs, each
 * may be NULL = zero), re-evaluate the decoder at the detached samples -- the
 * K minimum-|f| queries of each hit ray (seed alpha * dL/dz_c / sqrt(xt^2 +
 * yt^2 + 1)), the minimum-|f| query of each ray inside the unit sphere
 * (seed dL/dS * sign f) and the six central-difference points of each hit
 * (seeds +-(I - n n^T) dL/dn / (|n| 2 delta)) -- and accumulate
 *   g_z  device [n_latents, latent_dim]  (overwritten)
 *   g_W, g_b  host arrays of n_layers device pointers shaped like the weights
 *        [out][in] and biases [out] (overwritten); pass both NULL to skip the
 *        weight gradient.  Asking for it synchronises the host once (to size
 *        the per-row capture buffers) and costs roughly one more decoder
 *        pass per sample.
 * The reduction order is fixed, so results are bitwise reproducible. */
int dist_render_bwd(dist_ctx* ctx, const dist_saved* saved,
                    const float* g_depth, const float* g_normal, const float* g_sil,
                    float* g_z, float* const* g_W, float* const* g_b, void* stream);

/* dL/dz as dist_render_bwd, except that the depth term is the exact
 * derivative instead of the paper's approximation (the second term of Eq. 2
 * that Sec. 3.4 drops): a hit's surface point p = c + d v solves f(p, z) = 0,
 * so dd/dz = -(df/dz) / (grad_p f . v) at the Eq. 1 point (one sample per
 * hit, seed -dL/dz_c / |(xt, yt, 1)| / (grad_p f . v)); silhouette and normal
 * terms are the paper's.  Rays that graze the surface (|grad f . v| <= 1e-2
 * |grad f|) get no depth term.  Two passes: grad f . v at the hits, then the
 * backward.  Arguments and errors as dist_render_bwd (no weight gradient). */
int dist_render_bwd_implicit(dist_ctx* ctx, const dist_saved* saved,
                             const float* g_depth, const float* g_normal, const float* g_sil,
                             float* g_z, void* stream);

/* Gradient of the depth and silhouette terms w.r.t. the camera extrinsics
 * of every view (the camera-pose experiment of Sec. 4.1, "Back-Propagation
 * Effectiveness"; App. A.3: the soft silhouette is differentiable w.r.t. the
 * extrinsics).  As for z, the march points are detached (Sec. 3.4): each
 * depth/silhouette sample of the backward above keeps its ray parameter t,
 * and only its position p = c + t R_wc u (u = the pixel's unit direction in
 * the camera frame) moves, adding s grad_p f(p) to dL/dc and
 * s t grad_p f(p) u^T to dL/dR_wc; pixels whose ray misses the unit sphere
 * add dL/dS dS/d(c, R_wc) of S = sqrt(|c|^2 - (c.v)^2) - 1, v = R_wc u.
 * Normal terms are not part of this gradient.
 *   saved    from dist_render_fwd (the latent codes stay fixed)
 *   g_depth, g_sil  device [n_images][H][W] (either may be NULL = zero)
 *   g_cam    device float [n_views][12]: dL/dc (3), then dL/dR_wc (9,
 *            row-major); overwritten.  Views used by no image get zeros.
 * The reduction order is fixed, so results are bitwise reproducible. */
int dist_render_bwd_camera(dist_ctx* ctx, const dist_saved* saved,
                           const float* g_depth, const float* g_sil,
                           float* g_cam, void* stream);

/* Exact dL/dz of the depth and silhouette terms through the unrolled march:
 * Eq. 2 of Sec. 3.4 with both of its terms.  Each query's derivative is its
 * direct part df/dz at the point plus the part through the point,
 * (grad_p f . v) dt/dz, where t accumulates the steps t += alpha f; the
 * result is the derivative of the rendered outputs along the forward's
 * discrete trajectory (its step counts, statuses, minimum-|f| steps and
 * coarse-to-fine decisions held fixed): the depth through Eq. 1 with its
 * residual term (d = t + f at the last query), the silhouette through the
 * minimum-|f| query (dS/dz = sign f df/dz).  A child ray of the coarse-to-fine
 * split passes its dt to its parent unless the clamp into its own unit-sphere
 * interval bound.  Computed in reverse over the marching steps: at each step
 * the decoder is re-evaluated at every ray's point of that step (the
 * recompute of App. B.2) and back-propagated, costing about two decoder
 * passes per march query.
 *   saved    from dist_render_fwd with keep_history = 1 (DIST_EINVAL
 *            otherwise)
 *   g_depth, g_sil  device [n_images][H][W] (either may be NULL = zero)
 *   g_z      device [n_latents, latent_dim]; overwritten
 * Normal terms are not part of this gradient.  The reduction order is fixed,
 * so results are bitwise reproducible. */
int dist_render_bwd_unrolled(dist_ctx* ctx, const dist_saved* saved,
                             const float* g_depth, const float* g_sil,
                             float* g_z, void* stream);

/* Colour rendered jointly with the geometry (Sec. 3.3, "Color and
 * Semantics"; App. C: the texture network has the geometry network's
 * architecture and reads the concatenated shape and texture codes).  A
 * context created with a last layer of width 3 is a colour network; each
 * channel is 0.5 (1 + tanh(m_c)).  It is evaluated at the Eq. 1 point of every
 * hit of a saved geometry render (the points are detached for the backward,
 * as Sec. 3.4 treats the march points).
 *   cctx       colour context (dist_create with out_dims[n_layers-1] = 3); a
 *              geometry entry point given a colour context returns DIST_EINVAL
 *   geom       saved state of dist_render_fwd (another context's)
 *   zc         device [n_latents][latent_dim of cctx]: one code per latent of
 *              the render (e.g. [z_shape, z_tex])
 *   precision  DIST_FP32, or DIST_BF16 (bf16 forward; the backward recomputes
 *              in split bf16 as the geometry's backward does)
 *   rgb        device float [n_images][H][W][3], overwritten; 0 off the hits
 * Calls on one colour context share its buffers: issue them on one stream. */
int dist_render_color(dist_ctx* cctx, const dist_saved* geom, const float* zc,
                      int32_t n_latents, int32_t precision, float* rgb, void* stream);

/* dL/dzc of the colour at the hits: g_rgb device [n_images][H][W][3]
 * (dL/d(colour)); g_zc device [n_latents][latent_dim], overwritten.  Fixed
 * reduction order, bitwise reproducible.  Arguments as dist_render_color. */
int dist_render_color_bwd(dist_ctx* cctx, const dist_saved* geom, const float* zc,
                          int32_t n_latents, int32_t precision, const float* g_rgb,
                          float* g_zc, void* stream);

/* Cross-view photometric loss of multi-view reconstruction (Sec. 4, the
 * multi-view objective sum_i sum_{j in N_i} |I_i - I_{j->i}|; App. C: L1,
 * visibility by Delta_d^2 < 0.001, weight 5.0 in the paper).  For every
 * ordered pair (i, j) and every pixel x of view i with a finite depth, the
 * surface point X = c_i + z_c |(xt, yt, 1)| v_i(x) is projected into view j;
 * the pixel counts if X is in front of view j, the pixel of view j nearest to
 * the projection has a finite depth D_j with (depth of X in view j - D_j)^2
 * < 1e-3, and the 2x2 bilinear footprint lies inside the image; it then adds
 * weight / (H W) * sum over the 3 channels of |I_i(x) - I_j(projection)|.
 * The gradient flows to the depth of view i only (the visibility decision
 * and view j's depth are constants).
 *   cams     host array of n_views cameras (1..16 views, shared H and W)
 *   depth    device float [n_views][H][W]: rendered z_c (+inf = background)
 *   images   device float [n_views][H][W][3]: colour images
 *   pairs    host int32 [n_pairs][2] (1..64 pairs): (i, j) warps view j into
 *            view i; a view may have several neighbours
 *   weight   loss weight
 *   loss_map device float [n_views][H][W]: each pixel's loss (overwritten)
 *   loss     device float scalar: the total, summed in a fixed order
 *   g_depth  device float [n_views][H][W]: dL/d(depth) (overwritten), or NULL
 * Stream-ordered, no allocation; bitwise reproducible.  DIST_EINVAL for bad
 * arguments. */
int dist_photometric_loss(const dist_camera* cams, int32_t n_views,
                          const float* depth, const float* images,
                          const int32_t* pairs, int32_t n_pairs, float weight,
                          float* loss_map, float* loss, float* g_depth, void* stream);

/* Image-space loss of the latent fit and its gradient w.r.t. the rendered
 * maps (Sec. 4.2.1: L1 depth; App. A.3: silhouette hinge; App. B.3: the normal
 * term is the negative dot product; App. B.4 weights depth 10, silhouette 1).
 * Per image i of H x W pixels:
 *   loss[i] = 1/(H W) [ w_depth  sum_{fg_r & fg_t} |depth - depth_t|
 *                     + w_sil    sum_pix sil_t max(0, sil) + (1 - sil_t) max(0, -sil)
 *                     + w_normal sum_{fg_r & fg_t} -(normal . normal_t) ]
 * fg_r is the rendered silhouette (sil < 0), fg_t the target's (sil_t > 0.5);
 * sign(0) = 0 and max'(0) = 0; a hinge term whose weight sil_t or 1 - sil_t is
 * zero adds nothing (so a target depth off its silhouette is never read).
 *   depth, sil, depth_t, sil_t   device [n_images][H][W] (sil_t in [0, 1]);
 *                                1 <= n_images <= 65535, H W <= 2^22
 *   normal, normal_t             device [n_images][H][W][3]; read only when
 *                                w_normal != 0 (then both are required)
 *   loss                         device [n_images], overwritten
 *   g_depth, g_sil               device [n_images][H][W], dL/d(map) with L the
 *   g_normal                     sum of loss[i] ([..][3]); each may be NULL
 *                                (not written); g_normal is zero when
 *                                w_normal = 0
 * One workgroup per image sums in a fixed order: bitwise reproducible.
 * Stream-ordered, allocates nothing.  DIST_EINVAL for bad arguments. */
int dist_render_loss(int32_t n_images, int32_t H, int32_t W,
                     const float* depth, const float* normal, const float* sil,
                     const float* depth_t, const float* normal_t, const float* sil_t,
                     float w_depth, float w_sil, float w_normal,
                     float* loss, float* g_depth, float* g_normal, float* g_sil, void* stream);

/* One Adam step on n values (App. B.4: latent codes are optimised with Adam,
 * learning rate 1e-2): with step count t >= 1,
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   z -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
 * z, m, v device [n] (updated in place; m and v start at zero), g device [n].
 * Stream-ordered, allocates nothing.  DIST_EINVAL for bad arguments. */
int dist_adam_step(float* z, float* m, float* v, const float* g, int32_t n, float lr,
                   float beta1, float beta2, float eps, int32_t t, void* stream);

/* Convergence threshold of App. A.2: the radius eps at which the eps-balls
 * around the front ends of neighbouring pixels' rays stop overlapping, for a
 * camera with focal length `focal`, sensor size `sensor` (same unit as
 * focal), `resolution` pixels across the sensor, objects about `d_min` away
 * and a ray at angle `theta` (radians) to the optical axis:
 *   eps = d_min sensor cos^2(theta) / (2 focal resolution)
 * (in pixel units sensor / focal = W / fx).  Host arithmetic only, no GPU.
 * DIST_EINVAL unless d_min, sensor, focal > 0, resolution >= 1 and theta is
 * finite. */
int dist_eps_for_camera(double d_min, double sensor, double focal, int32_t resolution, double theta,
                        double* eps);

/* Free a forward state. */
int dist_saved_free(dist_saved* saved);

/* Decoder query (one network feed-forward per point, paper Sec. 3.2):
 * f[i] = f(points[i], z[latent_ids[i]]).  points device [n, 3], latent_ids
 * device int32 [n] in [0, n_latents), z device [n_latents, latent_dim],
 * f device [n].  precision DIST_FP32, DIST_BF16 or DIST_BF16X3.  n = 0 is a
 * no-op (the arrays may then be NULL). */
int dist_sdf_eval(dist_ctx* ctx, const float* points, const int32_t* latent_ids,
                  const float* z, int32_t n_latents, int64_t n, int32_t precision,
                  float* f, void* stream);

/* The decoder query of dist_sdf_eval without any allocation, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, result and
 * errors as dist_sdf_eval; its one scratch buffer (the per-latent folded
 * biases) is a fixed 1 MiB array per GPU that the library takes at
 * dist_create and keeps until the process ends, so n_latents * (width of
 * layer 0 + width of the skip layer) must fit 262144 floats (256 latents for
 * the DeepSDF decoder; larger requests return DIST_EINVAL).  The context's
 * device must be current.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (two streams, two threads, two contexts) race and
 * must be serialised by the caller.  No timing hooks are recorded. */
int dist_sdf_eval_noalloc(dist_ctx* ctx, const float* points, const int32_t* latent_ids,
                          const float* z, int32_t n_latents, int64_t n, int32_t precision,
                          float* f, void* stream);

/* Vector-Jacobian product of the decoder at detached points (the per-sample
 * term of Eq. 2): g_z[l] = sum_{i: latent_ids[i] = l} seeds[i] df(points[i],
 * z_l)/dz_l, and optionally the weight gradient.  points device [n, 3],
 * latent_ids device int32 [n] (ids outside [0, n_latents) are clamped to
 * that range, as in dist_sdf_eval), seeds device [n], z device [n_latents,
 * latent_dim], g_z device [n_latents, latent_dim]; g_W / g_b as for
 * dist_render_bwd.  precision DIST_FP32 (float32 throughout) or DIST_BF16 /
 * DIST_BF16X3 (split-bf16 recompute, bf16 back-propagation).  The samples
 * are grouped by latent on the device (a stable sort, so the sum order is
 * fixed and the result reproducible bit for bit); the call is stream-ordered
 * and does not synchronise the host, except with g_W, where it reads the
 * sample count once to size its chunk loop.  With n = 0, g_z (and g_W, g_b)
 * are zeroed and points, latent_ids and seeds may be NULL. */
int dist_sdf_vjp(dist_ctx* ctx, const float* points, const int32_t* latent_ids,
                 const float* seeds, const float* z, int32_t n_latents, int64_t n,
                 int32_t precision, float* g_z, float* const* g_W, float* const* g_b,
                 void* stream);

/* ---- serving: continuous batching of render and inverse-optimisation ---- */
#define DIST_REQ_RENDER 0
#define DIST_REQ_ZOPT   1

/* A request.  Buffers are device memory owned by the caller and must stay
 * alive until dist_poll reports completion.
 *   cams/n_views  host, copied at submit; all views share H, W
 *   z             device [latent_dim]: RENDER reads it; ZOPT reads it as the
 *                 initial code and writes the optimised code into z_out
 *   depth/sil/normal/status  optional outputs [n_views, H, W](x3)
 *   ZOPT: target_depth/target_sil device [n_views, H, W] (sil in {0,1}),
 *         iters Adam iterations with learning rate lr (paper App. B.4:
 *         Adam, 1e-2), loss w_depth * L1 depth + w_sil * silhouette hinge
 *         (App. A.3), z_out device [latent_dim].
 * A request whose render meets a non-finite signed distance ends with
 * status DIST_ENUMERIC; a z-opt request then stops optimising and leaves
 * z_out unwritten. */
typedef struct {
  int32_t kind;
  int32_t n_views;
  const dist_camera* cams;
  dist_trace_params prm;
  const float* z;
  float* depth;
  float* sil;
  float* normal;
  uint8_t* status;
  const float* target_depth;
  const float* target_sil;
  int32_t iters;
  float lr, w_depth, w_sil;
  float* z_out;
} dist_request;

typedef struct {
  int32_t status;        /* DIST_OK, DIST_ECANCELLED, DIST_ENUMERIC, ...   */
  int64_t latency_ns;    /* submit -> completion                           */
  int64_t queries;       /* decoder queries spent marching                 */
  float final_loss;      /* ZOPT: loss at the last iteration               */
} dist_result;

/* Queue a request; returns a ticket.  Admission waits for slots and memory
 * (HBM budget); DIST_EBUSY if the queue is full, DIST_ENOMEM if the request
 * can never fit the budget, DIST_EINVAL for malformed requests. */
int dist_submit(dist_ctx* ctx, const dist_request* req, uint64_t* ticket);

/* Wait up to timeout_us (0 = just check, <0 = forever) for a ticket.
 * DIST_OK with *res filled when done (the ticket is then released),
 * DIST_PENDING if still running, DIST_ENOTFOUND for unknown tickets. */
int dist_poll(dist_ctx* ctx, uint64_t ticket, dist_result* res, int64_t timeout_us);

/* ---- kernel timing ------------------------------------------------------
 * When enabled, the library records a pair of HIP events on the caller's
 * stream around every launch of its decoder kernels.  dist_timing_read
 * synchronises on those events and returns, for one kernel class, the
 * number of launches and their summed duration since timing was enabled.
 * kernel: 0 = march step (decoder + march update), 1 = plain decoder queries
 * (normals, dist_sdf_eval), 2 = adjoint (backward recompute + VJP),
 * 3 = VJP of the normal-stencil samples from the ReLU masks the forward
 * saved (no recompute), 4 = weight-gradient contraction over the captured
 * rows (one launch per layer and chunk; rows are not counted). */
typedef struct {
  int64_t launches;
  double ms;
  int64_t rows;      /* decoder evaluations processed (rays, points or samples) */
} dist_kernel_time;

int dist_timing_enable(dist_ctx* ctx, int on);
int dist_timing_read(dist_ctx* ctx, int32_t kernel, dist_kernel_time* out);

/* Thread-local message describing the last error. */
const char* dist_last_error(void);

/* Library version string. */
const char* dist_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DIST_H_ */
