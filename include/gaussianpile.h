/*
 * gaussianpile.h -- C-ABI of the MI355X (gfx950) Focus-Gaussian slice renderer.
 *
 * The library renders axial slices of a set of anisotropic 3-D Gaussians under
 * GaussianPile's finite-thickness focus model (Sec. 4.2), differentiates the
 * rendering (Sec. 4.3, "Backward pass"; supplement, "Derivation of Differentiable Backward Pass"), updates parameters
 * with Adam (Sec. 5.1, implementation details) and serves slices of resident
 * volumes.
 *
 * Conventions shared by every entry point
 *   - Pointers named d_* are device pointers on the calling thread's current
 *     HIP device, owned by the caller (the library never frees them).  Pointers
 *     named h_* are host pointers, read before the call returns.
 *   - gp_workspace and gp_server objects are owned by the library; create and
 *     destroy them with the matching calls.  A workspace may be used by one
 *     thread at a time.
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Every compute entry point is asynchronous on that stream unless stated.
 *   - Every entry point returns a gp_status.  On failure, gp_last_error()
 *     returns a thread-local description.  No C++ exception crosses the ABI.
 *
 * Gaussian parameters (supplement, "Derivation of Forward rendering process": G = (mu, s, q, alpha)) are stored as
 * planes ("SoA"): plane r of a set with row stride `stride` starts at element
 * r * stride.  The eleven rows are
 *     0..2  mu_x, mu_y, mu_z            position (world units)
 *     3..5  l_x, l_y, l_z               log-scales, s = exp(l) * scale_mod
 *     6..9  q_w, q_x, q_y, q_z          rotation quaternion, any non-zero norm
 *     10    alpha                       intensity coefficient (used linearly)
 * and the library reads `means` (rows 0..2) and `attrs` (rows 3..10) through
 * two pointers so that 16-bit attributes can sit beside float32 positions.
 *
 * A slice is the axial plane z = const imaged with axial PSF width sigma_z
 * (Sec. 4.1, sensitivity map h(-z_c) = exp(-z_c^2 / 2 sigma_z^2)); its camera is
 * R_c = I, t = (0, 0, -z) (supplement, "Derivation of Forward rendering process").  Pixel (px, py) has centre
 * (x0 + (px + 1/2) dx, y0 + (py + 1/2) dy).  Images of a batch are packed back
 * to back in slice order, each row-major [height][width] float32.
 */
#ifndef GAUSSIANPILE_H
#define GAUSSIANPILE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gp_status;
#define GP_OK          0
#define GP_EINVAL     -1   /* bad argument (null pointer, size, dtype, ...) */
#define GP_ENOMEM     -2   /* device or host allocation failed */
#define GP_EHIP       -3   /* a HIP runtime call failed */
#define GP_EOVERFLOW  -4   /* a fixed-capacity workspace was too small */
#define GP_EAGAIN     -5   /* serving: result not ready yet */
#define GP_ECANCELED  -6   /* serving: request cancelled by server shutdown */
#define GP_ESTATE     -7   /* call order violated (e.g. backward without forward) */

#define GP_F32  0
#define GP_BF16 1
#define GP_F16  2
/* GP_Q16: 16-bit storage for served volumes.  Log-scales and intensity are
 * IEEE half precision; the quaternion is stored normalised, each component as
 * int16 fixed point: v = rint(q_i / sqrt(((qw^2 + qx^2) + qy^2) + qz^2) * 32767)
 * in binary32 (round half to even), read back as v / 32767.  Half-precision
 * quaternions dominate the error of 16-bit storage for thin, elongated
 * Gaussians; fixed point gives 2^-15 absolute resolution instead. */
#define GP_Q16  3
/* GP_QM: the Morton-ordered fixed-point codec of gp_encode (both mean_dtype and
 * attr_dtype): means points at 11 uint16 code planes [11][stride], attrs at
 * the 9-float gp_codec_header in device memory.  Decoded in registers by the
 * forward renderer (the backward and the voxeliser take float32 or 16-bit
 * attributes only). */
#define GP_QM   4

/* Render options.  q_cut: axial cull threshold on the Mahalanobis change of the
 * opacity modulation (Sec. 4.2, "cull primitives with opacity below a small
 * threshold"); a (Gaussian, slice) pair is drawn iff m^2 / (sigma_z^2 +
 * Sigma_zz) <= q_cut.  bbox_sigmas: half-width of the tile footprint in
 * standard deviations of Sigma_2d.  scale_mod: the `mod` factor of
 * S = diag(mod * s) (supplement, "Derivation of Forward rendering process").  GP_FLAG_EXACT: no cull and no
 * footprint, every Gaussian reaches every pixel (reference mode).
 * GP_FLAG_CONV_EXACT: instead of the paper's phenomenological intensity
 * alpha~ = alpha opacity_r / sqrt(det Sigma_2d) (Sec. 4.2, intensity
 * normalisation), the exact value of the convolution integral of Sec. 4.2
 * (I = integral of h(t) g_c(x, y, t) dt): alpha~ = alpha opacity_r
 * sqrt(2 pi det Sigma_e / det Sigma_2d), i.e. the paper's value times
 * sqrt(2 pi det Sigma_e) with det Sigma_e = det Sigma sigma_z^2 / (sigma_z^2 +
 * Sigma_zz) (0 for sigma_z = 0, det Sigma for sigma_z = +inf).  Forward and
 * backward; the membership (bins) does not change.
 * GP_FLAG_FORWARD_ONLY: the render keeps no bookkeeping for a backward (the
 * per-record tile rectangles and instance slots, 16 B per record, are not
 * written); images are identical, and gp_render_backward on that workspace
 * returns GP_ESTATE.  For inference: stacks rendered for viewing, serving. */
#define GP_FLAG_EXACT 1u
#define GP_FLAG_CONV_EXACT 2u
#define GP_FLAG_FORWARD_ONLY 4u
typedef struct gp_render_opts {
  float q_cut;        /* default 2 ln 255 = 11.0825...: opacity_r >= 1/255 */
  float bbox_sigmas;  /* default 3 */
  float scale_mod;    /* default 1 */
  uint32_t flags;
} gp_render_opts;

typedef struct gp_gaussians {
  const void* means;  /* d_: [3][stride], mean_dtype (GP_F32; GP_QM: codes)   */
  const void* attrs;  /* d_: [8][stride], attr_dtype (GP_F32, GP_BF16, GP_F16, GP_Q16; GP_QM: header) */
  int64_t n;          /* number of Gaussians, 0 <= n <= stride, n < 2^31      */
  int64_t stride;     /* elements between planes                              */
  int32_t mean_dtype;
  int32_t attr_dtype;
} gp_gaussians;

typedef struct gp_slice {
  float z;            /* depth of the imaging plane (world units)              */
  float sigma_z;      /* axial PSF width, 0 <= sigma_z <= +inf                 */
  float x0, y0;       /* world position of the grid's lower corner             */
  float dx, dy;       /* pixel pitch, > 0                                      */
  int32_t width;      /* pixels, 1 .. 16384                                    */
  int32_t height;     /* pixels, 1 .. 16384                                    */
} gp_slice;

typedef struct gp_workspace gp_workspace;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t gp_version(void);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* gp_last_error(void);

/* Fills *o with the defaults listed above.  GP_EINVAL if o is NULL. */
gp_status gp_default_opts(gp_render_opts* o);

/* Creates a workspace on the current device.  max_records / max_instances fix
 * the capacity of the per-(Gaussian, slice) record and per-(record, tile) list
 * buffers.  0 for both selects automatic sizing: each render reads the counts
 * back once (one host synchronisation) and grows the buffers when needed.  With
 * fixed capacities no render synchronises; an overflow drops entries, is
 * remembered and reported as GP_EOVERFLOW by gp_workspace_check.
 * Errors: GP_EINVAL (ws NULL, negative capacity), GP_ENOMEM, GP_EHIP. */
gp_status gp_workspace_create(gp_workspace** ws, int64_t max_records, int64_t max_instances);

/* Waits for the workspace's last stream, then frees it.  NULL is accepted. */
gp_status gp_workspace_destroy(gp_workspace* ws);

/* Counts of the most recent render: records (visible or axially kept
 * (Gaussian, slice) pairs), instances (tile-list entries) and bins (16x16
 * tiles over all slices).  Synchronises with the workspace's last stream.
 * Returns GP_EOVERFLOW if any render since creation overflowed a fixed
 * capacity (the flag is then cleared). */
gp_status gp_workspace_check(gp_workspace* ws, int64_t* records, int64_t* instances, int64_t* bins);

/* Forward rendering of n_slices axial slices (Sec. 4.2: Focus Gaussian,
 * opacity modulation, screen-space projection, intensity normalisation and
 * additive rasterisation; supplement, "Derivation of Forward rendering process" for the full derivation):
 *   I_k(p) = sum over the members i of p's tile list on slice k of
 *            alpha~_ik exp(-1/2 d^T Sigma_2d,ik^-1 d),  d = p - mu_2d,ik
 *   alpha~ = alpha * opacity_r / sqrt(det Sigma_2d).
 * h_slices: host array [n_slices].  d_out: device float32, sum_k width_k *
 * height_k elements, overwritten.  The tile lists are kept in `ws` for a
 * following gp_render_backward.  Errors: GP_EINVAL, GP_ENOMEM, GP_EHIP. */
gp_status gp_render_slices(gp_workspace* ws, const gp_gaussians* g, const gp_slice* h_slices,
                           int32_t n_slices, const gp_render_opts* opts, float* d_out, void* stream);

/* Backward of the preceding gp_render_slices on the same workspace, Gaussian
 * set and slices (Sec. 4.3 "Backward pass", supplement, "Derivation of Differentiable Backward Pass"): given
 * d_grad_out = dL/dI (same layout as d_out), ADDS dL/dparams to d_grad
 * ([11][grad_stride] float32, rows as above; grad_stride >= n).  Per-pixel
 * contributions are recomputed from the tile lists, not stored.  The result is
 * deterministic (no floating-point atomics).
 * Errors: GP_ESTATE if the workspace holds no matching forward, GP_EINVAL,
 * GP_EHIP. */
gp_status gp_render_backward(gp_workspace* ws, const gp_gaussians* g, const gp_slice* h_slices,
                             int32_t n_slices, const gp_render_opts* opts, const float* d_grad_out,
                             float* d_grad, int64_t grad_stride, void* stream);

/* Oblique slices: gp_render_slices / gp_render_backward with a camera pose per
 * slice (supplement, "Derivation of Forward rendering process": each slice's
 * view matrix [R_c | t] maps mu_c = R_c mu + t, Sigma_c = R_c Sigma R_c^T).
 * h_poses: host array [n_slices][12] float32, R_c row-major then t (the caller
 * keeps ownership; it is copied before the call returns).  R_c must be a
 * rotation (|R_c R_c^T - I| <= 1e-4 entrywise, det > 0), else GP_EINVAL.  Slice
 * k then samples the plane z_c = z of its camera frame, with pixel centres at
 * (x_c, y_c) = (x0 + (px + 1/2) dx, y0 + (py + 1/2) dy); the identity pose is
 * the axial slice (and gives bit-identical bins and images).  Membership stays
 * binary32-exact: R_c R_q and mu_c are formed in a fixed order (documented with
 * the binning specification).  h_poses = NULL is the axial call.  The backward
 * must get the same poses as its forward (else GP_ESTATE). */
gp_status gp_render_slices_posed(gp_workspace* ws, const gp_gaussians* g, const gp_slice* h_slices,
                                 const float* h_poses, int32_t n_slices, const gp_render_opts* opts,
                                 float* d_out, void* stream);
gp_status gp_render_backward_posed(gp_workspace* ws, const gp_gaussians* g, const gp_slice* h_slices,
                                   const float* h_poses, int32_t n_slices, const gp_render_opts* opts,
                                   const float* d_grad_out, float* d_grad, int64_t grad_stride, void* stream);

/* L1 term of the loss (Sec. 4.3, loss function): d_grad[j] = scale * sign(d_image[j] -
 * d_target[j]) with sign(0) = 0, and *d_loss += scale * sum_j |d_image[j] -
 * d_target[j]| (d_loss may be NULL).  scale is normally 1 / n.
 * Errors: GP_EINVAL (n < 0, NULL arrays), GP_EHIP. */
gp_status gp_l1_loss_grad(const float* d_image, const float* d_target, int64_t n, float scale,
                          float* d_grad, float* d_loss, void* stream);

/* The full slice loss (Sec. 4.3, loss function; lambda = 0.2 in Sec. 5.1):
 *   L = mean |I - T| + lambda * (1 - mean SSIM(I, T))
 * over a batch of n_slices slices of one grid, packed [n_slices][height][width]
 * float32.  SSIM (Wang et al. 2004): 11 x 11 Gaussian window of standard
 * deviation 1.5 with unit sum, zeros outside the slice, C1 = 0.01^2,
 * C2 = 0.03^2, evaluated at every pixel.  d_grad receives dL/dI (written,
 * sign(0) = 0 in the L1 part); d_loss, if not NULL, float[2]: += the L1 term,
 * += the D-SSIM term (1 - mean SSIM).  ws provides scratch of 24 bytes per
 * pixel (grown on demand, which synchronises).  Arithmetic in float64.
 * Errors: GP_EINVAL (NULL, negative sizes, n_slices > 65535, lambda < 0 or
 * not finite), GP_ENOMEM/GP_EHIP. */
gp_status gp_l1_dssim_loss_grad(gp_workspace* ws, const float* d_image, const float* d_target, int32_t n_slices,
                                int32_t width, int32_t height, float lambda, float* d_grad, float* d_loss,
                                void* stream);

/* gp_l1_dssim_loss_grad without a workspace and without allocating, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving or training loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results as gp_l1_dssim_loss_grad; its scratch (coefficient maps
 * and per-block sums, float64) lives in a static device array of 6,422,528
 * elements (51.4 MB) that every GPU the library runs on holds until the process
 * ends.  A call needs 3 * n_slices * width * height + 2 * n_slices *
 * ceil(width / 32) * ceil(height / 16) elements: up to 2^21 pixels of slices
 * whose sides are multiples of 32 and 16 (e.g. 8 slices of 512 x 512 or 32 of
 * 256 x 256).  Larger requests return GP_EINVAL before anything is launched.
 * All calls on one GPU share that array, which keeps the last call's contents
 * (nothing in it needs clearing: every element read is first written by the
 * same call); calls whose executions overlap on one GPU (other streams, other
 * threads) race on it and must be serialised by the caller.  The first call on
 * a device looks up the array's address there (no allocation).
 * Errors: GP_EINVAL (as gp_l1_dssim_loss_grad, or too large), GP_EHIP. */
gp_status gp_l1_dssim_loss_grad_noalloc(const float* d_image, const float* d_target, int32_t n_slices,
                                        int32_t width, int32_t height, float lambda, float* d_grad,
                                        float* d_loss, void* stream);

/* Adam (Kingma & Ba, Algorithm 1; the optimiser named in Sec. 5.1) on float32
 * planes [11][stride] in place: for every element
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2
 *   p -= lr_group * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
 * with lr_group = lr[0] for rows 0..2 (positions), lr[1] rows 3..5
 * (log-scales), lr[2] rows 6..9 (quaternion), lr[3] row 10 (intensity).
 * GP_ADAM_CLAMP_ALPHA projects row 10 onto alpha >= 0 after the step;
 * GP_ADAM_ZERO_GRAD writes zero into d_grad after reading it.
 * Errors: GP_EINVAL (step < 1, n > stride, NULL), GP_EHIP. */
#define GP_ADAM_CLAMP_ALPHA 1u
#define GP_ADAM_ZERO_GRAD   2u
typedef struct gp_adam_cfg {
  float lr[4];
  float beta1, beta2, eps;
  int32_t step;
  uint32_t flags;
} gp_adam_cfg;
gp_status gp_adam_step(float* d_params, float* d_grad, float* d_m, float* d_v, int64_t n,
                       int64_t stride, const gp_adam_cfg* cfg, void* stream);

/* ------------------------------------------------------------------------
 * Codec (Sec. 4.3, "Quantization and compression"): Gaussians sorted along the
 * Morton curve of their 14-bit position codes; positions normalised to the
 * bounding box of the finite means, 14 bits per axis; log-scales on the range
 * of the finite log-scales, 12 bits; the quaternion normalised, moved to w >= 0
 * and each component coded on [-1, 1] with 12 bits; intensity normalised to
 * [0, 1] by the largest finite intensity amax, 12 bits.  Codes are floor(((v - lo) / (hi - lo)) * (levels - 1) +
 * 0.5) in binary32, clamped (0 for an empty range or a non-finite value);
 * values decode as lo + code * ((hi - lo) / (levels - 1)).  The entropy coder
 * that follows in the paper is not part of this codec.
 * ---------------------------------------------------------------------- */
typedef struct gp_codec_header {
  float lo[3], hi[3];   /* bounding box of the means */
  float lmin, lmax;     /* range of the log-scales */
  float amax;           /* largest intensity (>= 0) */
} gp_codec_header;

/* Encodes n Gaussians (d_params [11][stride] float32) into d_codes ([11][stride_out]
 * uint16, Morton order), the header into d_header (device, 9 floats) and, if
 * d_perm is not NULL, the original index of each coded Gaussian ([n] uint32).
 * Deterministic.  Allocates scratch and synchronises on stream.
 * Errors: GP_EINVAL, GP_ENOMEM, GP_EHIP. */
gp_status gp_encode(const float* d_params, int64_t n, int64_t stride, uint16_t* d_codes, int64_t stride_out,
                    uint32_t* d_perm, float* d_header, void* stream);

/* ------------------------------------------------------------------------
 * Differentiable voxeliser (Sec. 4.3, "Differentiable Voxelization"): the
 * volume sigma(x) = sum_i alpha_i exp(-1/2 (x - mu_i)^T Sigma_i^-1 (x - mu_i))
 * of the world-space Gaussians (no focus re-parameterisation), accumulated over
 * 8 x 8 x 8-voxel tiles, each keeping the Gaussians whose 3-sigma box (half-
 * widths bbox_sigmas * sqrt(Sigma_aa), decided in binary32) reaches it; with
 * GP_FLAG_EXACT every finite Gaussian reaches every voxel.  Voxel (i, j, k)
 * has centre (x0 + (i + 1/2) dx, y0 + (j + 1/2) dy, z0 + (k + 1/2) dz).
 * ---------------------------------------------------------------------- */
typedef struct gp_volume_grid {
  float x0, y0, z0;     /* corner of the volume */
  float dx, dy, dz;     /* voxel pitch, > 0 */
  int32_t nx, ny, nz;   /* voxels per axis, >= 0 */
  int32_t pad;
} gp_volume_grid;

/* Writes the volume [nz][ny][nx] float32 into d_volume.  Uses ws for the tile
 * lists (replacing any slice forward it held) and synchronises once on stream
 * (the tile-list size is read back).  Deterministic.
 * Errors: GP_EINVAL (bad grid, more than 2^30 tiles, NULL), GP_ENOMEM, GP_EHIP. */
gp_status gp_voxelize(gp_workspace* ws, const gp_gaussians* g, const gp_volume_grid* grid,
                      const gp_render_opts* opts, float* d_volume, void* stream);

/* Adds dL/dparams of L = sum_v d_grad_volume[v] * V[v] into d_grad ([11][grad_stride]
 * float32) for the Gaussians and grid of the last gp_voxelize on ws.
 * Deterministic (no floating-point atomics).
 * Errors: GP_ESTATE (ws holds no matching voxelisation), GP_EINVAL, GP_EHIP. */
gp_status gp_voxelize_backward(gp_workspace* ws, const gp_gaussians* g, const gp_volume_grid* grid,
                               const gp_render_opts* opts, const float* d_grad_volume, float* d_grad,
                               int64_t grad_stride, void* stream);

/* ------------------------------------------------------------------------
 * Densify and prune (Sec. 4.3, "Prune and densification": driven by the
 * Gaussians' footprint radii on the slices and their intensities; thresholds
 * of Sec. 5.1).  The procedure is the usual Gaussian-splatting control:
 *   prune  alpha < min_alpha, non-finite parameters, or largest footprint
 *          half-width (pixels, over the accumulated backwards) > max_radius;
 *   grow   mean norm of the projected-mean gradient (pixel units, per visible
 *          record) > grad_threshold: clone (exact copy) if the largest scale
 *          exp(l) <= split_scale, else split into two children at
 *          mu + R(q) diag(s) n_k, n_k = d_noise[3k..3k+2][j], log-scales
 *          reduced by ln(split_factor), q and alpha copied.
 * Adam moments are carried over for kept Gaussians and zero for new ones.
 * ---------------------------------------------------------------------- */
typedef struct gp_densify_cfg {
  float grad_threshold;   /* 5e-5 (Sec. 5.1)                                  */
  float min_alpha;        /* 0.02 (Sec. 5.1)                                  */
  float max_radius;       /* pixels                                            */
  float split_scale;      /* world units                                       */
  float split_factor;     /* 1.6                                               */
  uint32_t flags;
} gp_densify_cfg;
gp_status gp_densify_default_cfg(gp_densify_cfg* cfg);

/* While set, every gp_render_backward on ws also adds, for each Gaussian
 * j < n: the sum over its visible records of |dL/dmu_2d| in pixel units to
 * d_grad_norm[j], the number of those records to d_count[j], and raises
 * d_max_radius[j] to its largest footprint half-width in pixels.  One writer
 * per element (deterministic).  All pointers NULL disables.  Errors: GP_EINVAL. */
gp_status gp_workspace_set_densify_stats(gp_workspace* ws, float* d_grad_norm, int32_t* d_count,
                                         float* d_max_radius, int64_t n);

/* Applies densify/prune to n Gaussians ([11][stride] parameters and Adam
 * moments) and writes the new set, in Gaussian order (children adjacent), to
 * the *_out planes ([11][stride_out]).  d_noise: [6][n] float32 (two 3-vectors
 * per Gaussian; only rows of split Gaussians are read).  Synchronous:
 * *n_out receives the new count.  GP_EOVERFLOW (nothing written, *n_out set)
 * if stride_out is too small.  Errors: GP_EINVAL, GP_ENOMEM, GP_EHIP. */
gp_status gp_densify_prune(const float* d_params, const float* d_m, const float* d_v, int64_t n, int64_t stride,
                           const float* d_grad_norm, const int32_t* d_count, const float* d_max_radius,
                           const float* d_noise, const gp_densify_cfg* cfg, float* d_params_out, float* d_m_out,
                           float* d_v_out, int64_t stride_out, int64_t* n_out, void* stream);

/* ------------------------------------------------------------------------
 * Serving: many fitted volumes resident in HBM, slices rendered on request.
 * A server keeps each volume's positions in float32 and its log-scales,
 * quaternions and intensities in attr_dtype (16-bit storage, converted to
 * float32 in the kernels; accumulation is float32).  Requests for slices of
 * different volumes, depths, resolutions and sigma_z are admitted while
 * earlier batches run: a scheduler thread groups queued requests into one
 * batch whenever one of `slots` launch slots is free (the batch's estimated
 * list size must fit the slot's capacity), and renders the whole batch with
 * one replay of a captured hipGraph on that slot's stream.  Each request's
 * image goes straight into the caller's buffer.  A batch whose lists
 * overflow is re-run one request at a time; a single request that still does
 * not fit completes with GP_EOVERFLOW.  The rendering is the one of
 * gp_render_slices (Sec. 4.2) with the server's options.
 * ---------------------------------------------------------------------- */
typedef struct gp_server gp_server;

typedef struct gp_server_cfg {
  int64_t hbm_budget_bytes;    /* bytes of resident volume storage allowed      */
  int64_t max_gaussians;       /* per batch: sum of the batch's volume sizes    */
  int64_t max_records;         /* per slot: record capacity                     */
  int64_t max_instances;       /* per slot: tile-list capacity                  */
  int32_t max_bins;            /* per batch: 16x16 tiles over all its requests  */
  int32_t max_batch;           /* requests per batch (1 = one launch each)      */
  int32_t slots;               /* batches in flight, 1..4                       */
  int32_t attr_dtype;          /* GP_Q16, GP_F16, GP_BF16 or GP_F32              */
  int32_t use_graphs;          /* replay a captured graph per slot (else launch;
                                  a batch holding one request of more than
                                  16,383 tiles is always launched)              */
  int32_t device;              /* HIP device                                    */
  gp_render_opts opts;
} gp_server_cfg;

typedef struct gp_request {
  int32_t volume_id;
  float z, sigma_z;            /* depth and axial PSF width of the slice        */
  float x0, y0, dx, dy;        /* pixel grid (see gp_slice)                     */
  int32_t width, height;
} gp_request;

typedef struct gp_serve_result {
  int32_t status;              /* GP_OK, GP_EOVERFLOW, GP_ECANCELED, GP_EHIP     */
  int32_t batch_size;          /* requests in the batch that rendered it        */
  int64_t batch_id;
  double latency_ms;           /* arrival (the submit call, or the stamp given to
                                  gp_serve_submit_many) -> completion observed by
                                  the server                                   */
} gp_serve_result;

typedef struct gp_server_stats {
  int64_t submitted, completed, batches, retries, resident_bytes;
  int32_t volumes;
  int32_t pad;
} gp_server_stats;

/* Defaults: 16 GiB budget, 64 requests per batch, 3 slots, GP_Q16 attributes
 * (on filament-shaped volumes BF16 and FP16 storage exceed a 2e-3 image error,
 * GP_Q16 stays below it), graphs on. */
gp_status gp_server_default_cfg(gp_server_cfg* cfg);

/* Creates a server (its streams, slots and scheduler thread) on cfg->device.
 * Errors: GP_EINVAL, GP_ENOMEM, GP_EHIP. */
gp_status gp_server_create(gp_server** sv, const gp_server_cfg* cfg);

/* Copies a fitted Gaussian set (g: float32 means and attributes, any stride)
 * into resident storage, converting the attributes to cfg->attr_dtype.
 * Synchronous.  *volume_id receives its id.  Errors: GP_ENOMEM if the budget
 * would be exceeded, GP_EINVAL, GP_EHIP. */
gp_status gp_server_add_volume(gp_server* sv, const gp_gaussians* g, int32_t* volume_id);

/* Queues one request; d_out (device, width * height float32) receives the
 * image.  Non-blocking; *ticket identifies it.  Errors: GP_EINVAL (unknown
 * volume, bad grid, NULL), GP_ECANCELED (server shutting down). */
gp_status gp_serve_submit(gp_server* sv, const gp_request* req, float* d_out, uint64_t* ticket);

/* Queues n requests at once (one lock, one scheduler wake-up): request i
 * renders into d_outs[i] and receives tickets[i].  t_arrival_ms, if not NULL,
 * gives each request's arrival time on the server's clock (gp_clock_ms), from
 * which its latency is measured (a front end that receives requests in bursts
 * keeps their true waiting time); NULL stamps them now.  All requests are
 * checked before any is queued.  Errors: as gp_serve_submit (nothing queued). */
gp_status gp_serve_submit_many(gp_server* sv, const gp_request* reqs, float* const* d_outs,
                               const double* t_arrival_ms, int32_t n, uint64_t* tickets);

/* The server's clock: milliseconds of a steady (monotonic) clock. */
double gp_clock_ms(void);

/* Waits up to timeout_us (0: do not wait, < 0: forever) for a ticket.
 * Returns GP_OK and fills *res when the request finished (res->status tells
 * how), GP_EAGAIN if it is still pending, GP_EINVAL for an unknown ticket.
 * A finished ticket is forgotten once polled. */
gp_status gp_serve_poll(gp_server* sv, uint64_t ticket, int32_t timeout_us, gp_serve_result* res);

/* Counters since creation. */
gp_status gp_server_stats_get(gp_server* sv, gp_server_stats* st);

/* Stops admitting, cancels queued requests (GP_ECANCELED), waits for the
 * batches on the GPU, frees everything.  NULL is accepted. */
gp_status gp_server_destroy(gp_server* sv);

/* Per-stage kernel timing of a workspace, for measurement.  `enable` is a mask
 * of stages, bit (1 << GP_STAGE_x) for stage x (GP_TIMING_ALL for every stage,
 * 0 to switch timing off).  Each selected stage of a render or backward on this
 * workspace is bracketed by HIP events recorded on the call's stream (no host
 * synchronisation is added); gp_workspace_timings synchronises, resolves the
 * pending events and returns, per stage, the summed milliseconds and the number
 * of launches since timing was set.  Setting resets the sums.  Errors:
 * GP_EINVAL, GP_EHIP. */
#define GP_STAGE_PREPROCESS      0   /* activation, axial cull, counts, slot scan   */
#define GP_STAGE_EMIT            1   /* records and (bin, record) pairs             */
#define GP_STAGE_SORT            2   /* stable radix sort by bin, bin ranges        */
#define GP_STAGE_RASTER_FWD      3   /* additive rasterisation                      */
#define GP_STAGE_RASTER_BWD      4   /* per-entry moments of the upstream gradient */
#define GP_STAGE_PREPROCESS_BWD  5   /* chain rule to the Gaussian parameters       */
#define GP_N_STAGES              6
#define GP_TIMING_ALL            ((1 << GP_N_STAGES) - 1)
gp_status gp_workspace_set_timing(gp_workspace* ws, int32_t enable);
gp_status gp_workspace_timings(gp_workspace* ws, double* h_ms, int64_t* h_counts, int32_t n_stages);

/* Test hook: copies the tile lists of the most recent render (or voxelisation)
 * to host memory, synchronously.  h_keys[j] = (bin << 32) | gaussian index, in
 * list order, where bins are numbered slice by slice (in the order given) and
 * row-major within a slice (for a voxelisation: (tz * nty + ty) * ntx + tx); h_ranges[2b], h_ranges[2b+1] = [start, end) of bin b.
 * *n_keys receives the number of entries; h_keys must hold keys_cap entries and
 * h_ranges 2 * bins entries.  Errors: GP_EINVAL (too small), GP_ESTATE. */
gp_status gp_debug_export_bins(gp_workspace* ws, uint64_t* h_keys, int64_t keys_cap, int64_t* n_keys,
                               int64_t* h_ranges, int64_t ranges_cap);

#ifdef __cplusplus
}
#endif
#endif /* GAUSSIANPILE_H */
