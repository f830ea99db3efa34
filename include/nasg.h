/*
 * nasg.h - C ABI of the NASGabor / degree-3 SH appearance evaluator for
 * AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for every primitive i and view v, the view-dependent
 * colour of the appearance model of Section 4.2 (appearance-model equation)
 *
 *     rgb(i, v) = c0_i + sum_{l < K} w_{i,l} G_{i,l}(d_{i,v})
 *
 * with G the Normalized Anisotropic Spherical Gabor lobe of Section 5.1, and
 * the analytic gradients of a scalar loss L = sum grad_rgb * rgb with respect
 * to every stored input (Supplementary F, with dC^{-1}/dlambda read with a
 * minus sign), plus a degree-3 real spherical-harmonics evaluator (Section
 * 3.2) as the comparison model. Following the central-ray approximation of
 * Section 5.2 there is one evaluation per primitive per view, along
 *
 *     d_{i,v} = (mu_i - o_v) / |mu_i - o_v|        (ray r(t) = o + t d, Section 3.1)
 *
 * The library also composites per-primitive colours into an image (Section
 * 3.1: depth-sorted alpha blending of projected 3D Gaussians) with the
 * gradients of an image loss for colours, opacities and geometry; see the
 * compositing section at the end of this header.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array pointers are DEVICE pointers owned by the caller. The library
 *   never allocates, frees, synchronises or copies between host and device
 *   inside the evaluation calls, and reads the argument structs only on the
 *   host during the call (they may live on the caller's stack).
 * - Calls are asynchronous on `stream` (a hipStream_t; NULL = default stream).
 * - Sizes are 64-bit; element offsets are computed in 64 bits.
 * - The return value is the only error channel (NASG_OK or a negative
 *   nasg_status). Arguments are validated on the host before any launch; on
 *   an error nothing is launched and no output is touched.
 * - n == 0 is valid and launches nothing.
 * - Every output is fully overwritten (NASG_GRAD_OVERWRITE) or added to
 *   (NASG_GRAD_ACCUMULATE, gradients only). Appearance results are bitwise
 *   deterministic run to run: per-primitive sums over views are reduced in a
 *   fixed order in registers and wavefront lanes, without atomics. (The
 *   compositing backward at the end of this header is the one exception.)
 *
 * Layouts (primitive index fastest inside each lobe; K lobes lobe-major)
 * ---------------------------------------------------------------------
 *   quat   [K][N][4]  lobe frame as a quaternion (w, x, y, z), any nonzero
 *                     norm; the frame is the rotation of q/|q|: x, y, z are the
 *                     columns of R(q/|q|) (the paper's R = [x y z], y = z x x,
 *                     Supplementary C, with a quaternion in place of its
 *                     three cosines).                     16 B aligned (f32)
 *   shape  [K][N][4]  (lambda > 0, a > -1, k, zeta): bandwidth, anisotropy,
 *                     carrier frequency and carrier phase; the carrier is
 *                     (1 + cos(k d.x + zeta))/2 (zeta = 0 is the paper's).
 *                                                         16 B aligned (f32)
 *   rgbw   [K][3][N]  per-lobe RGB weight w, channel-planar
 *   c0     [N][3]     diffuse colour (always float32)
 *   means  [N][3], cams [V][3]     primitive centres and camera centres, or
 *   dirs   [N][3]     one raw view direction per primitive (normalised
 *                     inside; then V must be 1)
 *   rgb, grad_rgb   [V][N][3] float32
 *   sh     [16][3][N] SH coefficients, basis index l*l + l + m
 * With NASG_BF16 storage, quat / shape / rgbw hold bfloat16 values (8 B
 * aligned for quat / shape); arithmetic and accumulation stay float32 (frame
 * and view geometry float64) and every gradient is written as float32 in the
 * float32 layout above.
 *
 * Lobe parametrisation (nasg_params.param)
 * -----------------------------------------
 * NASG_PARAM_QUAT   : the slots hold the values above.
 * NASG_PARAM_ANGLES : the slots hold the paper's own stored values, before
 *   activation (Supplementary C and its activation table):
 *   quat  -> (u_theta, u_phi, u_psi, unused): frame cosines c = tanh(u),
 *            sines s = +sqrt(1 - c^2),
 *            z = (c_theta s_phi, s_theta s_phi, c_phi),
 *            x = (c_theta c_phi c_psi - s_theta s_psi,
 *                 s_theta c_phi c_psi + c_theta s_psi, -s_phi c_psi)
 *            (the supplement calls the in-plane angle tau in the construction
 *            and psi in the derivatives);
 *   shape -> (u_lambda, u_a, u_k, zeta): lambda = e^u, a = e^u,
 *            k = 20 (tanh u + 1), zeta unchanged (0 for the paper's carrier);
 *   rgbw  -> u_w: w = tanh u.
 *   Gradients are returned with respect to these raw values, in the same
 *   slots (the unused fourth frame slot gets 0): Supplementary F's frame
 *   derivatives chained through the activations, evaluated in a form that
 *   stays finite where a cosine saturates.
 */
#ifndef NASG_H
#define NASG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nasg_status {
  NASG_OK = 0,
  NASG_ERR_NULL = -1,      /* a required pointer is NULL                      */
  NASG_ERR_SHAPE = -2,     /* n < 0, k outside [1, NASG_MAX_LOBES], v outside
                              [1, NASG_MAX_VIEWS], dirs given with v != 1, or
                              compositing: image side or tile capacity out of
                              range, n >= 2^31                                */
  NASG_ERR_ALIGN = -3,     /* a pointer is not aligned as the layout requires */
  NASG_ERR_DTYPE = -4,     /* unknown storage dtype                           */
  NASG_ERR_MODE = -5,      /* unknown normaliser, gradient mode, lobe
                              parametrisation or lobe family                  */
  NASG_ERR_LAUNCH = -6,    /* the HIP runtime rejected a launch               */
  NASG_ERR_WORKSPACE = -7  /* batched or compositing: workspace too small, or
                              (batched) missing or stale                      */
} nasg_status;

enum { NASG_MAX_LOBES = 64, NASG_MAX_VIEWS = 4096 };

typedef enum nasg_dtype { NASG_F32 = 0, NASG_BF16 = 1 } nasg_dtype;

/* Normaliser of each lobe.
 * EXACT : 1 / I, I = pi (1 - e^{-2 lam}) / (lam sqrt(1+a)) (1 + cos(zeta) Psi),
 *         Psi = 2 Lam e^{-Lam} sinhc(sqrt(Lam^2 - k^2)) / (1 - e^{-2 Lam}),
 *         Lam = lam (1 + a): the closed-form integral of Section 5.1 (the phase
 *         multiplies Psi by cos zeta; zeta = 0 is the printed formula).
 * APPROX: C^{-1} = lam sqrt(1+a) / (2 pi (1 - e^{-2 lam})), the NASG
 *         normaliser that ignores the carrier (Section 5.1, used for the
 *         paper's results; Supplementary E/F).                                */
typedef enum nasg_norm { NASG_NORM_EXACT = 0, NASG_NORM_APPROX = 1 } nasg_norm;

typedef enum nasg_grad_mode { NASG_GRAD_OVERWRITE = 0, NASG_GRAD_ACCUMULATE = 1 } nasg_grad_mode;

/* What the quat / shape / rgbw slots hold (see "Lobe parametrisation"). */
typedef enum nasg_param { NASG_PARAM_QUAT = 0, NASG_PARAM_ANGLES = 1 } nasg_param;

/* Lobe family (the spherical functions of the paper's distribution table,
 * Supplementary A), evaluated on the same skeleton: rgb = c0 + sum w G. The
 * frame slot is read as for NASGabor; the shape slot holds the family's
 * values (unused entries are ignored and get zero gradients):
 *   NASGABOR : (lambda, a, k, zeta), normaliser per `norm` (Section 5.1).
 *   NASG     : (lambda, a, -, -): NASGabor without carrier (Supplementary E)
 *              with its exact normaliser lambda sqrt(1+a)/(2 pi (1-e^{-2 lambda}));
 *              also accepts NASG_PARAM_ANGLES (k and zeta unused).
 *   SG       : (lambda, -, -, -): lambda/(2 pi (1-e^{-2 lambda})) e^{lambda (z.d-1)}.
 *   SB       : (beta >= 0, -, -, -): (beta+1)/(2 pi) (z.d)^beta on z.d > 0, else 0
 *              (the hemisphere normalisation of Supplementary D).
 *   SC       : (rho in [0, 1), -, -, -):
 *              1/(4 pi) ((1 - rho^2)/(1 + rho^2 - 2 rho z.d))^2 (the spherical
 *              Cauchy distribution the table cites; its printed
 *              "1 - rho^2 - 2 rho z.d" is not a density).
 *   ASG      : (mu, lambda, -, -): max(z.d, 0) e^{-mu (x.d)^2 - lambda (y.d)^2},
 *              y = z x x, no normaliser (the table gives none).
 * SG, SB, SC and ASG take NASG_PARAM_QUAT only; `norm` is validated but used
 * by NASGabor only. The families other than NASGabor use a fixed lane
 * mapping by view count (tuning entries set the block size only) and are not
 * accepted by the persistent batch (NASG_ERR_MODE).                          */
typedef enum nasg_family {
  NASG_FAMILY_NASGABOR = 0,
  NASG_FAMILY_NASG = 1,
  NASG_FAMILY_SG = 2,
  NASG_FAMILY_SB = 3,
  NASG_FAMILY_SC = 4,
  NASG_FAMILY_ASG = 5
} nasg_family;

typedef struct nasg_params {
  const void* quat;   /* [K][N][4]  f32 or bf16                               */
  const void* shape;  /* [K][N][4]  f32 or bf16                               */
  const void* rgbw;   /* [K][3][N]  f32 or bf16                               */
  const float* c0;    /* [N][3]                                               */
  int64_t n;          /* primitives                                           */
  int32_t k;          /* lobes per primitive, 1..NASG_MAX_LOBES               */
  int32_t dtype;      /* nasg_dtype of quat / shape / rgbw                    */
  int32_t param;      /* nasg_param (NASG_ERR_MODE if unknown)                */
  int32_t family;     /* nasg_family (NASG_ERR_MODE if unknown or if the
                         family does not take `param`)                        */
} nasg_params;

typedef struct nasg_views {
  const float* means; /* [N][3]  used when dirs == NULL                       */
  const float* cams;  /* [V][3]  used when dirs == NULL                       */
  const float* dirs;  /* [N][3]  optional raw directions (then v must be 1)   */
  int32_t v;          /* views, 1..NASG_MAX_VIEWS                             */
} nasg_views;

/* Gradient outputs, float32, same layouts as the inputs. Any pointer may be
 * NULL to skip that gradient. `geom` receives dL/dmeans [N][3] (camera mode:
 * summed over views) or dL/ddirs [N][3] (direction mode). Camera centres get
 * no gradient.                                                               */
typedef struct nasg_grads {
  float* quat;        /* [K][N][4]                                            */
  float* shape;       /* [K][N][4]  (dL/dlam, dL/da, dL/dk, dL/dzeta)        */
  float* rgbw;        /* [K][3][N]                                            */
  float* c0;          /* [N][3]                                               */
  float* geom;        /* [N][3]                                               */
} nasg_grads;

/* Forward: rgb[V][N][3] = c0 + sum_l w_l G_l(d) (Section 4.2 appearance model,
 * Section 5.1 lobe). `norm` is a nasg_norm.                                  */
int nasg_eval_fwd(const nasg_params* p, const nasg_views* views, float* rgb,
                  int32_t norm, void* stream);

/* Backward: gradients of L = sum grad_rgb * rgb w.r.t. quat, shape, rgbw, c0
 * and means (or dirs), following the product-rule derivatives of
 * Supplementary F (plus the derivative of the EXACT normaliser, and
 * dG/dd = s_x x + s_z z where dG/dx = s_x d, dG/dz = s_z d). Lobe gradients
 * are summed over all V views of the call. If `rgb` is not NULL the forward
 * colours are written too (fused forward+backward, one pass over the
 * parameters). `grad_mode` is a nasg_grad_mode.                               */
int nasg_eval_bwd(const nasg_params* p, const nasg_views* views, const float* grad_rgb,
                  const nasg_grads* g, float* rgb, int32_t norm, int32_t grad_mode,
                  void* stream);

/* Degree-3 real SH (Section 3.2): rgb[V][N][3] = sum_{j<16} sh[j][c][i] Y_j(d),
 * real orthonormal basis from the complex harmonics with the Condon-Shortley
 * phase (Y_lm = sqrt2 Re Y_l^m for m > 0, sqrt2 Im Y_l^|m| for m < 0); no
 * offset or clamp. `sh` is float32 [16][3][N], 4 B aligned.                  */
int sh3_eval_fwd(const float* sh, int64_t n, const nasg_views* views, float* rgb,
                 void* stream);

/* Gradients of L = sum grad_rgb * rgb w.r.t. the SH coefficients (grad_sh,
 * [16][3][N]) and the means or dirs (grad_geom, [N][3]); either may be NULL.
 * `rgb` (nullable) also receives the forward colours.                        */
int sh3_eval_bwd(const float* sh, int64_t n, const nasg_views* views,
                 const float* grad_rgb, float* grad_sh, float* grad_geom, float* rgb,
                 int32_t grad_mode, void* stream);

/* ---- uneven multi-scene batches -------------------------------------------
 * Many independent scenes (different N, K and V), each evaluated exactly as
 * nasg_eval_bwd with a non-NULL rgb would (fused forward+backward, gradients
 * summed over that scene's views), in ONE persistent launch: the scenes are
 * cut into tiles of primitives, the tiles are ordered by cost (tile size x K x
 * V, largest first) and a grid of `blocks_per_cu` blocks per compute unit
 * pulls them from a device work queue. Each scene runs the lane mapping the
 * tuning table (nasg_set_tuning, kernel 1, its K and V, float32) holds for
 * it when the batch kernel carries that mapping -- (1, 1), (1, 2), (1, 4),
 * (4, 2) or (4, 4) -- and otherwise the smallest of these whose view chunk
 * holds its views (V = 1, 2, 3..4, 5..8, more). Gradient sums stay per primitive in
 * registers and lanes (the queue counter is the only atomic). Lobe parameters
 * must be float32 (NASG_F32).
 *
 * Use: nasg_batched_workspace_bytes -> caller allocates device memory ->
 * nasg_batched_plan (host side: validates every scene, builds the tile list,
 * copies it to the workspace and waits for that copy; not capturable) ->
 * nasg_batched_run any number of times (launches only: capturable into a
 * hipGraph). A plan stays valid while the workspace and every scene buffer
 * stay allocated; re-planning into the same workspace makes older nasg_batch
 * handles stale, and a stale handle's run does nothing on the device.       */
typedef struct nasg_scene {
  nasg_params p;          /* dtype must be NASG_F32                           */
  nasg_views views;
  const float* grad_rgb;  /* [V][N][3]                                        */
  nasg_grads g;           /* as for nasg_eval_bwd (NULL entries skipped)      */
  float* rgb;             /* [V][N][3] or NULL                                */
} nasg_scene;

typedef struct nasg_batch_tuning {
  int32_t tile_iters;     /* 256-thread block passes per tile, 1..64          */
  int32_t blocks_per_cu;  /* persistent blocks per compute unit, 1..8         */
} nasg_batch_tuning;

typedef struct nasg_batch { /* filled by nasg_batched_plan                    */
  void* workspace;
  size_t bytes;
  int32_t n_items;        /* tiles in the work list                           */
  int32_t n_scenes;
  int32_t grid;           /* persistent blocks launched by nasg_batched_run   */
  int32_t norm;
  uint64_t token;         /* identifies the plan written to the workspace     */
  int32_t raw;            /* 1 if a scene has the paper's raw values: the run
                             then launches the kernel that carries their lane
                             mappings too (more registers spilled)            */
  int32_t pad;
} nasg_batch;

/* Device bytes needed for the plan of these scenes (host-side computation;
 * `t` may be NULL for the defaults: 4 tile passes, 2 blocks per CU).        */
size_t nasg_batched_workspace_bytes(const nasg_scene* scenes, int32_t n_scenes,
                                    const nasg_batch_tuning* t);

/* Validate the scenes (same rules as nasg_eval_bwd), build and upload the
 * tile list into `workspace` (device, >= nasg_batched_workspace_bytes) on
 * `stream`, wait for the upload, and describe the plan in *out.              */
int nasg_batched_plan(const nasg_scene* scenes, int32_t n_scenes, int32_t norm,
                      const nasg_batch_tuning* t, void* workspace, size_t ws_bytes,
                      nasg_batch* out, void* stream);

/* Run a plan: one queue-reset kernel and one persistent kernel on `stream`.
 * No allocation, copy or synchronisation: capturable into a hipGraph.       */
int nasg_batched_run(const nasg_batch* b, void* stream);

/* ---- compositing into an image (Section 3.1) ------------------------------
 * C(pixel) = sum_i T_i alpha_i c_i over the primitives on the pixel's ray in
 * depth order, alpha_i = min(sigma_i rho_i, 0.99), T_i = prod_{j<i}(1 -
 * alpha_j), black background, no early termination. Each primitive is a 3D
 * Gaussian, Sigma = R S S^T R^T (Section 3.1's primitive), and rho_i is the
 * Gaussian projected onto the image plane by the local affine approximation
 * of the perspective map at its mean, evaluated at the pixel centre
 * (px + 1/2, py + 1/2):
 *   x_cam = R_cw x + t; u = fx X/Z + cx, v = fy Y/Z + cy;
 *   Sigma_2 = J R_cw Sigma R_cw^T J^T, J = [[fx/Z, 0, -fx X/Z^2],
 *                                         [0, fy/Z, -fy Y/Z^2]];
 *   rho = exp(-q/2), q = delta^T Sigma_2^{-1} delta, delta = centre - (u, v).
 * A primitive reaches a pixel only where q <= 9 and only if Z > 0.2; depth
 * order is by Z of the mean, ties by primitive index. The colours are any
 * per-primitive RGB, typically one view's rgb from nasg_eval_fwd (the
 * central-ray colour of Section 5.2), so that the backward's grad_colors is
 * the grad_rgb of nasg_eval_bwd for that view.
 *
 * Work is binned into 16 x 16-pixel tiles. Each tile keeps at most
 * `tile_capacity` (1..NASG_MAX_TILE_CAPACITY) primitives; when a tile
 * overflows, the extra primitives are dropped from it and the int32 at byte
 * offset 0 of the workspace is set nonzero (read it after the forward to
 * detect an incomplete image). All pointers are device pointers; nothing is
 * allocated, copied or synchronised, so both calls can be captured. */
enum { NASG_MAX_TILE_CAPACITY = 4096, NASG_MAX_IMAGE_SIDE = 32768 };

typedef struct nasg_camera {
  double rot[9];      /* world-to-camera rotation R_cw, row-major             */
  double t[3];        /* x_cam = R_cw x + t                                   */
  double fx, fy, cx, cy;
  int32_t width, height; /* pixels, 1..NASG_MAX_IMAGE_SIDE                    */
} nasg_camera;

typedef struct nasg_gaussians {
  const float* means;   /* [N][3]                                             */
  const float* scales;  /* [N][3] per-axis standard deviations (> 0)          */
  const float* rots;    /* [N][4] quaternion (w, x, y, z), any nonzero norm   */
  const float* opac;    /* [N]    sigma in [0, 1]                             */
  const float* colors;  /* [N][3] colour composited for this camera           */
  int64_t n;            /* 0..2^31-1 (n == 0 still writes a black image)      */
} nasg_gaussians;

/* Device bytes of the workspace for n primitives, this camera and capacity
 * (0 for invalid arguments). Layout, each part 256-byte aligned: header
 * (int32 overflow flag at offset 0, int32 stale flag at offset 4, the
 * forward's sizes from offset 16), tile cursors [tiles] int32, tile lists
 * [tiles][capacity] of 64-bit sort keys, render records [N] (64 B each), bin
 * records [N] (16 B each), the final
 * transmittance per pixel [H][W][2] FP64 (mantissa, power-of-two exponent)
 * and the FP64 gradient accumulators [N][10]. The workspace must be 256-byte
 * aligned. */
size_t nasg_raster_workspace_bytes(int64_t n, const nasg_camera* cam, int32_t tile_capacity);

/* Forward: image[H][W][3] (float32, every pixel written; transmittance and
 * colour sums are carried in FP64, rho in FP32). Leaves the projection, the
 * depth-sorted tile lists and each pixel's final transmittance in
 * `workspace` for the backward. */
int nasg_raster_fwd(const nasg_gaussians* g, const nasg_camera* cam, int32_t tile_capacity,
                    void* workspace, size_t ws_bytes, float* image, void* stream);

/* Backward of L = sum grad_image * image with respect to the colours
 * (grad_colors [N][3]), the opacities (grad_opac [N]) and, through rho, the
 * geometry: means [N][3], scales [N][3] and quaternions [N][4] (float32, the
 * layouts of the inputs). Every output may be NULL and is overwritten; the
 * geometry terms are computed only when one of their outputs is given.
 * dC/dc_i = alpha_i T_i; dC/dalpha_i = T_i c_i - S_i / (1 - alpha_i) with S_i
 * the colour composited behind i, evaluated back to front as
 * T_i (c_i - R_{i+1}), R_k = alpha_k c_k + (1 - alpha_k) R_{k+1};
 * dalpha/dsigma = rho and dalpha/dq = -sigma rho / 2 below the clamp, 0 at
 * it; q = delta^T Sigma_2^{-1} delta is differentiated through the pixel
 * mean, Sigma_2 = M M^T, M = J R_cw R(q/|q|) S and J (FP64 chain per
 * primitive). The support cut, the near plane and the clamp are held fixed
 * (their jumps have no derivative). Camera parameters get no gradient.
 * `workspace` must hold the forward's state for the same inputs, camera and
 * tile capacity: the backward reads the projected primitives, colours and
 * opacities from it (of `g` only the means, scales and rots are read, by the
 * geometry chain) and overwrites only its accumulator part, so it may be
 * repeated. A workspace holding no forward of the same n, tile grid and
 * capacity is detected on the device before any list is read: the backward
 * then computes nothing (every gradient output is zero) and sets the int32 at
 * byte offset 4 of the workspace nonzero.
 * Per-pixel terms are summed per wavefront in registers and then into FP64
 * per-primitive accumulators with atomics, so the float32 results are
 * reproducible up to the order of those FP64 additions. */
int nasg_raster_bwd(const nasg_gaussians* g, const nasg_camera* cam, int32_t tile_capacity,
                    void* workspace, size_t ws_bytes, const float* grad_image,
                    float* grad_colors, float* grad_opac, float* grad_means,
                    float* grad_scales, float* grad_rots, void* stream);

/* ---- compositing forward without allocation --------------------------------
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid it): nasg_raster_fwd with its
 * workspace taken from a fixed device array inside the library instead of a
 * caller buffer. Same inputs, image and kernels as nasg_raster_fwd; the
 * overflow flag, which nasg_raster_fwd leaves at workspace byte 0, is copied
 * to `overflow` (a device int32, nullable). The array holds
 * NASG_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU the library runs on, from the
 * first call on that GPU until the process ends; a forward whose workspace
 * (nasg_raster_workspace_bytes) exceeds it returns NASG_ERR_WORKSPACE and
 * launches nothing. Nothing is allocated, freed or synchronised. Every call
 * on one GPU uses that GPU's array and leaves its state there (each call
 * clears what must start at zero), so calls that overlap on one GPU (other
 * streams, other threads) race; a backward cannot follow this forward (use
 * nasg_raster_fwd with a caller workspace for training).                    */
#define NASG_NOALLOC_SCRATCH_BYTES (64u << 20)

int nasg_raster_fwd_noalloc(const nasg_gaussians* g, const nasg_camera* cam,
                            int32_t tile_capacity, float* image, int32_t* overflow,
                            void* stream);

/* ---- achievable HBM rate (measurement) -------------------------------------
 * Streams `bytes` (a multiple of 16) through HBM with plain 16-byte accesses:
 * NASG_STREAM_READ reads src (dst: at least 16 bytes, written only in a case
 * that no real buffer produces, so the reads cannot be optimised away),
 * NASG_STREAM_WRITE writes dst, NASG_STREAM_COPY copies src to dst (both
 * `bytes` long, not overlapping). `blocks` 256-thread blocks (1..2^20) stride
 * over the buffer, each thread keeping `unroll` (1, 2, 4 or 8) accesses in
 * flight; `nontemporal` (0 or 1) marks the accesses as streaming. Pointers
 * are device pointers, 16-byte aligned. Asynchronous on `stream`; nothing is
 * allocated. Used to measure the HBM ceiling the appearance kernels are
 * compared with beside the 8 TB/s specification.                            */
enum { NASG_STREAM_READ = 0, NASG_STREAM_WRITE = 1, NASG_STREAM_COPY = 2 };

int nasg_hbm_stream(int32_t mode, const void* src, void* dst, int64_t bytes, int32_t blocks,
                    int32_t unroll, int32_t nontemporal, void* stream);

/* ---- camera-spacing statistic (Section 4, implementation details) ---------
 * The appearance learning rates are scaled with how densely the cameras
 * sample the scene: d_knn is the distance from each camera centre to its k
 * nearest other centres (the paper uses k = 3), averaged over the k
 * neighbours and then over the cameras. `centres` is [n_cams][3] FP64,
 * finite; per_camera[i] (FP64, n_cams entries) receives camera i's mean
 * distance to its k nearest others (coincident centres count, at distance
 * 0), and mean[0] (one FP64) their average over the cameras, summed in a
 * fixed order, so repeated calls give identical bits. All three are device
 * pointers, 8-byte aligned, owned by the caller. 1 <= k <= NASG_KNN_MAX_K and
 * k < n_cams <= NASG_KNN_MAX_CAMERAS, else NASG_ERR_SHAPE; NULL pointers
 * give NASG_ERR_NULL, misaligned ones NASG_ERR_ALIGN. Asynchronous on
 * `stream` (two launches); nothing is allocated.                          */
enum { NASG_KNN_MAX_K = 32, NASG_KNN_MAX_CAMERAS = 1 << 16 };

int nasg_camera_knn(const double* centres, int32_t n_cams, int32_t k, double* per_camera,
                    double* mean, void* stream);

/* Human-readable name of a status code (static storage).                    */
const char* nasg_status_string(int status);

/* ---- launch tuning --------------------------------------------------------
 * The evaluators map each primitive to `lanes` consecutive lanes of a
 * wavefront (1, 2, 4, 8 or 16); lane j owns lobes j, j + lanes, ... With
 * bcast = 0 the views travel: each lane holds `views_per_lane` views of a
 * chunk of lanes * views_per_lane and passes them round the group, so every
 * lobe meets every view. With bcast = 1 every lane holds the same
 * `views_per_lane` views (a chunk of that many) and the per-view colour and
 * direction-gradient sums are reduced over the group afterwards: for few
 * views, it spreads a primitive's lobes over the lanes. V larger than a chunk
 * is processed in chunks, accumulated in place, so any accepted mapping
 * serves any V. Accepted (lanes, views_per_lane): bcast = 0: (1, 1), (1, 2),
 * (1, 4), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2), (4, 4), (8, 1), (8, 2),
 * (16, 1); bcast = 1 (NASGabor kernels 0 and 1 only): (4, 1), (8, 1),
 * (16, 1), (8, 2), (8, 4); others return NASG_ERR_SHAPE. nasg_set_tuning
 * overrides the built-in
 * choice for a (kernel, K, V, dtype) key; nasg_get_tuning reports the choice
 * that a call with that key would use. kernel: 0 = NASG forward, 1 = NASG
 * backward / fused, 2 = SH forward, 3 = SH backward. K is ignored for SH.
 * lanes = 0 removes an override. Host-side table, not thread-safe against
 * concurrent calls.                                                         */
typedef struct nasg_tuning {
  int32_t lanes;
  int32_t views_per_lane;
  int32_t block;       /* threads per block: 64, 128 or 256 (the kernels are
                          compiled for at most 256; other values return
                          NASG_ERR_SHAPE)                                     */
  int32_t bcast;       /* 0: travelling views, 1: broadcast views (above)     */
} nasg_tuning;

int nasg_set_tuning(int32_t kernel, int32_t k, int32_t v, int32_t dtype,
                    const nasg_tuning* t);
int nasg_get_tuning(int32_t kernel, int32_t k, int32_t v, int32_t dtype, nasg_tuning* t);

#ifdef __cplusplus
}
#endif

#endif /* NASG_H */
