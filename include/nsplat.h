/* nsplat.h -- C ABI of the MI355X (gfx950) NURBS Splatting render path.
 *
 * The path (Qiu & Zhou, "NURBS Splatting", Sec. 3):
 *   nsplat_sample    key points -> NURBS (Sec. 3.1) -> isotropic Gaussians:
 *                    contour samples (Sec. 3.2, Eq. 3-5) and the SDF-modulated
 *                    interior grid of filled closed curves (Sec. 3.3, Eq. 6-7,
 *                    Suppl. S2 Eq. S1-S3)
 *   nsplat_bin       Gaussians -> per-tile lists in stacking order (Sec. 3.4)
 *   nsplat_forward   front-to-back alpha compositing (Sec. 3.4, Eq. 8-9)
 *   nsplat_backward  exact adjoint of the three steps above, from dL/dImage to
 *                    the key points, weights, widths, knot intervals, colours
 *                    and opacities (the differentiability claim of Sec. 1/3.4)
 *
 * Conventions shared by every entry point
 *   - Pointers marked (dev) are device pointers, (host) host pointers.  All
 *     memory is owned by the caller; the library never allocates or frees
 *     caller memory.  Internal scratch lives in the caller's workspace
 *     (nsplat_workspace_size).
 *   - Every call is stream-ordered on `stream` (a hipStream_t; NULL = the
 *     default stream), never synchronises the device and never allocates, so
 *     a sequence of calls can be captured into a HIP graph.  The only host
 *     synchronising helper is nsplat_read_counters.
 *   - Sizes that change from step to step (Gaussians, tile pairs, boundary
 *     points) are computed on the device and stored in `counters`; buffers are
 *     sized by capacities.  If a capacity is exceeded the excess is not
 *     written (for the tile pairs: no pair is written, the pair count is 0
 *     and every tile list is left empty), the required size is stored and a
 *     status bit is set; the caller reads the counters, grows the buffer and
 *     calls again.
 *   - Return value: NSPLAT_OK, or an error code with a message available from
 *     nsplat_last_error.  Argument checks run on the host before any device
 *     work is issued.  Value errors that only the device can see (a curve with
 *     degree outside [1, NSPLAT_MAX_DEGREE], too few key points, a filled
 *     curve that is not closed, a wrong interval count) set
 *     NSPLAT_STATUS_DATA; such a curve produces no Gaussians.  Values outside
 *     the domain of Sec. 3.1 (a rational weight w_i <= 0, a stroke width
 *     <= 0, a knot interval < 0, intervals that sum to 0 so that the curve
 *     has no parameter domain, or a non-finite key point, weight, width,
 *     interval, colour or opacity) set NSPLAT_STATUS_VALUE, and such a curve
 *     too produces no Gaussians and receives zero gradients.  Both mark the
 *     curve NSPLAT_PLAN_INVALID in the plan.
 *   - Coordinates are pixels, y pointing down; pixel (x, y) has its centre at
 *     (x + 1/2, y + 1/2); a canvas spans [0, W] x [0, H].
 */
#ifndef NSPLAT_H
#define NSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NSPLAT_OK 0
#define NSPLAT_EINVAL 1     /* bad argument, detected on the host            */
#define NSPLAT_ECAPACITY 2  /* workspace or buffer smaller than required     */
#define NSPLAT_EHIP 3       /* a HIP runtime call failed                     */

#define NSPLAT_CLOSED 1     /* curve flag: closed (periodic knots, wrapped control polygon) */
#define NSPLAT_FILLED 2     /* curve flag: filled interior (requires CLOSED) */
/* curve flag: tangent-aligned (anisotropic) contour Gaussians instead of the
 * isotropic ones of Eq. 5, the contour sampling of Bezier Splatting that
 * Sec. 3.2 contrasts with (and the "BS Proto." of the supplementary
 * comparison): sample j gets the axis s_j / rho across the curve and
 * max(s_j / rho, |C'(u_j)| du / rho) along t_j = C'(u_j) / |C'(u_j)| (Eq. 2;
 * du the samples' spacing in u), and the count M = ceil(delta_a L).  A stroke
 * only: ANISO with FILLED is invalid data. */
#define NSPLAT_ANISO 4
#define NSPLAT_MAX_DEGREE 5

/* Version of the structure layouts below; nsplat_abi_version() returns the
 * value the library was built with, so a binding can refuse a library whose
 * structures it would misread. */
#define NSPLAT_ABI_VERSION 7

/* counters[] layout (dev int32[NSPLAT_NUM_COUNTERS]) */
#define NSPLAT_CNT_GAUSS 0      /* Gaussians produced (<= capacity)          */
#define NSPLAT_CNT_PAIRS 1      /* (tile, Gaussian) pairs produced           */
#define NSPLAT_CNT_STATUS 2     /* OR of NSPLAT_STATUS_* bits                */
#define NSPLAT_CNT_GAUSS_REQ 3  /* Gaussians required                        */
#define NSPLAT_CNT_PAIRS_REQ 4  /* pairs required                            */
#define NSPLAT_CNT_BOUND_REQ 5  /* boundary points required                  */
#define NSPLAT_CNT_BOUND 6      /* boundary points produced                  */
#define NSPLAT_NUM_COUNTERS 16

#define NSPLAT_STATUS_GAUSS_CAP 1   /* Gaussian capacity exceeded             */
#define NSPLAT_STATUS_PAIR_CAP 2    /* pair capacity exceeded                 */
#define NSPLAT_STATUS_BOUND_CAP 4   /* boundary-point capacity exceeded       */
#define NSPLAT_STATUS_DATA 8        /* invalid curve data (see above)         */
#define NSPLAT_STATUS_VALUE 16      /* a curve with invalid values (see above) */

/* Timed phases (nsplat_timing_read); each is one kernel unless noted. */
#define NSPLAT_T_PLAN 0        /* knots, arc length, counts, boundary, scans (5 kernels) */
#define NSPLAT_T_EMIT 1        /* Gaussian records                              */
#define NSPLAT_T_BIN 2         /* tile counts, their scan, pair emission        */
#define NSPLAT_T_SORT 3        /* all radix passes                              */
#define NSPLAT_T_RANGES 4      /* tile ranges                                   */
#define NSPLAT_T_BLEND_FWD 5   /* forward compositing                           */
#define NSPLAT_T_BLEND_BWD 6   /* compositing adjoint                           */
#define NSPLAT_T_ADJ_GAUSS 7   /* per-Gaussian sample adjoint                   */
#define NSPLAT_T_ADJ_BOUND 8   /* boundary-point adjoint                        */
#define NSPLAT_T_FOLD 9        /* zeroing and the fold to key points / tau      */
#define NSPLAT_T_REG 10        /* geometric regularisers (nsplat_backward_reg)  */
#define NSPLAT_NUM_TIMERS 11

/* plan[] row layout (dev int32[n_curves][NSPLAT_PLAN_STRIDE]) */
#define NSPLAT_PLAN_COUNT 0   /* Gaussians of the curve                        */
#define NSPLAT_PLAN_NSAMP 1   /* contour samples M (Sec. 3.2) or boundary points (Sec. 3.3) */
#define NSPLAT_PLAN_IX0 2     /* fill lattice window: first column index       */
#define NSPLAT_PLAN_IY0 3     /*                      first row index          */
#define NSPLAT_PLAN_NX 4      /*                      columns                  */
#define NSPLAT_PLAN_NY 5      /*                      rows                     */
#define NSPLAT_PLAN_GOFF 6    /* index of the curve's first Gaussian           */
#define NSPLAT_PLAN_BOFF 7    /* index of the curve's first boundary point     */
#define NSPLAT_PLAN_FLAGS 8   /* NSPLAT_PLAN_NEAR_INT | NSPLAT_PLAN_INVALID    */
#define NSPLAT_PLAN_STRIDE 9

/* Plan flags of a curve, rewritten by every nsplat_sample (frozen or not).
 * NEAR_INT: delta L (delta_c L for strokes, delta_b L for fills) lies within
 * 1e-9 of an integer, so the count M = ceil(delta L) of Sec. 3.2 / 3.3 could
 * round to either side under another summation order of the arc length.
 * INVALID: the curve has invalid data or values and produces no Gaussians
 * (its counts are set to 0, also under frozen != 0). */
#define NSPLAT_PLAN_NEAR_INT 1
#define NSPLAT_PLAN_INVALID 2

typedef struct nsplat_ctx nsplat_ctx;

/* Curves, CSR over curves (Sec. 3.1).  Curves must be grouped by scene in
 * ascending scene order; the Gaussian index order (curve by curve) is the
 * stacking order: a later curve is drawn over an earlier one. */
typedef struct {
  int32_t n_curves;        /* (host)                                         */
  int32_t channels;        /* (host) 1 or 3                                  */
  int32_t n_keys;          /* (host) total key points K                      */
  int32_t n_taus;          /* (host) total knot intervals                    */
  int32_t max_degree;      /* (host) an upper bound on every degree[c] in
                              [1, NSPLAT_MAX_DEGREE]; any other value means
                              NSPLAT_MAX_DEGREE.  A curve above it counts as
                              invalid data.  A bound of 3 or less selects
                              adjoint kernels with smaller register arrays */
  int32_t any_flags;       /* (host) the union (bitwise or) of flags[c] over
                              the batch, or a superset of it; a curve with a
                              flag outside it counts as invalid data.
                              Without NSPLAT_ANISO the blend kernels run
                              their forms without the tangent-aligned kind,
                              without NSPLAT_FILLED the fill adjoints are not
                              launched                                    */
  int32_t all_flags;       /* (host) the intersection (bitwise and) of
                              flags[c] over the batch, or a subset of it (0
                              declares nothing); a curve without one of its
                              flags counts as invalid data.  With
                              NSPLAT_FILLED (every curve filled) the stroke
                              adjoint is not launched                     */
  const int32_t* scene;    /* (dev) [n_curves] scene of each curve           */
  const int32_t* degree;   /* (dev) [n_curves] p                             */
  const int32_t* flags;    /* (dev) [n_curves] NSPLAT_CLOSED | NSPLAT_FILLED | NSPLAT_ANISO */
  const int32_t* key_off;  /* (dev) [n_curves+1] into the key arrays         */
  const int32_t* tau_off;  /* (dev) [n_curves+1] into tau; open curves hold
                              n_k - p intervals, closed curves n_k           */
  const float* key_xy;     /* (dev) [K][2] key points K_i                    */
  const float* key_w;      /* (dev) [K] rational weights w_i > 0             */
  const float* key_s;      /* (dev) [K] stroke widths (third coordinate) > 0 */
  const float* tau;        /* (dev) knot intervals tau_j >= 0                */
  const float* color;      /* (dev) [n_curves][channels]                     */
  const float* opacity;    /* (dev) [n_curves]                               */
} nsplat_curves;

typedef struct {
  int32_t n_scenes;        /* (host)                                         */
  const int32_t* hw_host;  /* (host) [S][2] = {H, W}                         */
  const int32_t* hw;       /* (dev)  [S][2], same values                     */
  const float* bg;         /* (dev)  [S][channels] background colour         */
} nsplat_scenes;

/* Method constants (Table S1 of the paper) and rasteriser settings. */
typedef struct {
  float delta_c;    /* contour density, samples per px of arc length (10)    */
  float delta_b;    /* fill boundary density (0.5)                           */
  float rho;        /* global scale ratio, sigma = s / rho (2)               */
  float eta;        /* fill coverage factor, sigma = eta h / rho (1.5)       */
  float gamma;      /* SDF sigmoid sharpness (5)                             */
  float nl_factor;  /* arc-length quadrature points N_L = nl_factor max(W,H) (3) */
  float fill_pad;   /* fill box padding, fraction of the box extent (0.1)    */
  float h;          /* fill grid step in px (1); see h_dev                   */
  float k_sigma;    /* support radius in sigmas (6)                          */
  float alpha_max;  /* per-pixel opacity clamp (0.99)                        */
  float eps_T;      /* a pixel stops once its transmittance drops below, in [0, 1] (1e-6) */
  float delta_a;    /* contour density of NSPLAT_ANISO strokes, samples per px (0.25) */
  int32_t kappa;    /* extra copies of each open-curve endpoint Gaussian (4) */
  int32_t tile;     /* tile side in px: 8, 16 or 32                          */
  int32_t batch;    /* Gaussians staged in LDS per block step: 32..256       */
  int32_t chunk;    /* list positions per chunk of the adjoint's split of each
                       tile list (the forward stores every pixel's state at
                       chunk boundaries; the adjoint runs one work item per
                       tile quadrant, or 8 x 8 block, and chunk): a power
                       of two in
                       [512, 8192], or 0: 512 for a batch without fills,
                       else chosen by nsplat_bin on the device from the pair
                       count (about pairs x quadrants per tile / (8 x compute
                       units), rounded to a power of two in [512, 8192]).
                       It only changes FP32 rounding.                        */
  const float* h_dev; /* (dev, optional) if non-NULL the grid step is read
                         from here, so a captured graph can anneal it        */
} nsplat_params;

typedef struct {
  int64_t gauss;      /* Gaussian records                                    */
  int64_t pairs;      /* (tile, Gaussian) pairs                              */
  int64_t boundary;   /* fill boundary points, all curves together           */
} nsplat_caps;

/* Buffers of one render state; all (dev) and caller-owned. */
typedef struct {
  int32_t* plan;      /* [n_curves][NSPLAT_PLAN_STRIDE]                      */
  void* gauss;        /* [caps.gauss] records of 32 bytes:
                         {double mx, my; float sigma, opacity; int32 curve, local};
                         sigma is the axis along the tangent for an
                         NSPLAT_ANISO curve's Gaussians, whose tangent and
                         axis across the curve live in the workspace */
  int32_t* ranges;    /* [n_tiles][2] slice [begin, end) of idx per tile     */
  int32_t* idx;       /* [caps.pairs] Gaussian indices, ascending within a tile;
                         front-to-back order is the slice read from its end  */
  int32_t* counters;  /* [NSPLAT_NUM_COUNTERS]                               */
  void* ws;           /* workspace, >= nsplat_workspace_size(...) bytes,
                         256-byte aligned; must be kept unchanged from
                         nsplat_sample to nsplat_backward                    */
  size_t ws_bytes;
  nsplat_caps caps;
} nsplat_buffers;

/* Parameter gradients (dev FP32, same shapes as the inputs; overwritten).  A
 * NULL pointer leaves that group out: it is not written (e.g. weights or knot
 * intervals held fixed, as in the ablations of Table 1). */
typedef struct {
  float* key_xy;  /* [K][2] */
  float* key_w;   /* [K]    */
  float* key_s;   /* [K]    */
  float* tau;     /* [n_taus] */
  float* color;   /* [n_curves][channels] */
  float* opacity; /* [n_curves] */
} nsplat_grads;

/* NSPLAT_ABI_VERSION as built (no device work).  Context: binds the library
 * to device `device` (made current by the caller's thread for every later
 * call).  Holds the last error message and the autotuner's choices.  A failed
 * nsplat_create (no such device, device set-up error) still stores a context
 * in *ctx that carries the message; the caller destroys it either way.  */
int nsplat_abi_version(void);
int nsplat_create(nsplat_ctx** ctx, int device);
int nsplat_destroy(nsplat_ctx* ctx);
const char* nsplat_last_error(const nsplat_ctx* ctx);

/* Number of tiles over all scenes for the given tile side (host only). */
int64_t nsplat_num_tiles(const nsplat_scenes* scenes, int32_t tile);

/* Workspace bytes for this batch shape and these capacities (host only). */
size_t nsplat_workspace_size(const nsplat_curves* curves, const nsplat_scenes* scenes,
                             const nsplat_params* params, const nsplat_caps* caps);

/* Sec. 3.1-3.3 (Eq. 1-7, S1-S3).  Builds knot vectors (cumulative sums of the
 * intervals), measures each curve's arc length (Eq. 3, N_L midpoints), sets
 * the counts M = ceil(delta_c L) (open >= 2, closed >= 3; open curves get
 * kappa extra copies of each endpoint) or N_b = max(3, ceil(delta_b L)) with
 * the fill lattice window, and writes one Gaussian record per sample: contour
 * samples at u_j uniform in [u_p, u_{m-p}] evaluated span-locally in FP64
 * (centre = C(u_j), sigma = s(u_j) / rho, opacity o), fill lattice points
 * q = ((i + 1/2) h, (j + 1/2) h) in the padded box with sigma = eta h / rho
 * and opacity o sigmoid(gamma / h sdf(q)).  frozen != 0 keeps the counts and
 * windows already in bufs->plan (piecewise-constant sampling, e.g. for finite
 * differences or graph replay) and only re-evaluates positions and opacities. */
int nsplat_sample(nsplat_ctx* ctx, const nsplat_curves* curves, const nsplat_scenes* scenes,
                  const nsplat_params* params, const nsplat_buffers* bufs, int frozen, void* stream);

/* Sec. 3.4 binning.  Each Gaussian covers the tiles of its conservative
 * rectangle, computed in FP32 from m = fl32(centre) and r = k_sigma * sigma as
 * [(m - r) - 1, (m + r) + 1] per axis.  Pairs are produced in Gaussian order
 * and sorted stably by (scene, tile) key with an LSD radix sort, so each
 * tile's slice of idx lists its Gaussians in ascending index. */
int nsplat_bin(nsplat_ctx* ctx, const nsplat_curves* curves, const nsplat_scenes* scenes,
               const nsplat_params* params, const nsplat_buffers* bufs, void* stream);

/* Eq. 8-9.  Per pixel, front to back (descending Gaussian index):
 * alpha = min(alpha_max, o exp(-|x - mu|^2 / (2 sigma^2))) for |x - mu| <=
 * k_sigma sigma, colour += c alpha T, T *= 1 - alpha, stop once T < eps_T;
 * image = colour + T bg.  Uses the tile lists and scene table built by the
 * last nsplat_bin on these buffers; NSPLAT_EINVAL if that call (on this
 * context) used another params.tile or params.chunk (the same holds for
 * nsplat_backward).  image is per scene [channels][H][W], concatenated
 * over scenes; T_final and n_last are per scene [H][W]: the final
 * transmittance and the idx position where the pixel stopped.
 * persistent != 0 runs one resident grid that pulls tiles from a device work
 * queue instead of one block per tile (same results, bit for bit). */
int nsplat_forward(nsplat_ctx* ctx, const nsplat_curves* curves, const nsplat_scenes* scenes,
                   const nsplat_params* params, const nsplat_buffers* bufs, float* image,
                   float* T_final, int32_t* n_last, int persistent, void* stream);

/* Adjoint of nsplat_forward o nsplat_bin o nsplat_sample for the upstream
 * gradient dL_dimage (layout of image).  Must follow the nsplat_forward of
 * the same buffers: it starts each chunk of a tile list (the chunk length
 * nsplat_bin chose) from the per-pixel state that forward stored in the
 * workspace at the chunk's back boundary, walks the chunk back to front
 * (from n_last where a pixel stopped inside it), and
 * chains through the Gaussians into the Cox-de Boor basis (control points,
 * weights, widths, knots -> intervals), the SDF (nearest segment, detached
 * sign), the sample parameters u_j (which depend on the domain ends) and the
 * key-point / interval parametrisation.  Counts, windows and span choices are
 * held fixed (piecewise constant).  All gradients are overwritten.
 * NSPLAT_EINVAL also when, at 32 x 32 tiles, the last nsplat_bin on these
 * buffers saw curves that differ from these in whether any is NSPLAT_FILLED:
 * it laid out the adjoint's work items per 8 x 8 pixel block for the tiles
 * of scenes with fills and per quadrant for the others. */
int nsplat_backward(nsplat_ctx* ctx, const nsplat_curves* curves, const nsplat_scenes* scenes,
                    const nsplat_params* params, const nsplat_buffers* bufs, const float* dL_dimage,
                    const float* T_final, const int32_t* n_last, const nsplat_grads* grads,
                    int persistent, void* stream);

/* Geometric regularisers of Sec. 3.5 added to the loss by nsplat_backward_reg.
 * Both are evaluated at the parameters u_j of each curve's own samples: the M
 * contour samples of a stroke (its endpoint copies counted once) and the N_b
 * boundary points of a fill.
 *   Bounding box (Eq. 12): bbox_weight * sum_j sum_{x,y} [phi(b_min - C(u_j))
 *     + phi(C(u_j) - b_max)], phi = ReLU (bbox_kind 0) or softplus (1), the box
 *     of each scene from `bbox` (dev FP32 [S][4] = {x_min, y_min, x_max, y_max})
 *     or, when bbox is NULL, the canvas [0, W] x [0, H].
 *   Derivative (Eq. 11): deriv_weight / n_scene * the domain average of
 *     ||C^(r)(u)||^2 for the planar curve (x, y), r = deriv_order in 1..3,
 *     taken with the trapezoid rule on an open curve's samples (both ends
 *     included) or the rectangle rule on a closed curve's, n_scene being the
 *     number of curves of the curve's scene (the loss averages over curves).
 *     C^(r) comes from the span's derivative control points (differences of
 *     the homogeneous control points over knot spans) evaluated with the
 *     degree p - k basis, and the rational Leibniz rule.
 * A weight of 0 switches a term off.  `loss` (dev FP32 [2], may be NULL)
 * receives the two terms' values (added to what it holds). */
typedef struct {
  float bbox_weight;
  int32_t bbox_kind;
  const float* bbox;
  float deriv_weight;
  int32_t deriv_order;
  float* loss;
} nsplat_reg;

/* nsplat_backward plus the gradients of the regularisers in `reg` (NULL: none;
 * then identical to nsplat_backward).  Needs the same state (nsplat_sample,
 * nsplat_bin and nsplat_forward of this step).  Errors as nsplat_backward, and
 * NSPLAT_EINVAL for a deriv_order outside 1..3 or a bbox_kind other than 0, 1. */
int nsplat_backward_reg(nsplat_ctx* ctx, const nsplat_curves* curves, const nsplat_scenes* scenes,
                        const nsplat_params* params, const nsplat_buffers* bufs, const float* dL_dimage,
                        const float* T_final, const int32_t* n_last, const nsplat_reg* reg,
                        const nsplat_grads* grads, int persistent, void* stream);

/* Distance-weighted image loss of the layer-wise vectorisation application
 * (Sec. 4.2: "udf_weight", with the weights of LIVE, Ma et al. 2022): for
 * every pixel centre q of a scene, d(q) = distance to the nearest boundary
 * segment of the scene's selected filled curves (the closed N_b-point
 * boundary polylines of Sec. 3.3 from this step's nsplat_sample; sel: dev
 * int32 [n_curves], nonzero = selected, or NULL for every filled curve),
 * w(q) = max(0, tau - d(q)) normalised to sum 1 over the scene (all 0 if no
 * pixel is within tau), and L = sum_q w(q) (1/C) sum_c (I_c(q) - I*_c(q))^2
 * with the weights held constant.  Writes dL/dImage to dL_dimage (dev FP32,
 * image layout) and adds L over all scenes to *loss (dev FP32, may be NULL).
 * NSPLAT_EINVAL for a NULL array or tau <= 0. */
int nsplat_udf_loss(nsplat_ctx* ctx, const nsplat_curves* curves, const nsplat_scenes* scenes,
                    const nsplat_params* params, const nsplat_buffers* bufs, const int32_t* sel, float tau,
                    const float* image, const float* target, float* dL_dimage, float* loss, void* stream);

/* nsplat_udf_loss for callers that cannot allocate device memory or bring
 * scratch of their own (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same arguments, results and errors,
 * but the per-scene weight sums live in a static device array of the library
 * (4096 doubles per device, held until the process ends) instead of the
 * workspace, and the call allocates nothing.  At most 4095 scenes
 * (NSPLAT_EINVAL above).  All calls on one device share that array, which
 * keeps the last call's sums (each call clears what it uses first): calls that
 * overlap on one device (different streams, or threads) race and give wrong
 * results.  The workspace in bufs is still read for the render state of this
 * step's nsplat_sample (boundary points, scene table). */
int nsplat_udf_loss_noalloc(nsplat_ctx* ctx, const nsplat_curves* curves, const nsplat_scenes* scenes,
                            const nsplat_params* params, const nsplat_buffers* bufs, const int32_t* sel, float tau,
                            const float* image, const float* target, float* dL_dimage, float* loss, void* stream);

/* Learnable parameters, writable (dev FP32; the arrays the curves point to). */
typedef struct {
  int32_t n_curves, channels, n_keys, n_taus;
  float* key_xy;   /* [K][2] */
  float* key_w;    /* [K]    */
  float* key_s;    /* [K]    */
  float* tau;      /* [T]    */
  float* color;    /* [N][C] */
  float* opacity;  /* [N]    */
} nsplat_values;

/* Optimiser settings of the supplementary material: Adam with per-group
 * learning rates (order key_xy, key_w, key_s, tau, color, opacity), each
 * decayed by a cosine from lr to final_ratio * lr over total_steps steps, and
 * the clamps of the rational weights to [w_min, w_max] and of the knot
 * intervals to [tau_min, tau_max] after every step. */
typedef struct {
  float lr[6];
  float beta1, beta2, eps;
  float final_ratio;
  int32_t total_steps;
  float w_min, w_max, tau_min, tau_max;
} nsplat_adam;

/* One Adam step (Kingma & Ba, Alg. 1, eps added to the bias-corrected root)
 * on every parameter, in place, at step t = *step_dev + 1 (dev int32: steps
 * taken so far; incremented), with learning rate
 * lr_t = lr (final_ratio + (1 - final_ratio) (1 + cos(pi min(1, (t - 1) / total_steps))) / 2).
 * m and v (dev FP32, each 4 K + T + N (C + 1) values, zero before the first
 * step) hold the moments, group after group in the order above. */
int nsplat_adam_step(nsplat_ctx* ctx, const nsplat_adam* cfg, const nsplat_values* params,
                     const nsplat_grads* grads, float* m, float* v, int32_t* step_dev, void* stream);

/* Eq. 14: writes h(t) = h_max + (h_min - h_max) (1 + cos(pi (1 - phi))) / 2,
 * phi = clamp((t / T - t_b) / (t_e - t_b), 0, 1), to h_dev (dev float), with t
 * read from step_dev (dev int32) when it is non-NULL (and then incremented),
 * else from `step`.  Lets a captured graph anneal the fill grid step. */
int nsplat_anneal_h(nsplat_ctx* ctx, float* h_dev, int32_t* step_dev, int32_t step, int32_t total_steps,
                    float h_max, float h_min, float t_b, float t_e, void* stream);

/* Helper kernels that a captured step needs: out[i] = 2 (a[i] - b[i]) for
 * i < n, and sum((a - b)^2) added into *loss (dev, FP32). */
int nsplat_l2_grad(nsplat_ctx* ctx, const float* a, const float* b, float* out, float* loss, int64_t n,
                   void* stream);

/* Per-phase timing.  nsplat_timing(ctx, 1) starts recording a HIP event pair
 * around every NSPLAT_T_* phase the library launches (on that call's stream)
 * and clears the sums; nsplat_timing(ctx, NSPLAT_TIMING_ONLY | mask) records
 * only the phases whose bits (1 << NSPLAT_T_*) are set in mask, so that one
 * kernel can be timed inside an otherwise unobserved run;
 * nsplat_timing(ctx, 0) stops.  nsplat_timing_read waits
 * for the recorded events, adds their elapsed times to ms[NSPLAT_NUM_TIMERS]
 * and launch counts to count[NSPLAT_NUM_TIMERS] (host arrays, overwritten
 * with the sums since the last enable) and recycles the events.  Not for use
 * under graph capture. */
#define NSPLAT_TIMING_ONLY 0x40000000
int nsplat_timing(nsplat_ctx* ctx, int enable);
int nsplat_timing_read(nsplat_ctx* ctx, double* ms, int64_t* count);

/* Copies the counters to host memory and waits for them (synchronising). */
int nsplat_read_counters(nsplat_ctx* ctx, const nsplat_buffers* bufs, int32_t* host_out, void* stream);

/* Frame of the tangent-aligned (NSPLAT_ANISO) stroke Gaussians of this
 * step's nsplat_sample (the contour variant of Eq. 5, Sec. 3.2): for the
 * first n Gaussians, out[4 g .. 4 g + 3] = (t_x, t_y, sp, sigma / sp): the
 * unit tangent C'(u) / |C'(u)| that the long axis (the record's sigma) lies
 * on, or (1, 0) where C'(u) = 0, sp = s(u) / rho, the axis across it, and
 * the axis ratio (exactly 1 where the two axes agree), each rounded once from
 * FP64.  The
 * entries of Gaussians of other kinds are unspecified.  out: dev FP32
 * [4 n], caller-owned; 0 <= n <= caps.gauss.  An asynchronous device copy on
 * `stream`.  NSPLAT_EINVAL for bad buffers, n outside that range or a NULL
 * out with n > 0. */
int nsplat_gauss_frame(nsplat_ctx* ctx, const nsplat_curves* curves, const nsplat_scenes* scenes,
                       const nsplat_buffers* bufs, float* out, int64_t n, void* stream);

/* Autotuner: times nsplat_bin + nsplat_forward + nsplat_backward on the given
 * state for every tile side in {8, 16, 32} and batch depth in
 * {32, 64, 128, 256} (after one warm-up each), returns the fastest in
 * *best_tile / *best_batch, and leaves the buffers, image and gradients as
 * nsplat_bin + nsplat_forward + nsplat_backward at that setting leave them.  The buffers must be sized for the largest tile
 * count (tile 8) and pair count (tile 8 has the most pairs).  times_ms, if
 * non-NULL, receives the 12 timings in (tile, batch) row-major order. */
int nsplat_autotune(nsplat_ctx* ctx, const nsplat_curves* curves, const nsplat_scenes* scenes,
                    const nsplat_params* params, const nsplat_buffers* bufs, float* image, float* T_final,
                    int32_t* n_last, const float* dL_dimage, const nsplat_grads* grads, int persistent,
                    int32_t* best_tile, int32_t* best_batch, float* times_ms, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NSPLAT_H */
