/*
 * prt.h -- C ABI of the MI355X (gfx950) path-recycling scattering-tomography
 * library.  The operations follow Czerninski & Schechner, "Accelerating
 * Inverse Rendering By Using a GPU and Reuse of Light Paths" (arXiv 2110.00085):
 * sampling light paths (Sec. 3.4), sorting them by size (Sec. 5.3), rendering
 * images from recycled paths (Sec. 5.2, Eq. forward_simualtion_recycling with
 * local estimation, Sec. 3.4.3), the loss gradient (Eq. loss_gradient with the
 * recycled derivative estimator, Eq. gradient_simualtion_recycling, and the
 * tomography path score function of Sec. 4.4), the correction factor
 * statistics that decide when to resample (Eq. correction factor, Alg. 2),
 * the appearance loss (Eq. appearance_loss) and the Adam update (Sec. 6).
 *
 * Conventions shared by every call
 *  - Grid: nx*ny*nz voxels of edge voxel_km [km]; box [0,nx]x[0,ny]x[0,nz] in
 *    grid units, z up; voxel v = ix + nx*(iy + ny*iz) (x fastest).
 *  - Extinction fields are float32 device arrays in 1/km; the air extinction
 *    is a constant added everywhere inside the box; vacuum outside.
 *  - Unless stated otherwise pointers to fields, images and gradients are
 *    DEVICE pointers owned by the caller; the library never frees caller
 *    memory.  Calls are asynchronous on the context's stream unless stated:
 *    caller buffers must stay valid until the stream has passed the call.
 *  - Every call returns PRT_OK (0) or a negative prt_status; prt_last_error()
 *    then gives a thread-local message.  No exception crosses the ABI.
 *    Arguments are validated before any work is enqueued.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = 64-bit seed,
 *    counter = (path id, event, 0); event 0 draws the entry point and the first
 *    optical depth, event b >= 1 the particle type, scattering cosine, azimuth
 *    and next optical depth at scatter b.  Paths are therefore reproducible
 *    one by one from (seed, path id) on any device.
 */
#ifndef PRT_H
#define PRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct prt_ctx_s* prt_ctx;
typedef struct prt_paths_s* prt_paths;

enum prt_status {
    PRT_OK = 0,
    PRT_E_INVALID = -1,   /* bad argument (null, size, non-finite or out-of-range value) */
    PRT_E_NOMEM = -2,     /* device or host allocation failed */
    PRT_E_CAPACITY = -3,  /* a size exceeds a documented limit */
    PRT_E_MISMATCH = -4,  /* scene grid differs from the grid the paths were sampled on */
    PRT_E_HIP = -5        /* a HIP runtime call or kernel launch failed */
};

enum prt_precision {
    PRT_TRAVERSAL_FP32 = 0,  /* voxel traversal (lengths, optical depths) in FP32; all else FP64 */
    PRT_ALL_FP64 = 1         /* everything in FP64 */
};

#define PRT_MAX_CAMERAS 24
#define PRT_MAX_ORDER 64
#define PRT_MAX_DIM 512   /* voxels per grid axis */

/* Scene (Sec. 4.4 and Sec. 6.1): cloud extinction beta_c on the grid (the
   unknowns), constant air extinction, the two single-scattering albedos
   (Eq. sinscat), the Henyey-Greenstein asymmetry g of the cloud phase
   function, Rayleigh air, and a sun of flux sun_flux with parallel rays from
   (zenith, azimuth) in degrees.  max_order caps the number of scattering
   events of a sampled path (1..PRT_MAX_ORDER).  Validated on every call:
   1 <= nx, ny, nz <= PRT_MAX_DIM (PRT_E_CAPACITY beyond), finite values, beta_air >= 0, 0 < albedos <= 1, |g| < 1, 0 <= zenith < 90,
   sun_flux > 0, voxel_km > 0. */
typedef struct {
    int32_t nx, ny, nz, max_order;
    double voxel_km;
    double beta_air;
    double albedo_cloud;
    double albedo_air;
    double g;
    double sun_zenith_deg;
    double sun_azimuth_deg;
    double sun_flux;
    const float* beta_cloud;   /* device [nz][ny][nx], 1/km, >= 0 (not checked element-wise) */
} prt_scene;

/* Pinhole cameras (Sec. 6.1): n <= PRT_MAX_CAMERAS cameras sharing the image
   size; HOST arrays, copied at each call.  rot is world->camera with rows
   (right, up, forward); a point x projects to u = f (R(x-c)).x/(R(x-c)).z + W/2,
   v = f (R(x-c)).y/(R(x-c)).z + H/2, pixel (floor(v), floor(u)) when
   0 <= u < W, 0 <= v < H and (R(x-c)).z > 0.  Images are [n][H][W] of the
   pixel-averaged radiance: the pixel response is 1/Omega_p with Omega_p the
   exact solid angle of the pixel (reading of the response W_d, Sec. 3.3). */
typedef struct {
    int32_t n, width, height, pad;
    const double* pos;   /* host [n][3], km */
    const double* rot;   /* host [n][3][3] row-major */
    const double* f_px;  /* host [n], focal length in pixels */
} prt_cameras;

/* Work counters accumulated by the context since the last reset.
   voxel_segments: nonzero-length (ray piece, voxel) intersections visited by
   free-flight segments and in-image connections (each pass counts its own);
   local_estimates: in-image (scatter, camera) connections; paths: stored paths
   processed by prt_render; overhead_segments: extra traversals done only to scatter the
   gradient along connections already traversed for their transmittance. */
typedef struct {
    uint64_t voxel_segments;
    uint64_t local_estimates;
    uint64_t paths;
    uint64_t overhead_segments;
} prt_counters_t;

typedef struct {
    uint64_t n_paths;       /* N, including paths that never scattered */
    uint64_t n_vertices;    /* stored vertex records including batch padding */
    uint64_t n_batches;     /* wavefront batches of 64 paths */
    uint64_t seed;
    uint64_t bytes;         /* device bytes held by the store */
    int32_t max_order, nx, ny, nz;
} prt_paths_info_t;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` using `hip_stream` (a hipStream_t,
   borrowed, may be NULL for the null stream) and a precision mode.  The
   context owns its scratch memory. */
int prt_create(int device, void* hip_stream, int precision, prt_ctx* out);
/* Destroy a context after waiting for all work on its device.  Stores built
   with it stay valid. */
void prt_destroy(prt_ctx ctx);
int prt_set_stream(prt_ctx ctx, void* hip_stream);
/* Largest temporary, in bytes, that prt_sample / prt_resample may allocate to
   draw the paths in one pass (kept by the context for later draws).  A draw
   takes, in this order of preference: whole rows of max_order + 2 vertex
   records of 16 bytes per path; rows of 2 records per path (entry and exit:
   all a path without a scatter needs) plus a pool of 128-byte segments of 7
   records that the sampler's wavefronts claim as paths grow, chained per
   path, with 4 bytes per path for its first segment -- the pool sized from
   the store's previous draw with a margin (a new store takes a segment for
   half of its paths and needs room for a quarter), cut to what the limit
   leaves; or, when neither fits (the pool does not hold the estimate), or
   the pool runs out, two passes per path
   from its Philox stream: first only its size and sort key, then, once the
   sort (Sec. 5.3) has fixed its place, its vertices straight into the store.
   All give the same store; the second pass checks every path's size against
   the first and fails with PRT_E_HIP otherwise.  Default 40 GiB; 0 always
   takes two passes. */
int prt_set_sample_scratch_limit(prt_ctx ctx, uint64_t bytes);
/* Thread-local text of the last error (never NULL). */
const char* prt_last_error(void);

/* --------------------------------------------------------------- paths */

/* Resample (Alg. 2, "Sample" then "Sort" then "set reference"): draw n_paths
   i.i.d. paths from the path-tracing pdf mu(.|beta) of Eq. final_mu with the
   sun as source (entry point uniform over the box's projected area, distance
   sampling Sec. 3.4.1, particle type with probability beta_s^(j)/beta_s and
   its phase function, Sec. 3.4.2; at most max_order scatters), sort them by
   size B with a stable counting sort (Sec. 5.3), lay them out in
   wavefront-batch order, and snapshot beta_cloud as the reference parameters.
   The store is owned by the library (free with prt_paths_destroy).
   Synchronises the stream (the store size depends on the sampled paths).
   n_paths in [1, 2^31 - 64]. */
int prt_sample(prt_ctx ctx, const prt_scene* scene, uint64_t seed, uint64_t n_paths, prt_paths* out);

/* Resample into an existing store (Alg. 2 after the first iteration): the
   same operation as prt_sample, reusing the store's device buffers when they
   are large enough (the store may change grid or size).  On failure the store
   is left valid and empty.  Synchronises. */
int prt_resample(prt_ctx ctx, const prt_scene* scene, uint64_t seed, uint64_t n_paths, prt_paths paths);

/* Build a store from host paths in CSR form: vertex k of path i is
   xyz[3*(off[i]+k)..] (grid units, float) with voxel vox[off[i]+k]; B[i]
   scatters; vertices 1..B[i] are scatter points with voxel ids in range,
   vertex 0 is the entry point (its voxel in range), and when B[i] < max_order
   the last vertex is the exit point with voxel -1 (so off[i+1]-off[i] is
   B[i]+2, or B[i]+1 when B[i] == max_order).  beta_ref is the HOST float
   field the paths were drawn from.  Host arrays are read before return.
   Synchronises. */
int prt_paths_import(prt_ctx ctx, const prt_scene* scene, uint64_t n_paths, const int64_t* off,
                     const float* xyz, const int32_t* vox, const int32_t* B, const float* beta_ref,
                     uint64_t seed, prt_paths* out);

/* Copy a store back to HOST arrays in path-id order (same CSR form as
   prt_paths_import; off has n_paths+1 entries, xyz/vox hold the number of
   vertices given by off[n_paths]).  Pass NULL for xyz/vox/beta_ref to get
   only off and B.  Synchronises. */
int prt_paths_export(prt_ctx ctx, prt_paths paths, int64_t* off, float* xyz, int32_t* vox,
                     int32_t* B, float* beta_ref);

/* Stable sort permutation of the store (sorted position -> path id), HOST
   int32 array of n_paths entries.  Synchronises. */
int prt_paths_permutation(prt_ctx ctx, prt_paths paths, int32_t* perm);

int prt_paths_info(prt_paths paths, prt_paths_info_t* info);
/* Free a store.  Independent of the context that built it (which may be
   destroyed first); waits for all work on the store's device. */
void prt_paths_destroy(prt_paths paths);

/* ------------------------------------------------------------ hot path */

/* Recycled forward model (Eq. forward_simualtion_recycling_factor with local
   estimation, Eq. Qd): images[d][p] = (1/N) sum_i sum_{b<=min(B_i,max_order_render)}
   c_{b,d}/Omega_p over the stored paths, where c is the MCF of the sub-path
   x_0..x_b -> camera d at beta_t = scene->beta_cloud divided by its sampling
   pdf at the store's reference field.  `images` (device FP64 [n][H][W]) is
   overwritten.  scene grid/max_order must equal the store's. */
int prt_render(prt_ctx ctx, const prt_scene* scene, const prt_cameras* cams, prt_paths paths,
               int32_t max_order_render, double* images);

/* Loss gradient on the stored paths (Eq. loss_gradient with Eq.
   gradient_simualtion_recycling and the tomography PSF, Sec. 4.4):
   grad[v] = sum_{d,p} residual[d][p] dF_{d,p}/dbeta_c[v], i.e. the vector-
   Jacobian product of prt_render (all orders) with `residual` (device FP64
   [n][H][W], e.g. F - I_gt for the loss of Eq. appearance_loss).  `grad`
   (device FP64 [nz][ny][nx]) is overwritten. */
int prt_grad(prt_ctx ctx, const prt_scene* scene, const prt_cameras* cams, prt_paths paths,
             const double* residual, double* grad);

/* Correction-factor statistics (Eq. correction factor over whole sampled
   paths, computed in log space in FP64): mean_r = (1/N) sum_i r_i and the
   effective sample size ess = (sum r)^2 / sum r^2, written to HOST doubles.
   Synchronises and reports any pending kernel error. */
int prt_reweight(prt_ctx ctx, const prt_scene* scene, prt_paths paths, double* mean_r, double* ess);

/* The statistics of prt_reweight without allocating, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc): stats is a caller-owned DEVICE buffer of
   2 doubles, set to {mean r, ess} on the context's stream; the call does not
   synchronise.  Its scratch (per-workgroup sums of r and r^2 and, for grids
   whose field beta_t - beta_ref exceeds the LDS, that field) is a fixed
   device array of PRT_NOALLOC_SCRATCH_BYTES inside the library, one per GPU,
   held until the process ends; a call needing more returns PRT_E_CAPACITY
   before launching anything (16 MiB hold the field of 4 Mi voxels with FP32
   traversal, 2 Mi in the all-FP64 mode).  Every call on one GPU, from any
   context, uses that GPU's array: calls that overlap on a GPU race.  The
   result equals prt_reweight's bit for bit.  No device memory is allocated
   or freed. */
#define PRT_NOALLOC_SCRATCH_BYTES (16u << 20)
int prt_reweight_noalloc(prt_ctx ctx, const prt_scene* scene, prt_paths paths, double* stats);

/* Appearance loss (Eq. appearance_loss): residual[i] = images[i] - target[i]
   and *loss = 0.5 sum residual^2 (all device FP64; n elements). */
int prt_loss(prt_ctx ctx, int64_t n, const double* images, const double* target, double* residual,
             double* loss);

/* One Adam step (Kingma & Ba; moment decays b1, b2, step size lr, epsilon
   eps, step count t >= 1) on the FP64 master field beta[n] with gradient
   grad[n] and moments m[n], v[n] (all device FP64, updated in place), then
   projection beta >= 0 and an FP32 copy into beta_f32[n] (device). */
int prt_adam(prt_ctx ctx, int64_t n, double* beta, float* beta_f32, const double* grad, double* m,
             double* v, int32_t t, double lr, double b1, double b2, double eps);

/* Space carving (Sec. 6.1: the reconstruction starts from the photo hull of
   the images, after Kutulakos & Seitz, filled with the mean extinction of the
   cloud).  Voxel v is removed (mask[v] = 0) when some camera d sees the
   centre of v (the projection of prt_cameras) on a pixel p with
   images[d][p] <= threshold[d]; a camera that does not see the centre
   (behind it, or outside its image) removes nothing; otherwise mask[v] = 1.
   images: device FP64 [n][H][W]; threshold: HOST double [n] (NaN rejected);
   mask: device uint8 [nz][ny][nx], overwritten; beta_out: optional device
   float32 [nz][ny][nx], set to fill_value (finite, >= 0) where kept and 0
   elsewhere.  scene gives the grid geometry (its beta_cloud is not read). */
int prt_space_carve(prt_ctx ctx, const prt_scene* scene, const prt_cameras* cams, const double* images,
                    const double* threshold, double fill_value, uint8_t* mask, float* beta_out);

/* -------------------------------------------- path-sorting ablation */

/* The paper's GPU design for comparison (Sec. 5.3, path sorting): one thread
   per stored path walks all of its scatters and cameras, as the paper's
   kernels do, on a per-path copy of the store taken in `order`:
   PRT_ORDER_BY_SIZE (the store's order, sorted by path size as Alg. 2's
   "Sort" step) or PRT_ORDER_BY_ID (the order the paths were drawn in, i.e.
   no sorting).  The copy is built on first use after each (re)fill of the
   store and kept with it.  prt_tpp_render computes the images of
   prt_render (all orders; FP64 atomics on the images); prt_tpp_grad the
   gradient of prt_grad, recomputing every contribution (LDS slab tallies or
   FP64 atomics, as prt_grad without a tape).  Same arguments, layouts,
   ownership and errors as prt_render / prt_grad; PRT_E_INVALID for another
   order.  Async. */
#define PRT_ORDER_BY_SIZE 0
#define PRT_ORDER_BY_ID 1
int prt_tpp_render(prt_ctx ctx, const prt_scene* scene, const prt_cameras* cams, prt_paths paths, int32_t order,
                   double* images);
int prt_tpp_grad(prt_ctx ctx, const prt_scene* scene, const prt_cameras* cams, prt_paths paths, int32_t order,
                 const double* residual, double* grad);

/* Coarse-to-fine measurements (Sec. 6.1: the reconstruction starts from
   down-sampled images and raises the resolution when the loss saturates).
   images: device FP64 [n][H][W] of the cameras cams (pixel-averaged
   radiance); coarse: device FP64 [n][H/factor][W/factor], overwritten with
   the solid-angle-weighted mean of each factor x factor block of pixels,
   which is the pixel-averaged radiance of the same pinhole camera with focal
   length f/factor and image sides divided by factor.  H and W must be
   multiples of factor (PRT_E_INVALID otherwise).  Async. */
int prt_downsample_images(prt_ctx ctx, const prt_cameras* cams, const double* images, int32_t factor,
                          double* coarse);

/* Reconstruction errors of Sec. 6: errors[0] = epsilon = ||b* - b||_1 /
   ||b*||_1 (relative L1 distance) and errors[1] = delta = (||b*||_1 -
   ||b||_1) / ||b*||_1 (relative mass bias) of the estimate beta_est (device
   FP64 [n]) against the true field beta_true (device FP32 [n]); errors is a
   device FP64 [2].  Sums in a fixed order.  Async. */
int prt_volume_errors(prt_ctx ctx, int64_t n, const double* beta_est, const float* beta_true, double* errors);

/* ----------------------------------------------------------- telemetry */

/* Read (and optionally reset) the work counters.  Synchronises. */
int prt_counters(prt_ctx ctx, prt_counters_t* out, int reset);

/* Per-kernel timing with HIP events on the context's stream.  enable != 0
   starts recording an event pair around every hot-path kernel launch;
   prt_kernel_times synchronises and returns, for kernel ids 0..n-1 (see
   prt_kernel_name), total milliseconds and launch counts since the last
   reset.  Returns the number of kernel ids. */
int prt_enable_timing(prt_ctx ctx, int enable);
/* As prt_enable_timing, for the kernel ids whose bit is set in kernel_mask
   only (0 stops recording): each event pair adds a little to the stream, so a
   timed run can record just the kernel it reports. */
int prt_enable_timing_mask(prt_ctx ctx, uint32_t kernel_mask);
int prt_kernel_times(prt_ctx ctx, double* total_ms, int64_t* launches, int n, int reset);
const char* prt_kernel_name(int id);

#ifdef __cplusplus
}
#endif
#endif /* PRT_H */
