/*
 * prt_surface.h -- C ABI of the reflectometry workload of Czerninski &
 * Schechner, "Accelerating Inverse Rendering By Using a GPU and Reuse of
 * Light Paths" (arXiv 2110.00085), Sec. 6.2: recovering the BRDF parameters
 * theta = (kappa_s, gamma) of one sphere (Eq. phong) in a closed box of
 * diffuse walls and spheres lit by a point light, with recycled light paths
 * (Sec. 5.2, Alg. 2).  Same library, contexts and conventions as prt.h
 * (status codes, prt_last_error, asynchronous calls on the context's stream,
 * caller-owned device buffers).
 *
 * The model.
 *  - Surface ids: walls x=0, x=L, y=0, y=L, z=0, z=L are 0..5; sphere k is
 *    6 + k.  Wall normals point into the box, sphere normals outwards.
 *  - BRDFs (Eq. fs, surface case): diffuse surfaces rho/pi; the unknown
 *    sphere the modified Phong model f = (1-kappa)/pi + kappa (gamma+2)/(2 pi)
 *    max(0, w_r . w_out)^gamma, w_r the mirror image of the arriving
 *    propagation direction about the normal (the energy-conserving reading of
 *    Eq. phong, diffuse and specular weights summing to one).
 *  - Paths (Sec. 3.4, forward path tracing from the light): a uniform
 *    direction from the light (Philox event 0: u0 -> cosine 1 - 2 u0 about
 *    +z, u1 -> azimuth), the nearest surface is vertex 1; at vertex b a new
 *    direction from Philox event b: diffuse surfaces cosine-weighted about
 *    the normal (cosine sqrt(u1), azimuth 2 pi u2); the unknown sphere the
 *    Phong lobe about w_r (cosine u1^(1/(gamma_ref+1))) when u0 < kappa_ref,
 *    else cosine-weighted; a lobe direction below the surface ends the path.
 *    At most max_order vertices.
 *  - Images (Eq. forward_simualtion_recycling with local estimation): every
 *    vertex connects to every camera it sees (camera on the outer side of the
 *    surface, no sphere between); a pixel averages radiance over its solid
 *    angle, as in prt.h.
 *  - Loss gradient (Eq. loss_gradient, Eq. gradient_simualtion_recycling):
 *    PSF (Eq. total_derivative_factor) = sum of d log f over the unknown
 *    sphere's bounces before a vertex and its connection to the camera.
 *  - theta of the render, gradient, reweight and Adam calls is a DEVICE
 *    array of 2 doubles {kappa_s, gamma}, so a loop of render, loss,
 *    gradient and Adam runs without host round trips; theta_ref of a draw is
 *    a HOST array (it is validated), or a DEVICE array for
 *    prt_surface_resample_device (it is clamped).
 */
#ifndef PRT_SURFACE_H
#define PRT_SURFACE_H

#include "prt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct prt_surface_paths_s* prt_surface_paths;

#define PRT_SURFACE_MAX_SPHERES 64

/* The closed box [0,box]^3: wall albedos (ids 0..5), the point light
   (position strictly inside the box and outside every sphere, radiant
   intensity > 0), n_spheres <= PRT_SURFACE_MAX_SPHERES spheres given by
   HOST arrays center[n][3], radius[n] > 0, albedo[n] (each sphere inside the
   box), phong = index of the sphere with the unknown BRDF (-1: none), and
   max_order in [1, PRT_MAX_ORDER].  Albedos lie in [0, 1]. */
typedef struct {
    double box;
    double wall_albedo[6];
    double light[3];
    double intensity;
    int32_t n_spheres, phong, max_order, pad;
    const double* center;
    const double* radius;
    const double* albedo;
} prt_surface_scene;

/* Draw n_paths >= 1 paths (ids 0 .. n_paths-1 of stream `seed`) at the HOST
   theta_ref[2] (0 <= kappa_s < 1, so that every direction the BRDF reaches
   can be drawn; 0 <= gamma <= 1e4) and build their tape
   (every theta-independent quantity of the render, gradient and correction
   factor: cosines, visibility, pixels, geometric factors) for the cameras
   `cams` (positions in scene units, strictly inside the box and outside every
   sphere; at most PRT_MAX_CAMERAS).  The store keeps theta_ref, the scene and
   the cameras.  *out receives a new store. */
int prt_surface_sample(prt_ctx ctx, const prt_surface_scene* scene, const prt_cameras* cams,
                       const double* theta_ref, uint64_t seed, int64_t n_paths, prt_surface_paths* out);

/* The same draw into an existing store (Alg. 2, resampling every N_r
   iterations): buffers are reused when large enough; theta_ref (HOST) is
   passed to the draw by value. */
int prt_surface_resample(prt_ctx ctx, prt_surface_paths paths, const prt_surface_scene* scene,
                         const prt_cameras* cams, const double* theta_ref, uint64_t seed, int64_t n_paths);

/* As prt_surface_resample with theta_ref a DEVICE array of 2 doubles (as
   theta of the render calls), read when the draw runs and clamped to the
   drawable range kappa_s in [0, 0.999], gamma in [0, 1e4] (NaN counts as
   0): the loop of Alg. 2 can redraw at its current theta without a host
   round trip.  The store keeps the clamped value.  Asynchronous when the
   scene's spheres and the cameras are those of the store's previous draw
   and its buffers are large enough; otherwise it synchronises first. */
int prt_surface_resample_device(prt_ctx ctx, prt_surface_paths paths, const prt_surface_scene* scene,
                                const prt_cameras* cams, const double* theta_ref, uint64_t seed, int64_t n_paths);

/* A store from HOST paths: B[n] vertex counts in [0, max_order], pos[n][M][3]
   and sid[n][M] (M = max_order; entries past B[i] ignored), drawn at the
   HOST theta_ref[2]; the tape is built as after sampling.  Synchronises. */
int prt_surface_import(prt_ctx ctx, const prt_surface_scene* scene, const prt_cameras* cams,
                       const double* theta_ref, int64_t n_paths, const int32_t* B, const double* pos,
                       const int32_t* sid, prt_surface_paths* out);

/* Copy a store to HOST arrays laid out as for prt_surface_import (entries
   past B[i] are zero / -1).  Synchronises. */
int prt_surface_export(prt_ctx ctx, prt_surface_paths paths, int32_t* B, double* pos, int32_t* sid);

/* Number of paths and max_order of a store. */
int prt_surface_info(prt_surface_paths paths, int64_t* n_paths, int32_t* max_order);

/* Work of the store's last draw (zero for an imported store): ray-sphere
   tests (n_spheres per nearest-surface query of a traced ray and per
   occlusion query of a camera connection in the image) and stored vertices.
   Synchronises. */
int prt_surface_work(prt_ctx ctx, prt_surface_paths paths, uint64_t* sphere_tests, uint64_t* vertices);

/* Recycled images F(theta | theta_ref) (Eq. forward_simualtion_recycling):
   images (device FP64 [n_cams][H][W]) are overwritten. */
int prt_surface_render(prt_ctx ctx, prt_surface_paths paths, const double* theta, double* images);

/* d loss / d theta for residual = F - I_gt (device FP64 [n_cams][H][W]):
   grad (device [2]) is overwritten. */
int prt_surface_grad(prt_ctx ctx, prt_surface_paths paths, const double* theta, const double* residual,
                     double* grad);

/* Correction-factor statistics at theta (Eq. correction factor, in log
   space): stats (device [2]) = {mean r, effective sample size
   (sum r)^2 / sum r^2}.  Does not synchronise. */
int prt_surface_reweight(prt_ctx ctx, prt_surface_paths paths, const double* theta, double* stats);

/* One Adam step (Kingma & Ba; step count t >= 1, per-parameter step sizes)
   on theta (device [2], updated in place with moments m, v (device [2])),
   then the projection 0 <= kappa_s <= 1, gamma >= 0. */
int prt_surface_adam(prt_ctx ctx, double* theta, const double* grad, double* m, double* v, int32_t t,
                     double lr_kappa, double lr_gamma, double b1, double b2, double eps);

void prt_surface_destroy(prt_surface_paths paths);

#ifdef __cplusplus
}
#endif

#endif /* PRT_SURFACE_H */
