// Device-side types and launchers of the reflectometry workload (Sec. 6.2):
// a closed box of diffuse walls and spheres, one sphere with the unknown
// modified Phong BRDF theta = (kappa_s, gamma), and a point light.
#pragma once

#include "launch.hpp"

namespace prt {

constexpr int kMaxSpheres = 64;
// per sphere in the device table: centre (3), radius, albedo, 1 / radius
constexpr int kSphStride = 6;
// largest set of images tallied in one workgroup's LDS (FP64)
constexpr int64_t kSurfImageLds = 64 * 1024;

struct SurfScene {
    double box;               // box [0, box]^3
    double wall_albedo[6];    // x=0, x=box, y=0, y=box, z=0, z=box
    double light[3];
    double intensity;         // radiant intensity of the point light
    int n_spheres, phong, max_order;
    const double* sph;        // device [n_spheres][kSphStride]
};

// Device view of a store of surface paths (rows of n paths per vertex order).
struct SurfStore {
    int64_t n;
    int32_t* B;               // [n] surface vertices per path
    double4* pos;             // [M][n] vertex positions (w unused)
    int32_t* sid;             // [M][n] surface ids (walls 0..5, sphere k at 6 + k)
    double2* tv;              // [M][n] drawn direction: {cos to mirror, cos to normal}, diffuse {rho, -1}
    double2* tc;              // [M][n_cams][n] {geometric factor, cos of camera direction to mirror}
    int32_t* pix;             // [M][n_cams][n] pixel or -1
    double* theta_ref;        // device [2] (written by the draw)
    const double* omega;      // [n_cams][W*H] reciprocal pixel solid angles
    unsigned long long* work; // [2]: ray-sphere tests and vertices of the last draw
};

// Largest theta_ref a draw takes: at kappa_s = 1 the diffuse part would never
// be drawn, so recycled estimates at kappa_s < 1 would miss it.
constexpr double kKappaRefMax = 0.999;
constexpr double kGammaRefMax = 1e4;

// theta_ref of a draw: {kappa, gamma} as given, or, when src is set, the
// device pair src[0..1] read by the draw and clamped to [0, kKappaRefMax] x
// [0, kGammaRefMax].
struct DrawTheta {
    double kappa, gamma;
    const double* src;
};

// omega[d][p] = 1 / solid angle of pixel p of camera d
hipError_t launch_surf_omega(hipStream_t stream, const DevCams& c, double* omega);
// Draw st.n paths (ids first_id ..) at theta_ref with their tape, and store
// theta_ref at st.theta_ref.
hipError_t launch_surf_draw(hipStream_t stream, const SurfScene& s, const DevCams& c, const SurfStore& st,
                            uint64_t seed, uint64_t first_id, const DrawTheta& th, int n_cu);
// The tape of the stored positions.
hipError_t launch_surf_tape(hipStream_t stream, const SurfScene& s, const DevCams& c, const SurfStore& st, int n_cu);
// Number of per-workgroup partial images the render writes (0: the images
// exceed the LDS and the render adds into the output with FP64 atomics).
int surf_render_parts(int64_t n, int n_cams, int npx, int n_cu);
// img (device [n_cams][npx]) = recycled images; part holds
// surf_render_parts(...) x n_cams x npx doubles.  w0 = 4 pi I0 / N.
hipError_t launch_surf_render(hipStream_t stream, const SurfStore& st, int n_cams, int npx, double w0,
                              const double* theta, double* img, double* part, int n_cu);
// Number of per-workgroup pairs of the gradient and reweight passes.
int surf_pair_blocks(int64_t n, int n_cu);
hipError_t launch_surf_grad(hipStream_t stream, const SurfStore& st, int n_cams, int npx, double w0,
                            const double* theta, const double* res, double* part, double* grad, int n_cu);
// stats (device [2]) = {mean r, effective sample size}
hipError_t launch_surf_reweight(hipStream_t stream, const SurfStore& st, const double* theta, double* part,
                                double* stats, int n_cu);
hipError_t launch_surf_adam(hipStream_t stream, double* theta, const double* g, double* m, double* v, double lr0,
                            double lr1, double b1, double b2, double eps, double bc1, double bc2);

}  // namespace prt
