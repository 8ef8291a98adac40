// Reflectometry workload (Sec. 6.2): forward path tracing from a point light
// in a box of spheres, one of which carries the unknown modified Phong BRDF
// theta = (kappa_s, gamma) (Eq. phong), and the recycled image, gradient and
// correction-factor passes over the stored paths (Sec. 5.2).
//
// What the passes share is split by what depends on theta.  A path's
// vertices, normals, visibility to each camera, pixel, solid angle and all
// its cosines are fixed once the path is drawn, so one tape pass after each
// (re)draw stores, per vertex: the two cosines of the drawn direction (to the
// mirror direction and to the normal) and, per camera, the pixel, the
// geometric factor |n.w_c| / (r^2 Omega_pixel) and the cosine of the camera
// direction to the mirror direction.  Diffuse vertices fold their albedo in
// (continuation weight rho, local-estimate factor rho/pi times the geometric
// factor) and are flagged by a negative normal cosine.  The render, gradient
// and correction-factor passes then stream the tape, one lane per path, and
// evaluate only the BRDF of the unknown sphere at theta_t and the draw
// density at theta_ref (all FP64).
//
// Layout: vertex b of path i at [b * n + i] (one row per vertex order, lanes
// of a wavefront read consecutive paths); per-camera entries at
// [(b * n_cams + d) * n + i].
#include <algorithm>

#include "surface.hpp"

namespace prt {

namespace {

constexpr int kSurfBlock = 256;
constexpr double kPiD = 3.14159265358979323846;

__device__ __forceinline__ double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Ray p + t w against sphere k (p outside it): b = (p - c).w and the
// discriminant disc = b^2 - (|p - c|^2 - r^2); the ray enters the sphere
// ahead (at -b - sqrt(disc) > 0) when disc >= 0 and b < 0.
__device__ __forceinline__ void sphere_terms(const double* sph, int k, const double p[3], const double w[3], double& b,
                                             double& disc)
{
    const double ox = p[0] - sph[kSphStride * k], oy = p[1] - sph[kSphStride * k + 1], oz = p[2] - sph[kSphStride * k + 2];
    const double r = sph[kSphStride * k + 3];
    b = ox * w[0] + oy * w[1] + oz * w[2];
    disc = b * b - (ox * ox + oy * oy + oz * oz - r * r);
}

// Does the entry -b - sqrt(disc) lie in (0, tmax)?  Decided without the
// square root: sqrt(disc) > -b - tmax holds outright when -b < tmax, else it
// is disc > (b + tmax)^2.
__device__ __forceinline__ bool enters_before(double b, double disc, double tmax)
{
    const double e = b + tmax;
    return disc >= 0.0 && b < 0.0 && (e > 0.0 || disc > e * e);
}

// Nearest surface along p + t w, skipping surface `skip` (walls 0..5, then
// spheres): id (or -1) and its t.  A sphere's entry point (the square root)
// is formed only when it comes before the nearest surface found so far.
__device__ __forceinline__ int nearest_surface(const SurfScene& s, const double* sph, const double p[3],
                                               const double w[3], int skip, double& t_best)
{
    t_best = INFINITY;
    int id = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (w[a] == 0.0) continue;
        const int wall = w[a] > 0.0 ? 2 * a + 1 : 2 * a;
        if (wall == skip) continue;
        const double t = ((w[a] > 0.0 ? s.box : 0.0) - p[a]) / w[a];
        if (t > 0.0 && t < t_best) {
            t_best = t;
            id = wall;
        }
    }
#pragma unroll 2
    for (int k = 0; k < s.n_spheres; ++k) {
        double b, disc;
        sphere_terms(sph, k, p, w, b, disc);
        if (6 + k != skip && enters_before(b, disc, t_best)) {
            const double t = -b - sqrt(disc);
            if (t > 0.0 && t < t_best) {
                t_best = t;
                id = 6 + k;
            }
        }
    }
    return id;
}

// Is the segment from x (on surface sid) to a point at distance dist along
// w cut by another sphere?
__device__ __forceinline__ bool occluded(const SurfScene& s, const double* sph, int sid, const double x[3],
                                         const double w[3], double dist)
{
    bool hit = false;
#pragma unroll 2
    for (int k = 0; k < s.n_spheres; ++k) {
        double b, disc;
        sphere_terms(sph, k, x, w, b, disc);
        hit = hit || (6 + k != sid && enters_before(b, disc, dist));
    }
    return hit;
}

// Inward wall normal, outward sphere normal.
__device__ __forceinline__ void surface_normal(const double* sph, int sid, const double x[3], double n[3])
{
    if (sid < 6) {
        n[0] = n[1] = n[2] = 0.0;
        n[sid >> 1] = (sid & 1) ? -1.0 : 1.0;
        return;
    }
    const int k = sid - 6;
    const double ir = sph[kSphStride * k + 5];
    n[0] = (x[0] - sph[kSphStride * k]) * ir;
    n[1] = (x[1] - sph[kSphStride * k + 1]) * ir;
    n[2] = (x[2] - sph[kSphStride * k + 2]) * ir;
}

__device__ __forceinline__ void mirror_dir(const double w[3], const double n[3], double r[3])
{
    const double c = 2.0 * dot3(w, n);
    r[0] = w[0] - c * n[0];
    r[1] = w[1] - c * n[1];
    r[2] = w[2] - c * n[2];
}

__device__ __forceinline__ void unit_to(const double a[3], const double b[3], double w[3], double& len, double& il)
{
    const double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    len = sqrt(dx * dx + dy * dy + dz * dz);
    il = 1.0 / len;
    w[0] = dx * il;
    w[1] = dy * il;
    w[2] = dz * il;
}

__device__ __forceinline__ void unit_to(const double a[3], const double b[3], double w[3], double& len)
{
    double il;
    unit_to(a, b, w, len, il);
}

// Does surface sid carry the unknown BRDF?  (phong < 0: no sphere does)
__device__ __forceinline__ bool is_phong(const SurfScene& s, int sid) { return s.phong >= 0 && sid == 6 + s.phong; }

__device__ __forceinline__ double albedo_of(const SurfScene& s, const double* sph, int sid)
{
    return sid < 6 ? s.wall_albedo[sid] : sph[kSphStride * (sid - 6) + 4];
}

// Exact solid angle of pixel (row, col) of a pinhole camera with focal length
// f pixels: F(x,y) = atan(xy / (f sqrt(x^2+y^2+f^2))) is the solid angle of
// the rectangle [0,x]x[0,y] on the image plane, combined by inclusion-exclusion.
__device__ __forceinline__ double pixel_omega(double f, int W, int H, int row, int col)
{
    auto F = [f](double x, double y) { return atan(x * y / (f * sqrt(x * x + y * y + f * f))); };
    const double x1 = col - 0.5 * W, x2 = x1 + 1.0, y1 = row - 0.5 * H, y2 = y1 + 1.0;
    return F(x2, y2) - F(x1, y2) - F(x2, y1) + F(x1, y1);
}

// The spheres (centre, radius, albedo) into LDS, shared by the workgroup.
__device__ __forceinline__ const double* load_spheres(const SurfScene& s, double* lds)
{
    for (int i = threadIdx.x; i < kSphStride * s.n_spheres; i += blockDim.x) lds[i] = s.sph[i];
    __syncthreads();
    return lds;
}

// The unknown BRDF at theta and the draw density at theta_ref, from the
// cosine c to the mirror direction (and nc to the normal).
struct PhongTerms {
    double kappa, gamma, fa, fb;      // f = fa + fb c^gamma
    double rgamma, ra, rb;            // pdf = ra nc + rb c^rgamma
    __device__ __forceinline__ void init(const double* theta, const double* theta_ref)
    {
        kappa = theta[0];
        gamma = theta[1];
        fa = (1.0 - kappa) / kPiD;
        fb = kappa * (gamma + 2.0) / (2.0 * kPiD);
        rgamma = theta_ref[1];
        ra = (1.0 - theta_ref[0]) / kPiD;
        rb = theta_ref[0] * (rgamma + 1.0) / (2.0 * kPiD);
    }
    // c^gamma (0 for c <= 0) as exp(gamma log c), with lc = log c (0 for c <= 0)
    __device__ __forceinline__ double lobe_log(double c, double& lc) const
    {
        lc = c > 0.0 ? log(c) : 0.0;
        return c > 0.0 ? exp(gamma * lc) : 0.0;
    }
    __device__ __forceinline__ double f(double c) const
    {
        double lc;
        return fa + fb * lobe_log(c, lc);
    }
    // f(c) nc / pdf_ref(nc, c): the continuation weight of a drawn direction
    __device__ __forceinline__ double carry(double c, double nc) const
    {
        const double lc = c > 0.0 ? log(c) : 0.0;
        const double l = c > 0.0 ? exp(gamma * lc) : 0.0, lr = c > 0.0 ? exp(rgamma * lc) : 0.0;
        return (fa + fb * l) * nc / (ra * fmax(nc, 0.0) + rb * lr);
    }
};

// Sum over the workgroup of one double per thread (wavefront shuffles, then
// LDS); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double* lds)
{
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
    const int wv = threadIdx.x / kWave;
    __syncthreads();
    if (threadIdx.x % kWave == 0) lds[wv] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += lds[i];
    return t;
}

}  // namespace

// Reciprocal pixel solid angles of every camera, once per draw:
// omega[d * npx + p] = 1 / Omega.
__global__ void surf_omega_kernel(DevCams c, double* omega)
{
    const int npx = c.W * c.H;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= c.n * npx) return;
    const int d = k / npx, p = k % npx;
    omega[k] = 1.0 / pixel_omega(c.f[d], c.W, c.H, p / c.W, p % c.W);
}

namespace {

// The per-camera records of vertex b of path i at x (surface sid, normal n_,
// mirror direction r): pixel (or -1 when the camera does not see x) and
// {geometric factor, cosine of the camera direction to r}; a diffuse
// vertex's factor includes rho/pi.  Returns the number of occlusion queries.
__device__ __forceinline__ int camera_records(const SurfScene& s, const double* sph, const DevCams& c,
                                              const SurfStore& st, int b, int64_t i, const double x[3], int sid,
                                              const double n_[3], const double r[3], bool ph, double rho)
{
    const int64_t n = st.n;
    const int npx = c.W * c.H;
    int queries = 0;
    for (int d = 0; d < c.n; ++d) {
        const int64_t e = ((int64_t)b * c.n + d) * n + i;
        int pix = project(c, d, x[0], x[1], x[2], 1.0);
        double2 tc = make_double2(0.0, 0.0);
        if (pix >= 0) {
            double wc[3], dist, idist;
            unit_to(x, c.pos[d], wc, dist, idist);
            const double cn = dot3(n_, wc);
            queries += cn > 0.0;
            if (cn > 0.0 && !occluded(s, sph, sid, x, wc, dist)) {
                const double geo = cn * (idist * idist) * st.omega[d * npx + pix];
                tc = ph ? make_double2(geo, dot3(r, wc)) : make_double2(geo * rho / kPiD, 0.0);
            } else {
                pix = -1;
            }
        }
        st.tc[e] = tc;
        st.pix[e] = pix;
    }
    return queries;
}

// Drawn-direction record of a vertex: {cos to the mirror direction, cos to
// the normal} of the direction to the next vertex at the unknown sphere,
// {rho, -1} at a diffuse surface; the unknown sphere's last vertex (no next
// vertex) gets {0, 0}: its flag still selects its BRDF for the local
// estimates.
__device__ __forceinline__ double2 direction_record(bool ph, double rho, bool has_next, const double x[3],
                                                    const double y[3], const double n_[3], const double r[3])
{
    if (!ph) return make_double2(rho, -1.0);
    if (!has_next) return make_double2(0.0, 0.0);
    double w_out[3], len;
    unit_to(x, y, w_out, len);
    return make_double2(dot3(r, w_out), dot3(n_, w_out));
}

}  // namespace

// The theta-independent tape of every stored vertex (see the file comment),
// from the stored positions (imported stores).
__global__ void __launch_bounds__(kSurfBlock) surf_tape_kernel(SurfScene s, DevCams c, SurfStore st)
{
    __shared__ double lsph[kSphStride * kMaxSpheres];
    const double* sph = load_spheres(s, lsph);
    const int64_t n = st.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int Bn = st.B[i];
        double prev[3] = {s.light[0], s.light[1], s.light[2]};
        double4 q = Bn > 0 ? st.pos[i] : make_double4(0.0, 0.0, 0.0, 0.0);
        for (int b = 0; b < Bn; ++b) {
            const double x[3] = {q.x, q.y, q.z};
            const int sid = st.sid[(int64_t)b * n + i];
            const bool ph = is_phong(s, sid);
            double n_[3], w_in[3], len;
            surface_normal(sph, sid, x, n_);
            unit_to(prev, x, w_in, len);
            double r[3];
            mirror_dir(w_in, n_, r);
            const double rho = ph ? 0.0 : albedo_of(s, sph, sid);
            const bool has_next = b + 1 < Bn;
            if (has_next) q = st.pos[(int64_t)(b + 1) * n + i];
            const double y[3] = {q.x, q.y, q.z};
            st.tv[(int64_t)b * n + i] = direction_record(ph, rho, has_next, x, y, n_, r);
            camera_records(s, sph, c, st, b, i, x, sid, n_, r, ph, rho);
            prev[0] = x[0];
            prev[1] = x[1];
            prev[2] = x[2];
        }
    }
}

// Forward path tracing from the light at theta_ref (Sec. 3.4 with surfaces)
// and the tape in one pass, one lane per path, FP64: a uniform direction from
// the light, then at each vertex a cosine-weighted draw (diffuse) or the
// mixture of a cosine-weighted and a Phong-lobe draw (unknown sphere; a lobe
// draw below the surface ends the path).  Each vertex's camera records are
// formed when it is found and its drawn-direction record when the next
// vertex is found, from the positions as surf_tape_kernel forms them, so that
// a store and an import of its exported paths hold the same tape.
__global__ void __launch_bounds__(kSurfBlock) surf_draw_kernel(SurfScene s, DevCams c, SurfStore st, uint64_t seed,
                                                                uint64_t first_id, DrawTheta th)
{
    __shared__ double lsph[kSphStride * kMaxSpheres];
    const double* sph = load_spheres(s, lsph);
    // theta_ref: given, or read from the device and clamped to the drawable
    // range; the first thread keeps it in the store for the later kernels
    double kr = th.kappa, gr = th.gamma;
    if (th.src) {
        kr = fmin(fmax(th.src[0], 0.0), kKappaRefMax);
        gr = fmin(fmax(th.src[1], 0.0), kGammaRefMax);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st.theta_ref[0] = kr;
        st.theta_ref[1] = gr;
    }
    const double ge = 1.0 / (gr + 1.0);
    const int M = s.max_order;
    const int64_t n = st.n;
    unsigned long long queries = 0, verts = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t id = first_id + (uint64_t)i;
        double u[4];
        uniforms4(seed, id, 0u, u);
        const double mu0 = 1.0 - 2.0 * u[0], st0 = sqrt(fmax(0.0, 1.0 - mu0 * mu0));
        double sp, cp;
        sincos(2.0 * kPiD * u[1], &sp, &cp);
        double w[3] = {st0 * cp, st0 * sp, mu0};
        double p[3] = {s.light[0], s.light[1], s.light[2]};
        // the previous vertex, whose drawn-direction record waits for this one
        double xp[3] = {0.0, 0.0, 0.0}, np_[3] = {0.0, 0.0, 0.0}, rp[3] = {0.0, 0.0, 0.0};
        bool php = false;
        double rhop = 0.0;
        int skip = -1, b = 0;
        while (b < M) {
            double t;
            const int hid = nearest_surface(s, sph, p, w, skip, t);
            ++queries;
            if (hid < 0 || !isfinite(t)) break;
            double x[3] = {p[0] + t * w[0], p[1] + t * w[1], p[2] + t * w[2]};
            if (hid < 6) x[hid >> 1] = (hid & 1) ? s.box : 0.0;
            st.pos[(int64_t)b * n + i] = make_double4(x[0], x[1], x[2], 0.0);
            st.sid[(int64_t)b * n + i] = hid;
            if (b > 0) st.tv[(int64_t)(b - 1) * n + i] = direction_record(php, rhop, true, xp, x, np_, rp);
            // tape of this vertex: normal, arriving direction from the
            // positions, mirror direction, camera records
            const bool ph = is_phong(s, hid);
            const double rho = ph ? 0.0 : albedo_of(s, sph, hid);
            double n_[3], w_in[3], len, r[3];
            surface_normal(sph, hid, x, n_);
            unit_to(p, x, w_in, len);
            mirror_dir(w_in, n_, r);
            queries += camera_records(s, sph, c, st, b, i, x, hid, n_, r, ph, rho);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                xp[a] = x[a];
                np_[a] = n_[a];
                rp[a] = r[a];
            }
            php = ph;
            rhop = rho;
            ++b;
            if (b == M) break;
            uniforms4(seed, id, (uint32_t)b, u);
            double wn[3];
            if (ph && u[0] < kr) {
                double rr[3];
                mirror_dir(w, n_, rr);
                scatter_direction(rr, pow(u[1], ge), 2.0 * kPiD * u[2], wn);
                if (!(dot3(n_, wn) > 0.0)) break;
            } else {
                scatter_direction(n_, sqrt(u[1]), 2.0 * kPiD * u[2], wn);
            }
            p[0] = x[0];
            p[1] = x[1];
            p[2] = x[2];
            w[0] = wn[0];
            w[1] = wn[1];
            w[2] = wn[2];
            skip = hid;
        }
        if (b > 0) st.tv[(int64_t)(b - 1) * n + i] = direction_record(php, rhop, false, xp, xp, np_, rp);
        st.B[i] = b;
        verts += (unsigned long long)b;
    }
    // work of the draw: one nearest-surface query per traced ray and one
    // occlusion query per in-image camera connection, n_spheres tests each
    for (int o = kWave / 2; o > 0; o >>= 1) {
        queries += __shfl_xor(queries, o);
        verts += __shfl_xor(verts, o);
    }
    if (threadIdx.x % kWave == 0 && st.work) {
        atomicAdd(&st.work[0], queries * (unsigned long long)s.n_spheres);
        atomicAdd(&st.work[1], verts);
    }
}

// Recycled images F(theta_t | theta_ref) (Eq. forward_simualtion_recycling):
// one lane per path walks its tape; the local estimate of vertex b is
// w_b f(c_cam) geo (diffuse: w_b geo'), and the weight carries on by
// f(c) nc / pdf_ref (diffuse: rho).  kLds: the workgroup tallies all images
// in LDS (FP64) and writes them to its partial slot; else FP64 atomics on
// the output.
template <bool kLds>
__global__ void __launch_bounds__(kSurfBlock) surf_render_kernel(SurfStore st, int n_cams, int npx, double w0,
                                                                  const double* theta, double* out)
{
    extern __shared__ double simg[];
    const int ni = n_cams * npx;
    if (kLds) {
        for (int k = threadIdx.x; k < ni; k += blockDim.x) simg[k] = 0.0;
        __syncthreads();
    }
    PhongTerms P;
    P.init(theta, st.theta_ref);
    const int64_t n = st.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int Bn = st.B[i];
        double w = w0;
        for (int b = 0; b < Bn; ++b) {
            const double2 tv = st.tv[(int64_t)b * n + i];
            const bool ph = tv.y >= 0.0;
            for (int d = 0; d < n_cams; ++d) {
                const int64_t e = ((int64_t)b * n_cams + d) * n + i;
                const int pix = st.pix[e];
                if (pix < 0) continue;
                const double2 tc = st.tc[e];
                const double v = w * (ph ? P.f(tc.y) * tc.x : tc.x);
                if (kLds)
                    atomicAdd(&simg[d * npx + pix], v);
                else
                    atomicAdd(&out[(int64_t)d * npx + pix], v);
            }
            if (b + 1 < Bn) w *= ph ? P.carry(tv.x, tv.y) : tv.x;
        }
    }
    if (kLds) {
        __syncthreads();
        double* dst = out + (int64_t)blockIdx.x * ni;
        for (int k = threadIdx.x; k < ni; k += blockDim.x) dst[k] = simg[k];
    }
}

// out[k] = sum over the partial images in workgroup order.
// out[k] = sum over the partial images of pixel k in a fixed order: a block
// holds 16 pixels x 16 partial segments; each thread sums its segment's
// partials (8 loads in flight, added in order), then the 16 segment sums of a
// pixel are added in segment order.
constexpr int kRedPix = 16, kRedSeg = 16;

__global__ void __launch_bounds__(kRedPix * kRedSeg) surf_image_reduce_kernel(const double* __restrict__ part,
                                                                              int n_part, int ni,
                                                                              double* __restrict__ out)
{
    __shared__ double seg[kRedSeg][kRedPix];
    const int px = threadIdx.x % kRedPix, sg = threadIdx.x / kRedPix;
    const int k = blockIdx.x * kRedPix + px;
    const int per = (n_part + kRedSeg - 1) / kRedSeg;
    const int j0 = sg * per, j1 = min(n_part, j0 + per);
    double acc = 0.0;
    if (k < ni) {
        int j = j0;
        for (; j + 8 <= j1; j += 8) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = part[(int64_t)(j + q) * ni + k];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc += v[q];
        }
        for (; j < j1; ++j) acc += part[(int64_t)j * ni + k];
    }
    seg[sg][px] = acc;
    __syncthreads();
    if (sg == 0 && k < ni) {
        double t = 0.0;
        for (int q = 0; q < kRedSeg; ++q) t += seg[q][px];
        out[k] = t;
    }
}

// Loss gradient in (kappa_s, gamma) (Eq. loss_gradient with Eq.
// gradient_simualtion_recycling): every local estimate adds residual[pixel]
// x contribution x PSF, the PSF being the sum of d log f over the unknown
// sphere's bounces before the vertex and its connection (Eq.
// total_derivative_factor).  Per-workgroup pairs go to part[2 * block].
__global__ void __launch_bounds__(kSurfBlock) surf_grad_kernel(SurfStore st, int n_cams, int npx, double w0,
                                                                const double* theta, const double* __restrict__ res,
                                                                double* part)
{
    __shared__ double red[kSurfBlock / kWave];
    PhongTerms P;
    P.init(theta, st.theta_ref);
    const double dka = -1.0 / kPiD, dkb = (P.gamma + 2.0) / (2.0 * kPiD), dgb = P.kappa / (2.0 * kPiD);
    double g0 = 0.0, g1 = 0.0;
    const int64_t n = st.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int Bn = st.B[i];
        double w = w0, s0 = 0.0, s1 = 0.0;
        for (int b = 0; b < Bn; ++b) {
            const double2 tv = st.tv[(int64_t)b * n + i];
            const bool ph = tv.y >= 0.0;
            for (int d = 0; d < n_cams; ++d) {
                const int64_t e = ((int64_t)b * n_cams + d) * n + i;
                const int pix = st.pix[e];
                if (pix < 0) continue;
                const double2 tc = st.tc[e];
                const double r = res[(int64_t)d * npx + pix];
                if (ph) {
                    // f, d f / d kappa, d f / d gamma at the camera cosine
                    double lc;
                    const double l = P.lobe_log(tc.y, lc);
                    const double f = P.fa + P.fb * l;
                    const double v = r * w * tc.x;
                    g0 += v * (f * s0 + dka + dkb * l);
                    g1 += v * (f * s1 + dgb * l * (1.0 + (P.gamma + 2.0) * lc));
                } else {
                    const double v = r * w * tc.x;
                    g0 += v * s0;
                    g1 += v * s1;
                }
            }
            if (b + 1 < Bn) {
                if (ph) {
                    const double c = tv.x, nc = tv.y;
                    const double lc = c > 0.0 ? log(c) : 0.0;
                    const double l = c > 0.0 ? exp(P.gamma * lc) : 0.0, lr = c > 0.0 ? exp(P.rgamma * lc) : 0.0;
                    const double f = P.fa + P.fb * l;
                    const double fi = 1.0 / f;
                    s0 += (dka + dkb * l) * fi;
                    s1 += dgb * l * (1.0 + (P.gamma + 2.0) * lc) * fi;
                    w *= f * nc / (P.ra * fmax(nc, 0.0) + P.rb * lr);
                } else {
                    w *= tv.x;
                }
            }
        }
    }
    const double t0 = block_sum(g0, red);
    const double t1 = block_sum(g1, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = t0;
        part[2 * blockIdx.x + 1] = t1;
    }
}

// Correction factor of each path (Eq. correction factor): the product over
// its draws at the unknown sphere of pdf(theta_t) / pdf(theta_ref), formed as
// a sum of logs; per-workgroup (sum r, sum r^2) to part[2 * block].
__global__ void __launch_bounds__(kSurfBlock) surf_reweight_kernel(SurfStore st, const double* theta, double* part)
{
    __shared__ double red[kSurfBlock / kWave];
    PhongTerms P;
    P.init(theta, st.theta_ref);
    const double ta = (1.0 - P.kappa) / kPiD, tb = P.kappa * (P.gamma + 1.0) / (2.0 * kPiD);
    double s1 = 0.0, s2 = 0.0;
    const int64_t n = st.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int Bn = st.B[i];
        double lr = 0.0;
        for (int b = 0; b + 1 < Bn; ++b) {
            const double2 tv = st.tv[(int64_t)b * n + i];
            if (tv.y < 0.0) continue;
            const double c = tv.x, nc = fmax(tv.y, 0.0);
            const double lc = c > 0.0 ? log(c) : 0.0;
            const double l = c > 0.0 ? exp(P.gamma * lc) : 0.0, lrf = c > 0.0 ? exp(P.rgamma * lc) : 0.0;
            lr += log((ta * nc + tb * l) / (P.ra * nc + P.rb * lrf));
        }
        const double r = exp(lr);
        s1 += r;
        s2 += r * r;
    }
    const double t1 = block_sum(s1, red);
    const double t2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = t1;
        part[2 * blockIdx.x + 1] = t2;
    }
}

// out[0..1] = sums of the pairs part[2j], part[2j+1] over j < n in order
// (gradient); with stats set, out = {sum/n_paths, sum^2 / sum of squares}.
// out[0..1] = sums of the pairs part[2j], part[2j+1] over j < n in a fixed
// order (each of 256 threads sums a contiguous range, then the 256 range sums
// are added in thread order); with stats set, out = {sum/n_paths, sum^2 / sum
// of squares}.
__global__ void __launch_bounds__(256) surf_pairs_kernel(const double* __restrict__ part, int n, double n_paths,
                                                         int stats, double* out)
{
    __shared__ double sa[256], sb[256];
    const int per = (n + 255) / 256;
    const int j0 = threadIdx.x * per, j1 = min(n, j0 + per);
    double a = 0.0, b = 0.0;
    for (int j = j0; j < j1; ++j) {
        a += part[2 * j];
        b += part[2 * j + 1];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x != 0) return;
    a = b = 0.0;
    for (int t = 0; t < 256; ++t) {
        a += sa[t];
        b += sb[t];
    }
    if (stats) {
        out[0] = a / n_paths;
        out[1] = b > 0.0 ? a * a / b : 0.0;
    } else {
        out[0] = a;
        out[1] = b;
    }
}

// One Adam step (Kingma & Ba) per parameter with its own step size, then the
// box 0 <= kappa_s <= 1, gamma >= 0.
__global__ void surf_adam_kernel(double* theta, const double* g, double* m, double* v, double lr0, double lr1,
                                 double b1, double b2, double eps, double bc1, double bc2)
{
    const int k = threadIdx.x;
    if (k >= 2) return;
    const double gk = g[k];
    const double mk = b1 * m[k] + (1.0 - b1) * gk;
    const double vk = b2 * v[k] + (1.0 - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    double t = theta[k] - (k == 0 ? lr0 : lr1) * (mk / bc1) / (sqrt(vk / bc2) + eps);
    t = fmax(t, 0.0);
    if (k == 0) t = fmin(t, 1.0);
    theta[k] = t;
}

// ------------------------------------------------------------- launchers

static unsigned surf_blocks(int64_t n, int n_cu, int per_cu)
{
    const int64_t need = (n + kSurfBlock - 1) / kSurfBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)n_cu * per_cu));
}

hipError_t launch_surf_omega(hipStream_t stream, const DevCams& c, double* omega)
{
    const int k = c.n * c.W * c.H;
    surf_omega_kernel<<<(k + 255) / 256, 256, 0, stream>>>(c, omega);
    return hipGetLastError();
}

hipError_t launch_surf_draw(hipStream_t stream, const SurfScene& s, const DevCams& c, const SurfStore& st,
                            uint64_t seed, uint64_t first_id, const DrawTheta& th, int n_cu)
{
    if (st.n == 0) return hipSuccess;
    surf_draw_kernel<<<surf_blocks(st.n, n_cu, 8), kSurfBlock, 0, stream>>>(s, c, st, seed, first_id, th);
    return hipGetLastError();
}

hipError_t launch_surf_tape(hipStream_t stream, const SurfScene& s, const DevCams& c, const SurfStore& st, int n_cu)
{
    if (st.n == 0) return hipSuccess;
    surf_tape_kernel<<<surf_blocks(st.n, n_cu, 8), kSurfBlock, 0, stream>>>(s, c, st);
    return hipGetLastError();
}

int surf_render_parts(int64_t n, int n_cams, int npx, int n_cu)
{
    if ((int64_t)n_cams * npx * (int64_t)sizeof(double) > kSurfImageLds) return 0;
    return (int)surf_blocks(n, n_cu, 4);
}

hipError_t launch_surf_render(hipStream_t stream, const SurfStore& st, int n_cams, int npx, double w0,
                              const double* theta, double* img, double* part, int n_cu)
{
    const int ni = n_cams * npx;
    const int np = surf_render_parts(st.n, n_cams, npx, n_cu);
    if (np > 0) {
        surf_render_kernel<true><<<np, kSurfBlock, (size_t)ni * sizeof(double), stream>>>(st, n_cams, npx, w0, theta,
                                                                                          part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        surf_image_reduce_kernel<<<(ni + kRedPix - 1) / kRedPix, kRedPix * kRedSeg, 0, stream>>>(part, np, ni, img);
        return hipGetLastError();
    }
    hipError_t e = launch_fill(stream, img, ni, 0.0);
    if (e != hipSuccess) return e;
    if (st.n == 0) return hipSuccess;
    surf_render_kernel<false><<<surf_blocks(st.n, n_cu, 8), kSurfBlock, 0, stream>>>(st, n_cams, npx, w0, theta, img);
    return hipGetLastError();
}

int surf_pair_blocks(int64_t n, int n_cu) { return (int)surf_blocks(n, n_cu, 8); }

hipError_t launch_surf_grad(hipStream_t stream, const SurfStore& st, int n_cams, int npx, double w0,
                            const double* theta, const double* res, double* part, double* grad, int n_cu)
{
    const int nb = surf_pair_blocks(st.n, n_cu);
    surf_grad_kernel<<<nb, kSurfBlock, 0, stream>>>(st, n_cams, npx, w0, theta, res, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    surf_pairs_kernel<<<1, 256, 0, stream>>>(part, nb, 0.0, 0, grad);
    return hipGetLastError();
}

hipError_t launch_surf_reweight(hipStream_t stream, const SurfStore& st, const double* theta, double* part,
                                double* stats, int n_cu)
{
    const int nb = surf_pair_blocks(st.n, n_cu);
    surf_reweight_kernel<<<nb, kSurfBlock, 0, stream>>>(st, theta, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    surf_pairs_kernel<<<1, 256, 0, stream>>>(part, nb, (double)st.n, 1, stats);
    return hipGetLastError();
}

hipError_t launch_surf_adam(hipStream_t stream, double* theta, const double* g, double* m, double* v, double lr0,
                            double lr1, double b1, double b2, double eps, double bc1, double bc2)
{
    surf_adam_kernel<<<1, 64, 0, stream>>>(theta, g, m, v, lr0, lr1, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace prt
