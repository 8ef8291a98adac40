/*
 * surface_oracle.c -- plain FP64 CPU oracle for the reflectometry workload of
 * Czerninski & Schechner, "Accelerating Inverse Rendering By Using a GPU and
 * Reuse of Light Paths" (arXiv 2110.00085), Sec. 6.2.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * only tests/, the smoke check and the CPU-baseline leg of bench.py use it.  It
 * shares no source with the HIP library; it is linked into the same oracle
 * library as prt_oracle.c and uses that file's Philox stream, direction basis,
 * pinhole projection and pixel solid angles (all oracle code).
 *
 * The scene: a closed box [0,L]^3 with diffuse walls, diffuse spheres and one
 * sphere whose BRDF is the unknown (kappa_s, gamma) of Eq. phong, lit by an
 * isotropic point light inside the box (Sec. 3.4, forward path tracing from
 * the light).  Definitions followed, evaluated the slow, obvious way:
 *   - SRE and the geometric term:  Eq. surface_rendering, Eq. geomterm
 *   - MCF and its SCFs:            Eqs. gk, g0K, cont_func; BRDF f of Eq. fs
 *   - local estimation:            Sec. 3.4.3 (a connection to each camera at
 *                                  every surface vertex)
 *   - recycling:                   Eqs. forward_simualtion_recycling,
 *                                  correction factor, gradient_simualtion_recycling
 *   - loss gradient:               Eq. loss_gradient with the PSF of
 *                                  Eq. total_derivative_factor, where only the
 *                                  BRDF of the unknown sphere depends on theta.
 *
 * Readings of the paper (it leaves these open):
 *   - Eq. phong as written has no 1/pi and its lobe points along the incoming
 *     direction; this oracle takes the energy-conserving modified Phong model
 *     (Lafortune & Willems 1994): f = (1-kappa)/pi + kappa (gamma+2)/(2 pi)
 *     max(0, w_r . w_out)^gamma, w_r the mirror image of the propagation
 *     direction about the normal; "no absorption" = diffuse and specular
 *     weights summing to one.
 *   - Directions at the unknown sphere are drawn from the mixture
 *     (1-kappa_ref) cos/pi + kappa_ref (gamma_ref+1)/(2 pi) cos_r^gamma_ref
 *     (lobe chosen by u0 < kappa_ref); a lobe sample below the surface ends
 *     the path.  Diffuse surfaces draw cosine-weighted directions, so their
 *     continuation weight is their albedo.
 *   - Paths end after max_order surface vertices.
 *
 * Units: scene units for lengths (cameras share them); the light has radiant
 * intensity I0 per steradian, so the first vertex carries 4 pi I0 (the uniform
 * direction pdf 1/(4 pi); the geometric terms cancel as after Eq.
 * explicit_foward).  A pixel averages radiance over its solid angle, as in the
 * tomography oracle.
 *
 * Surface ids: 0..5 the walls x=0, x=L, y=0, y=L, z=0, z=L; 6+k sphere k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PSO_PI 3.14159265358979323846

typedef struct {
    double box;                 /* edge L of the box [0,L]^3 */
    double wall_albedo[6];      /* x=0, x=L, y=0, y=L, z=0, z=L */
    double light[3];            /* point light position (inside the box, outside every sphere) */
    double intensity;           /* radiant intensity I0 of the light */
    int32_t n_spheres, phong, max_order, pad;
    const double* center;       /* [n_spheres][3] */
    const double* radius;       /* [n_spheres] */
    const double* albedo;       /* [n_spheres] diffuse albedo (unused for the Phong sphere) */
} pso_scene;

/* same layout as the tomography oracle's camera set */
typedef struct {
    int32_t n, width, height, pad;
    const double* pos;
    const double* rot;
    const double* f_px;
} pso_cams;

/* from prt_oracle.c (same library) */
void prto_uniforms(uint64_t seed, uint64_t path, uint64_t event, double u[4]);
void prto_new_direction(const double n[3], double mu, double phi, double out[3]);
void prto_pixel_solid_angles(double f, int W, int H, double* out);
int prto_project(const pso_cams* c, int d, const double x[3]);

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void unit3(const double a[3], const double b[3], double w[3], double* len)
{
    double d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double l = sqrt(dot3(d, d));
    for (int i = 0; i < 3; ++i) w[i] = d[i] / l;
    if (len) *len = l;
}

/* Does surface sid carry the unknown BRDF?  (phong < 0: no sphere does) */
static int is_phong(const pso_scene* s, int sid) { return s->phong >= 0 && sid == 6 + s->phong; }

/* Outward normal of a sphere, inward normal of a wall. */
void psso_normal(const pso_scene* s, int sid, const double x[3], double n[3])
{
    n[0] = n[1] = n[2] = 0.0;
    if (sid < 6) {
        n[sid / 2] = (sid % 2 == 0) ? 1.0 : -1.0;
        return;
    }
    int k = sid - 6;
    for (int i = 0; i < 3; ++i) n[i] = (x[i] - s->center[3 * k + i]) / s->radius[k];
}

/* Smallest t > 0 where p + t w meets sphere k (entry from outside), or +inf. */
double psso_sphere_hit(const double c[3], double r, const double p[3], const double w[3])
{
    double oc[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]};
    double b = dot3(oc, w);
    double cc = dot3(oc, oc) - r * r;
    double disc = b * b - cc;
    if (disc < 0.0) return INFINITY;
    double t = -b - sqrt(disc);
    return t > 0.0 ? t : INFINITY;
}

/* Nearest surface along p + t w (t > 0), skipping surface `skip`: returns its
   id and sets *t; -1 when nothing is hit. */
int psso_nearest(const pso_scene* s, const double p[3], const double w[3], int skip, double* t_out)
{
    double best = INFINITY;
    int id = -1;
    for (int a = 0; a < 3; ++a) {
        if (w[a] == 0.0) continue;
        int wall = w[a] > 0.0 ? 2 * a + 1 : 2 * a;
        if (wall == skip) continue;
        double t = ((w[a] > 0.0 ? s->box : 0.0) - p[a]) / w[a];
        if (t > 0.0 && t < best) { best = t; id = wall; }
    }
    for (int k = 0; k < s->n_spheres; ++k) {
        if (6 + k == skip) continue;
        double t = psso_sphere_hit(s->center + 3 * k, s->radius[k], p, w);
        if (t < best) { best = t; id = 6 + k; }
    }
    *t_out = best;
    return id;
}

/* Mirror image of the propagation direction w about n. */
static void mirror(const double w[3], const double n[3], double r[3])
{
    double c = 2.0 * dot3(w, n);
    for (int i = 0; i < 3; ++i) r[i] = w[i] - c * n[i];
}

/* Modified Phong BRDF (Eq. phong, reading above) from the cosine c between
   the outgoing direction and the mirror direction. */
double psso_phong(double kappa, double gamma, double c)
{
    double lobe = c > 0.0 ? pow(c, gamma) : 0.0;
    return (1.0 - kappa) / PSO_PI + kappa * (gamma + 2.0) / (2.0 * PSO_PI) * lobe;
}

/* d f / d kappa and d f / d gamma at cosine c. */
void psso_phong_deriv(double kappa, double gamma, double c, double d[2])
{
    double lobe = c > 0.0 ? pow(c, gamma) : 0.0;
    d[0] = -1.0 / PSO_PI + (gamma + 2.0) / (2.0 * PSO_PI) * lobe;
    d[1] = c > 0.0 ? kappa / (2.0 * PSO_PI) * lobe * (1.0 + (gamma + 2.0) * log(c)) : 0.0;
}

/* Density per steradian of the direction draw at the Phong sphere:
   ncos = n . w_out, c = w_r . w_out. */
double psso_phong_pdf(double kappa, double gamma, double ncos, double c)
{
    double dif = ncos > 0.0 ? ncos / PSO_PI : 0.0;
    double lobe = c > 0.0 ? (gamma + 1.0) / (2.0 * PSO_PI) * pow(c, gamma) : 0.0;
    return (1.0 - kappa) * dif + kappa * lobe;
}

/* BRDF of surface sid at theta for light arriving along w_in, leaving along
   w_out (Eq. fs, surface case). */
static double brdf(const pso_scene* s, int sid, const double theta[2], const double n[3], const double w_in[3],
                   const double w_out[3])
{
    if (is_phong(s, sid)) {
        double r[3];
        mirror(w_in, n, r);
        return psso_phong(theta[0], theta[1], dot3(r, w_out));
    }
    double rho = sid < 6 ? s->wall_albedo[sid] : s->albedo[sid - 6];
    return rho / PSO_PI;
}

/* One bounce at surface sid (at x, light arriving along w_in) from uniforms
   u[0..2]: the new direction and the continuation weight f |n . w_out| / pdf
   at theta (the same theta draws and weighs).  Returns 0 when the draw ends
   the path (a lobe sample below the surface). */
int psso_bounce(const pso_scene* s, int sid, const double theta[2], const double x[3], const double w_in[3],
                const double u[3], double w_out[3], double* weight)
{
    double n[3];
    psso_normal(s, sid, x, n);
    double phi = 2.0 * PSO_PI * u[2];
    int ph = is_phong(s, sid);
    if (ph && u[0] < theta[0]) {
        double r[3];
        mirror(w_in, n, r);
        prto_new_direction(r, pow(u[1], 1.0 / (theta[1] + 1.0)), phi, w_out);
        if (!(dot3(n, w_out) > 0.0)) return 0;
    } else {
        prto_new_direction(n, sqrt(u[1]), phi, w_out);
    }
    double nc = dot3(n, w_out);
    double pdf;
    if (ph) {
        double r[3];
        mirror(w_in, n, r);
        pdf = psso_phong_pdf(theta[0], theta[1], nc, dot3(r, w_out));
    } else {
        pdf = nc / PSO_PI;
    }
    *weight = brdf(s, sid, theta, n, w_in, w_out) * nc / pdf;
    return 1;
}

/* Forward path tracing from the light (Sec. 3.4 with surfaces): paths
   first_id .. first_id+n-1 at theta_ref.  Vertices x_1..x_B go to
   pos[(i*M + b)*3], their surface ids to sid[i*M + b], B to B[i]. */
void psso_sample(const pso_scene* s, const double theta_ref[2], uint64_t seed, uint64_t first_id, int64_t n,
                 int32_t* B, double* pos, int32_t* sid)
{
    const int M = s->max_order;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t id = first_id + (uint64_t)i;
        double u[4];
        prto_uniforms(seed, id, 0, u);
        double mu = 1.0 - 2.0 * u[0], st = sqrt(fmax(0.0, 1.0 - mu * mu)), ph = 2.0 * PSO_PI * u[1];
        double w[3] = {st * cos(ph), st * sin(ph), mu};
        double p[3] = {s->light[0], s->light[1], s->light[2]};
        int skip = -1, b = 0;
        while (b < M) {
            double t;
            int id_hit = psso_nearest(s, p, w, skip, &t);
            if (id_hit < 0 || !isfinite(t)) break;
            double x[3] = {p[0] + t * w[0], p[1] + t * w[1], p[2] + t * w[2]};
            if (id_hit < 6) x[id_hit / 2] = (id_hit % 2 == 0) ? 0.0 : s->box;
            for (int a = 0; a < 3; ++a) pos[(i * M + b) * 3 + a] = x[a];
            sid[i * M + b] = id_hit;
            ++b;
            if (b == M) break;
            prto_uniforms(seed, id, (uint64_t)b, u);
            double wn[3], wt;
            if (!psso_bounce(s, id_hit, theta_ref, x, w, u, wn, &wt)) break;
            for (int a = 0; a < 3; ++a) { p[a] = x[a]; w[a] = wn[a]; }
            skip = id_hit;
        }
        B[i] = b;
    }
}

/* Is camera position c seen from surface point x (id sid, normal n)?  The
   camera must lie on the outer side and no other sphere may cut the segment
   (the walls of a box that holds the camera cannot). */
static int visible(const pso_scene* s, int sid, const double x[3], const double n[3], const double c[3],
                   double wc[3], double* dist)
{
    unit3(x, c, wc, dist);
    if (!(dot3(n, wc) > 0.0)) return 0;
    for (int k = 0; k < s->n_spheres; ++k) {
        if (6 + k == sid) continue;
        if (psso_sphere_hit(s->center + 3 * k, s->radius[k], x, wc) < *dist) return 0;
    }
    return 1;
}

typedef struct {
    const pso_scene* s;
    const pso_cams* cm;
    const double* omega;    /* [n][H*W] pixel solid angles */
} pso_ctx;

/* Walk one path at theta_t over paths drawn at theta_ref.  For every local
   estimate (vertex b, camera d) calls back with the pixel, the recycled
   contribution C(theta_t)/p(theta_ref) (Eq. forward_simualtion_recycling) and
   the PSF of its sub-path (Eq. total_derivative_factor: the d log f terms of
   the unknown sphere's BRDF at every bounce before b and at the connection). */
typedef void (*pso_visit)(void* user, int d, int pix, double c, const double psf[2]);

static void walk_path(const pso_ctx* X, const double theta_t[2], const double theta_ref[2], int Bn,
                      const double* P, const int32_t* S, pso_visit visit, void* user)
{
    const pso_scene* s = X->s;
    const pso_cams* cm = X->cm;
    const int npx = cm->width * cm->height;
    double w = 4.0 * PSO_PI * s->intensity;
    double psf[2] = {0.0, 0.0};
    double w_in[3];
    unit3(s->light, P, w_in, NULL);
    for (int b = 0; b < Bn; ++b) {
        const double* x = P + 3 * b;
        const int sid = S[b];
        const int ph = is_phong(s, sid);
        double n[3];
        psso_normal(s, sid, x, n);
        for (int d = 0; d < cm->n; ++d) {
            int pix = prto_project(cm, d, x);
            if (pix < 0) continue;
            double wc[3], dist;
            if (!visible(s, sid, x, n, cm->pos + 3 * d, wc, &dist)) continue;
            double f = brdf(s, sid, theta_t, n, w_in, wc);
            double c = w * f * dot3(n, wc) / (dist * dist) / X->omega[(size_t)d * npx + pix];
            double q[2] = {psf[0], psf[1]};
            if (ph) {
                double r[3], dv[2];
                mirror(w_in, n, r);
                psso_phong_deriv(theta_t[0], theta_t[1], dot3(r, wc), dv);
                q[0] += dv[0] / f;
                q[1] += dv[1] / f;
            }
            visit(user, d, pix, c, q);
        }
        if (b + 1 == Bn) break;
        double w_out[3];
        unit3(x, P + 3 * (b + 1), w_out, NULL);
        double nc = dot3(n, w_out);
        double f = brdf(s, sid, theta_t, n, w_in, w_out);
        double pdf;
        if (ph) {
            double r[3], dv[2];
            mirror(w_in, n, r);
            double cr = dot3(r, w_out);
            pdf = psso_phong_pdf(theta_ref[0], theta_ref[1], nc, cr);
            psso_phong_deriv(theta_t[0], theta_t[1], cr, dv);
            psf[0] += dv[0] / f;
            psf[1] += dv[1] / f;
        } else {
            pdf = nc / PSO_PI;
        }
        w *= f * nc / pdf;
        for (int a = 0; a < 3; ++a) w_in[a] = w_out[a];
    }
}

static double* solid_angles(const pso_cams* cm)
{
    size_t npx = (size_t)cm->width * cm->height;
    double* om = (double*)malloc(sizeof(double) * npx * (size_t)cm->n);
    for (int d = 0; d < cm->n; ++d) prto_pixel_solid_angles(cm->f_px[d], cm->width, cm->height, om + npx * d);
    return om;
}

typedef struct {
    double* img;
    const double* res;
    double g[2];
    int npx;
    double scale;
} pso_acc;

static void visit_render(void* user, int d, int pix, double c, const double psf[2])
{
    (void)psf;
    pso_acc* A = (pso_acc*)user;
    A->img[(size_t)d * A->npx + pix] += c * A->scale;
}

static void visit_grad(void* user, int d, int pix, double c, const double psf[2])
{
    pso_acc* A = (pso_acc*)user;
    double e = A->res[(size_t)d * A->npx + pix] * c * A->scale;
    A->g[0] += e * psf[0];
    A->g[1] += e * psf[1];
}

/* Recycled images F(theta_t | theta_ref): img[d][p] = (1/n_total) sum over
   paths and local estimates landing on p.  Per-thread images are summed in
   thread order. */
void psso_render(const pso_scene* s, const pso_cams* cm, const double theta_t[2], const double theta_ref[2],
                 int64_t n_total, int64_t n, const int32_t* B, const double* pos, const int32_t* sid, double* img)
{
    pso_ctx X = {s, cm, solid_angles(cm)};
    const int npx = cm->width * cm->height;
    const size_t ni = (size_t)npx * cm->n;
    const int M = s->max_order;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double* part = (double*)calloc(ni * (size_t)nt, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        pso_acc A = {part + ni * (size_t)tid, NULL, {0.0, 0.0}, npx, 1.0 / (double)n_total};
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            walk_path(&X, theta_t, theta_ref, B[i], pos + (size_t)i * M * 3, sid + (size_t)i * M, visit_render, &A);
    }
    for (size_t p = 0; p < ni; ++p) {
        double acc = 0.0;
        for (int t = 0; t < nt; ++t) acc += part[ni * (size_t)t + p];
        img[p] = acc;
    }
    free(part);
    free((void*)X.omega);
}

/* d loss / d (kappa, gamma) (Eq. loss_gradient with Eq.
   gradient_simualtion_recycling): (1/n_total) sum over local estimates of
   residual[pixel] * contribution * PSF. */
void psso_grad(const pso_scene* s, const pso_cams* cm, const double theta_t[2], const double theta_ref[2],
               int64_t n_total, int64_t n, const int32_t* B, const double* pos, const int32_t* sid,
               const double* residual, double grad[2])
{
    pso_ctx X = {s, cm, solid_angles(cm)};
    const int npx = cm->width * cm->height;
    const int M = s->max_order;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double* part = (double*)calloc(2 * (size_t)nt, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        pso_acc A = {NULL, residual, {0.0, 0.0}, npx, 1.0 / (double)n_total};
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            walk_path(&X, theta_t, theta_ref, B[i], pos + (size_t)i * M * 3, sid + (size_t)i * M, visit_grad, &A);
        part[2 * tid] = A.g[0];
        part[2 * tid + 1] = A.g[1];
    }
    grad[0] = grad[1] = 0.0;
    for (int t = 0; t < nt; ++t) {
        grad[0] += part[2 * t];
        grad[1] += part[2 * t + 1];
    }
    free(part);
    free((void*)X.omega);
}

/* log of the correction factor (Eq. correction factor) of each path: the sum
   over the directions drawn at the unknown sphere (those that led to a
   recorded vertex) of log pdf(theta_t) - log pdf(theta_ref); every other
   draw does not depend on theta. */
void psso_log_r(const pso_scene* s, const double theta_t[2], const double theta_ref[2], int64_t n,
                const int32_t* B, const double* pos, const int32_t* sid, double* log_r)
{
    const int M = s->max_order;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double* P = pos + (size_t)i * M * 3;
        const int32_t* S = sid + (size_t)i * M;
        double lr = 0.0, w_in[3];
        unit3(s->light, P, w_in, NULL);
        for (int b = 0; b + 1 < B[i]; ++b) {
            double w_out[3], n[3];
            unit3(P + 3 * b, P + 3 * (b + 1), w_out, NULL);
            if (is_phong(s, S[b])) {
                psso_normal(s, S[b], P + 3 * b, n);
                double r[3];
                mirror(w_in, n, r);
                double nc = dot3(n, w_out), cr = dot3(r, w_out);
                lr += log(psso_phong_pdf(theta_t[0], theta_t[1], nc, cr)) -
                      log(psso_phong_pdf(theta_ref[0], theta_ref[1], nc, cr));
            }
            for (int a = 0; a < 3; ++a) w_in[a] = w_out[a];
        }
        log_r[i] = lr;
    }
}
