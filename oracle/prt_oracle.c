/*
 * prt_oracle.c -- plain FP64 CPU oracle for path-recycling scattering tomography
 * (Czerninski & Schechner, "Accelerating Inverse Rendering By Using a GPU and
 * Reuse of Light Paths", arXiv 2110.00085).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this library:
 * only tests/, the smoke check and the CPU-baseline leg of bench.py use it.  It
 * shares no source with the HIP library; the only thing the two sides share is
 * the path-store format (FP32 grid-unit vertices + int32 voxel ids) and the
 * random-number stream definition (Philox4x32-10, Salmon et al., SC'11).
 *
 * Everything is written straight from the paper's definitions, evaluated the
 * slow, obvious way:
 *   - distance sampling:  Sec. 3.4.1 (tau ~ Exp(1), solve T = exp(-tau))
 *   - direction sampling: Sec. 3.4.2 (choose particle type, sample its phase fn)
 *   - path pdf mu:        Eq. final_mu / App. B Eq. final_mu_app
 *   - contribution f:     Eq. cont_func_scattering with local estimation
 *                         (Sec. 3.4.3, Eq. Qd); G terms of sampled segments
 *                         cancel between f and mu (stated after Eq. explicit_foward)
 *   - recycling:          Eqs. forward_simualtion_recycling, correction factor,
 *                         gradient_simualtion_recycling (Sec. 5.2)
 *   - loss gradient:      Eq. loss_gradient with the tomography PSF of Sec. 4.4
 *                         (derived in App. C, Eq. fs_deriv)
 * Voxel/segment intersection lengths are found by listing every grid-plane
 * crossing, sorting them, and assigning each piece to the voxel containing its
 * midpoint (no incremental DDA).
 *
 * Units: lengths inside the grid are in voxel units ("grid units"); optical
 * depth = beta[1/km] * length[grid] * voxel_km.  Box = [0,nx]x[0,ny]x[0,nz],
 * z up, voxel v = ix + nx*(iy + ny*iz).
 *
 * Parity-unpinned parts: none of the functions below lacks a pin in tests/
 * except the absolute multiple-scattering radiance, which is pinned only by
 * the exit-flux cross-check (two different estimators of the same quantity).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PO_PI 3.14159265358979323846

/* ------------------------------------------------------------------ types */

typedef struct {
    int32_t nx, ny, nz, max_order;
    double voxel_km;          /* voxel edge [km] */
    double beta_air;          /* constant air extinction [1/km] (Sec. 6.1 scene settings) */
    double albedo_cloud;      /* single-scattering albedo of cloud droplets (Eq. sinscat) */
    double albedo_air;        /* single-scattering albedo of air */
    double g;                 /* Henyey-Greenstein asymmetry of the cloud phase function */
    double sun_zenith_deg, sun_azimuth_deg;
    double sun_flux;          /* F0, irradiance normal to the beam */
} po_scene;

typedef struct {
    int32_t n, width, height, pad;
    const double* pos;   /* [n][3] km */
    const double* rot;   /* [n][3][3] world->camera, rows = right, up, forward */
    const double* f_px;  /* [n] focal length in pixels */
} po_cams;

typedef struct { int32_t v; double t0, l; } po_piece;

/* ------------------------------------------------- Philox4x32-10 (SC'11) */

static const uint32_t PO_M0 = 0xD2511F53u;
static const uint32_t PO_M1 = 0xCD9E8D57u;
static const uint32_t PO_W0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PO_W1 = 0xBB67AE85u; /* sqrt(3) - 1 */

/* Ten Philox4x32 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
   multiplies words 0 and 2 by the two multipliers, and the new words are
   (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0); the key is bumped by the Weyl
   constants between rounds. */
void prto_philox4x32_10(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t k0 = key[0], k1 = key[1];
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PO_W0; k1 += PO_W1; }
        uint64_t p0 = (uint64_t)PO_M0 * x0;
        uint64_t p1 = (uint64_t)PO_M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Four uniforms for (path, event): key = (seed lo, seed hi), counter =
   (path lo, path hi, event, 0); u = (x + 1/2) * 2^-32, exact in FP64 and
   strictly inside (0, 1). */
static void po_uniforms(uint64_t seed, uint64_t path, uint64_t event, double u[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)path, (uint32_t)(path >> 32), (uint32_t)event, 0u};
    uint32_t x[4];
    prto_philox4x32_10(key, ctr, x);
    for (int i = 0; i < 4; ++i) u[i] = ((double)x[i] + 0.5) * 0x1p-32;
}

void prto_uniforms(uint64_t seed, uint64_t path, uint64_t event, double u[4])
{
    po_uniforms(seed, path, event, u);
}

/* --------------------------------------------------- phase functions */

/* Henyey-Greenstein, per steradian, mu = cos(scattering angle). */
double prto_phase_hg(double mu, double g)
{
    double d = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * PO_PI * d * sqrt(d));
}

/* Rayleigh, per steradian. */
double prto_phase_rayleigh(double mu)
{
    return 3.0 * (1.0 + mu * mu) / (16.0 * PO_PI);
}

/* Inverse CDF of HG in mu. */
double prto_sample_hg(double u, double g)
{
    double mu;
    if (fabs(g) < 1e-6) {
        mu = 2.0 * u - 1.0;
    } else {
        double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
        mu = (1.0 + g * g - s * s) / (2.0 * g);
    }
    return mu < -1.0 ? -1.0 : (mu > 1.0 ? 1.0 : mu);
}

/* Inverse CDF of Rayleigh in mu: root of mu^3 + 3 mu + 4 - 8u = 0 (Cardano). */
double prto_sample_rayleigh(double u)
{
    double q = 4.0 * u - 2.0;
    double s = cbrt(q + sqrt(q * q + 1.0));
    double mu = s - 1.0 / s;
    return mu < -1.0 ? -1.0 : (mu > 1.0 ? 1.0 : mu);
}

/* New unit direction at cosine mu and azimuth phi about n, in the branchless
   orthonormal basis of Duff et al., JCGT 6(1), 2017. */
void prto_new_direction(const double n[3], double mu, double phi, double out[3])
{
    double sgn = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sgn + n[2]);
    double b = n[0] * n[1] * a;
    double e1[3] = {1.0 + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]};
    double e2[3] = {b, sgn + n[1] * n[1] * a, -n[1]};
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double c = cos(phi), s = sin(phi);
    double w[3];
    for (int i = 0; i < 3; ++i) w[i] = mu * n[i] + st * (c * e1[i] + s * e2[i]);
    double len = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    for (int i = 0; i < 3; ++i) out[i] = w[i] / len;
}

/* ------------------------------------------------------------ medium */

/* Total extinction (Eq. ext_particles): cloud + air. */
static double po_beta(const po_scene* s, const double* bc, int v)
{
    return bc[v] + s->beta_air;
}

/* Scattering coefficient beta_s = w_c beta_c + w_a beta_a (Eqs. sinscat, eff_sinscat). */
static double po_beta_s(const po_scene* s, const double* bc, int v)
{
    return s->albedo_cloud * bc[v] + s->albedo_air * s->beta_air;
}

/* Directional function f_s = beta_s * f_p (Eq. fs, Eq. fs_scattering). */
static double po_fs(const po_scene* s, const double* bc, int v, double mu)
{
    return s->albedo_cloud * bc[v] * prto_phase_hg(mu, s->g)
         + s->albedo_air * s->beta_air * prto_phase_rayleigh(mu);
}

/* ------------------------------------------------------ ray pieces */

static int po_cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* Pieces of the ray p + t*w, t in [0, tmax], that lie inside the box.
   tbuf must hold nx+ny+nz+8 doubles, out the same number of pieces.
   *t_end receives the end of the clipped interval (box exit or tmax).
   Returns the number of pieces of nonzero length. */
static int po_ray_pieces(const po_scene* s, const double p[3], const double w[3], double tmax,
                         po_piece* out, double* tbuf, double* t_end)
{
    const int n[3] = {s->nx, s->ny, s->nz};
    double t0 = 0.0, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        if (w[a] == 0.0) {
            if (p[a] < 0.0 || p[a] > n[a]) { *t_end = 0.0; return 0; }
            continue;
        }
        double ta = (0.0 - p[a]) / w[a], tb = (n[a] - p[a]) / w[a];
        if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    *t_end = t1;
    if (!(t1 > t0)) { *t_end = t0 > 0.0 ? t0 : 0.0; return 0; }
    int m = 0;
    tbuf[m++] = t0;
    for (int a = 0; a < 3; ++a) {
        if (w[a] == 0.0) continue;
        double c0 = p[a] + t0 * w[a], c1 = p[a] + t1 * w[a];
        double lo = c0 < c1 ? c0 : c1, hi = c0 < c1 ? c1 : c0;
        for (double k = ceil(lo); k <= floor(hi); k += 1.0) {
            double t = (k - p[a]) / w[a];
            if (t > t0 && t < t1) tbuf[m++] = t;
        }
    }
    qsort(tbuf + 1, (size_t)(m - 1), sizeof(double), po_cmp_double);
    tbuf[m++] = t1;
    int np = 0;
    for (int i = 0; i + 1 < m; ++i) {
        double ta = tbuf[i], tb = tbuf[i + 1];
        if (!(tb > ta)) continue;
        double tm = 0.5 * (ta + tb);
        int idx[3];
        for (int a = 0; a < 3; ++a) {
            int k = (int)floor(p[a] + tm * w[a]);
            idx[a] = k < 0 ? 0 : (k >= n[a] ? n[a] - 1 : k);
        }
        out[np].v = idx[0] + s->nx * (idx[1] + s->ny * idx[2]);
        out[np].t0 = ta;
        out[np].l = tb - ta;
        ++np;
    }
    return np;
}

static int po_piece_cap(const po_scene* s) { return s->nx + s->ny + s->nz + 8; }

/* Exported for the DDA pins: pieces of the segment p -> p + tmax*w. */
int prto_ray_pieces(const po_scene* s, const double p[3], const double w[3], double tmax,
                    int32_t* vox, double* len, double* t_end)
{
    int cap = po_piece_cap(s);
    po_piece* pc = (po_piece*)malloc(sizeof(po_piece) * (size_t)cap);
    double* tb = (double*)malloc(sizeof(double) * (size_t)cap);
    int np = po_ray_pieces(s, p, w, tmax, pc, tb, t_end);
    for (int i = 0; i < np; ++i) { vox[i] = pc[i].v; len[i] = pc[i].l; }
    free(pc); free(tb);
    return np;
}

/* Optical depth [1] of a list of pieces under cloud field bc. */
static double po_tau(const po_scene* s, const double* bc, const po_piece* pc, int np)
{
    double tau = 0.0;
    for (int i = 0; i < np; ++i) tau += po_beta(s, bc, pc[i].v) * pc[i].l * s->voxel_km;
    return tau;
}

/* ------------------------------------------------------------ source */

/* Sun propagation direction (parallel rays, Sec. 6.1). */
static void po_sun_dir(const po_scene* s, double w[3])
{
    double th = s->sun_zenith_deg * PO_PI / 180.0, ph = s->sun_azimuth_deg * PO_PI / 180.0;
    w[0] = sin(th) * cos(ph);
    w[1] = sin(th) * sin(ph);
    w[2] = -cos(th);
}

/* Projected areas [km^2] of the lit faces (top, x-face, y-face) seen along w. */
static void po_lit_areas(const po_scene* s, const double w[3], double a[3])
{
    double Lx = s->nx * s->voxel_km, Ly = s->ny * s->voxel_km, Lz = s->nz * s->voxel_km;
    a[0] = Lx * Ly * fabs(w[2]);
    a[1] = Ly * Lz * fabs(w[0]);
    a[2] = Lx * Lz * fabs(w[1]);
}

double prto_source_weight(const po_scene* s)
{
    double w[3], a[3];
    po_sun_dir(s, w);
    po_lit_areas(s, w, a);
    return s->sun_flux * (a[0] + a[1] + a[2]);
}

/* --------------------------------------------------------- sampling */

static void po_store_vertex(float* xyz, int32_t* vox, int64_t slot, const double x[3], int32_t v)
{
    xyz[3 * slot + 0] = (float)x[0];
    xyz[3 * slot + 1] = (float)x[1];
    xyz[3 * slot + 2] = (float)x[2];
    vox[slot] = v;
}

/* Sample one path under cloud field bc (the reference parameters).  Writes
   up to max_order+2 vertices at slots [base, base+nv).  Returns B. */
static int po_sample_path(const po_scene* s, const double* bc, uint64_t seed, uint64_t id,
                          float* xyz, int32_t* vox, int64_t base, int32_t* nv_out,
                          po_piece* pc, double* tb)
{
    double u[4], w[3], a[3], x[3];
    po_sun_dir(s, w);
    po_lit_areas(s, w, a);
    double A = a[0] + a[1] + a[2];
    po_uniforms(seed, id, 0, u);
    /* entry point uniform over the projected area: pick a lit face with
       probability proportional to its projected area, then a uniform point */
    if (u[0] * A < a[0]) {
        x[0] = u[1] * s->nx; x[1] = u[2] * s->ny; x[2] = s->nz;
    } else if (u[0] * A < a[0] + a[1]) {
        x[0] = w[0] > 0.0 ? 0.0 : s->nx; x[1] = u[1] * s->ny; x[2] = u[2] * s->nz;
    } else {
        x[0] = u[1] * s->nx; x[1] = w[1] > 0.0 ? 0.0 : s->ny; x[2] = u[2] * s->nz;
    }
    int ix = (int)floor(x[0]), iy = (int)floor(x[1]), iz = (int)floor(x[2]);
    ix = ix < 0 ? 0 : (ix >= s->nx ? s->nx - 1 : ix);
    iy = iy < 0 ? 0 : (iy >= s->ny ? s->ny - 1 : iy);
    iz = iz < 0 ? 0 : (iz >= s->nz ? s->nz - 1 : iz);
    int nv = 0;
    po_store_vertex(xyz, vox, base + nv++, x, ix + s->nx * (iy + s->ny * iz));
    double tau = -log(u[3]);
    int b = 0;
    for (;;) {
        /* distance sampling: walk the pieces until the optical depth passes tau */
        double t_end;
        int np = po_ray_pieces(s, x, w, INFINITY, pc, tb, &t_end);
        double acc = 0.0;
        int hit = -1;
        double ts = 0.0;
        for (int i = 0; i < np; ++i) {
            double bt = po_beta(s, bc, pc[i].v);
            double dt = bt * pc[i].l * s->voxel_km;
            if (tau < acc + dt) {
                hit = pc[i].v;
                ts = pc[i].t0 + (tau - acc) / (bt * s->voxel_km);
                break;
            }
            acc += dt;
        }
        if (hit < 0) {
            double xe[3] = {x[0] + t_end * w[0], x[1] + t_end * w[1], x[2] + t_end * w[2]};
            po_store_vertex(xyz, vox, base + nv++, xe, -1);
            break;
        }
        for (int k = 0; k < 3; ++k) x[k] = x[k] + ts * w[k];
        ++b;
        po_store_vertex(xyz, vox, base + nv++, x, hit);
        if (b >= s->max_order) break;
        /* direction sampling: particle type with probability beta_s^(j)/beta_s,
           then a direction from that type's phase function */
        po_uniforms(seed, id, (uint64_t)b, u);
        double bsc = s->albedo_cloud * bc[hit];
        double bs = po_beta_s(s, bc, hit);
        double mu = (u[0] * bs < bsc) ? prto_sample_hg(u[1], s->g) : prto_sample_rayleigh(u[1]);
        double wn[3];
        prto_new_direction(w, mu, 2.0 * PO_PI * u[2], wn);
        w[0] = wn[0]; w[1] = wn[1]; w[2] = wn[2];
        tau = -log(u[3]);
    }
    *nv_out = nv;
    return b;
}

/* Sample n paths with ids ids[i] (or first_id + i when ids == NULL).  Output
   vertices go to fixed-capacity rows of max_order+2 slots. */
void prto_sample(const po_scene* s, const double* beta_c, uint64_t seed, uint64_t first_id,
                 const int64_t* ids, int64_t n, float* xyz, int32_t* vox, int32_t* B, int32_t* nv)
{
    const int64_t cap = s->max_order + 2;
#pragma omp parallel
    {
        int pcap = po_piece_cap(s);
        po_piece* pc = (po_piece*)malloc(sizeof(po_piece) * (size_t)pcap);
        double* tb = (double*)malloc(sizeof(double) * (size_t)pcap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            uint64_t id = ids ? (uint64_t)ids[i] : first_id + (uint64_t)i;
            B[i] = po_sample_path(s, beta_c, seed, id, xyz, vox, i * cap, &nv[i], pc, tb);
        }
        free(pc); free(tb);
    }
}

/* ---------------------------------------------------- local estimation */

/* Pinhole projection (FP64): pixel index row*W+col, or -1 when the point is
   behind the camera or outside the image. */
static int po_project(const po_cams* c, int d, const double xkm[3])
{
    const double* R = c->rot + 9 * d;
    const double* C = c->pos + 3 * d;
    double q[3] = {xkm[0] - C[0], xkm[1] - C[1], xkm[2] - C[2]};
    double px = R[0] * q[0] + R[1] * q[1] + R[2] * q[2];
    double py = R[3] * q[0] + R[4] * q[1] + R[5] * q[2];
    double pz = R[6] * q[0] + R[7] * q[1] + R[8] * q[2];
    if (!(pz > 0.0)) return -1;
    double uu = c->f_px[d] * px / pz + 0.5 * c->width;
    double vv = c->f_px[d] * py / pz + 0.5 * c->height;
    if (!(uu >= 0.0 && uu < c->width && vv >= 0.0 && vv < c->height)) return -1;
    int col = (int)floor(uu), row = (int)floor(vv);
    if (col >= c->width) col = c->width - 1;
    if (row >= c->height) row = c->height - 1;
    return row * c->width + col;
}

int prto_project(const po_cams* c, int d, const double xkm[3]) { return po_project(c, d, xkm); }

/* Exact solid angle of the pixel rectangle seen from the pinhole.
   F(x,y) = atan(x y / (f sqrt(x^2+y^2+f^2))) is the solid angle of the
   rectangle [0,x]x[0,y] on the image plane at distance f; the pixel's angle
   follows by inclusion-exclusion. */
static double po_F(double x, double y, double f)
{
    return atan(x * y / (f * sqrt(x * x + y * y + f * f)));
}

void prto_pixel_solid_angles(double f, int W, int H, double* out)
{
    for (int r = 0; r < H; ++r)
        for (int c = 0; c < W; ++c) {
            double x1 = c - 0.5 * W, x2 = x1 + 1.0, y1 = r - 0.5 * H, y2 = y1 + 1.0;
            out[r * W + c] = po_F(x2, y2, f) - po_F(x1, y2, f) - po_F(x2, y1, f) + po_F(x1, y1, f);
        }
}

/* ----------------------------------------------- per-path evaluation */

typedef struct {
    int B, Br, nv;
    double x[80][3];    /* vertices (grid units, FP64 copies of the stored FP32) */
    int v[80];
    double w[80][3];    /* direction of segment k (x_k -> x_{k+1}) */
    double len[80];
} po_path;

static int po_load_path(const po_scene* s, const int64_t* off, const float* xyz, const int32_t* vox,
                        const int32_t* B, int64_t i, int Brender, po_path* P)
{
    int64_t o = off[i];
    P->nv = (int)(off[i + 1] - o);
    P->B = B[i];
    P->Br = P->B < Brender ? P->B : Brender;
    if (P->nv > 80) return -1;
    for (int k = 0; k < P->nv; ++k) {
        for (int a = 0; a < 3; ++a) P->x[k][a] = (double)xyz[3 * (o + k) + a];
        P->v[k] = vox[o + k];
    }
    for (int k = 0; k + 1 < P->nv; ++k) {
        double d[3] = {P->x[k + 1][0] - P->x[k][0], P->x[k + 1][1] - P->x[k][1], P->x[k + 1][2] - P->x[k][2]};
        double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        P->len[k] = L;
        for (int a = 0; a < 3; ++a) P->w[k][a] = L > 0.0 ? d[a] / L : 0.0;
    }
    (void)s;
    return 0;
}

static double po_dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

typedef struct {
    double* seg_tau_t;   /* per segment optical depth at beta_t */
    double* seg_tau_r;   /* per segment optical depth at beta_ref */
    po_piece* seg_pc;    /* cached pieces of each segment (for the PSF) */
    int* seg_np;
    po_piece* pc;        /* scratch for connections */
    double* tb;
    int pcap;
} po_work;

static void po_work_init(const po_scene* s, po_work* W)
{
    W->pcap = po_piece_cap(s);
    int ns = s->max_order + 2;
    W->seg_tau_t = (double*)malloc(sizeof(double) * (size_t)ns);
    W->seg_tau_r = (double*)malloc(sizeof(double) * (size_t)ns);
    W->seg_pc = (po_piece*)malloc(sizeof(po_piece) * (size_t)ns * (size_t)W->pcap);
    W->seg_np = (int*)malloc(sizeof(int) * (size_t)ns);
    W->pc = (po_piece*)malloc(sizeof(po_piece) * (size_t)W->pcap);
    W->tb = (double*)malloc(sizeof(double) * (size_t)W->pcap);
}

static void po_work_free(po_work* W)
{
    free(W->seg_tau_t); free(W->seg_tau_r); free(W->seg_pc); free(W->seg_np); free(W->pc); free(W->tb);
}

/* Segments 0..nseg-1 of the stored path: pieces and optical depths under
   beta_t and beta_ref.  Returns the number of nonzero-length pieces. */
static int64_t po_segments(const po_scene* s, const double* bt, const double* br, const po_path* P,
                           int nseg, po_work* W)
{
    int64_t count = 0;
    for (int k = 0; k < nseg; ++k) {
        double t_end;
        po_piece* pk = W->seg_pc + (size_t)k * W->pcap;
        int np = po_ray_pieces(s, P->x[k], P->w[k], P->len[k], pk, W->tb, &t_end);
        W->seg_np[k] = np;
        W->seg_tau_t[k] = po_tau(s, bt, pk, np);
        W->seg_tau_r[k] = po_tau(s, br, pk, np);
        count += np;
    }
    return count;
}

typedef struct {
    double logf, logmu;   /* log MCF / log pdf of the prefix x_0..x_b (no connection) */
} po_prefix;

/* Prefix terms for the local-estimate sub-path ending at scatter b:
   log mu_ref = log(1/A) + sum_{k=1..b} [log beta_ref(x_k) - tau_ref(seg k-1)]
                        + sum_{k=1..b-1} log f_p,ref(x_k, mu_k)           (Eq. final_mu)
   log f_t    = log F0   - sum_{k=0..b-1} tau_t(seg k) + sum_{k=1..b-1} log f_s,t(x_k, mu_k)
                                                                          (Eq. cont_func_scattering) */
static po_prefix po_prefix_terms(const po_scene* s, const double* bt, const double* br, const po_path* P,
                                 int b, const po_work* W)
{
    double sw[3], a[3];
    po_sun_dir(s, sw);
    po_lit_areas(s, sw, a);
    double A = a[0] + a[1] + a[2];
    po_prefix r;
    r.logmu = -log(A);
    r.logf = log(s->sun_flux);
    for (int k = 1; k <= b; ++k) {
        r.logmu += log(po_beta(s, br, P->v[k])) - W->seg_tau_r[k - 1];
        r.logf += -W->seg_tau_t[k - 1];
    }
    for (int k = 1; k <= b - 1; ++k) {
        double mu = po_dot(P->w[k - 1], P->w[k]);
        r.logmu += log(po_fs(s, br, P->v[k], mu)) - log(po_beta_s(s, br, P->v[k]));
        r.logf += log(po_fs(s, bt, P->v[k], mu));
    }
    return r;
}

typedef struct {
    int pix;            /* pixel or -1 */
    double c;           /* contribution f/mu times the pixel response 1/Omega_p */
    double mu_bd;       /* cosine toward the camera */
    int np;             /* connection pieces (in W->pc) */
} po_le;

/* Local estimate from scatter b to camera d (Sec. 3.4.3): returns the
   recycled contribution f(x|beta_t) W_d / mu(x|beta_ref) (Eq.
   forward_simualtion_recycling); connection pieces are left in W->pc. */
static po_le po_local_estimate(const po_scene* s, const po_cams* cm, const double* bt, const po_path* P,
                               int b, int d, const po_prefix* pre, const double* omega, po_work* W)
{
    po_le e;
    e.pix = -1; e.c = 0.0; e.np = 0; e.mu_bd = 0.0;
    double xkm[3] = {P->x[b][0] * s->voxel_km, P->x[b][1] * s->voxel_km, P->x[b][2] * s->voxel_km};
    int pix = po_project(cm, d, xkm);
    if (pix < 0) return e;
    double cg[3], dv[3];
    for (int a = 0; a < 3; ++a) { cg[a] = cm->pos[3 * d + a] / s->voxel_km; dv[a] = cg[a] - P->x[b][a]; }
    double dist = sqrt(po_dot(dv, dv));
    double wd[3] = {dv[0] / dist, dv[1] / dist, dv[2] / dist};
    double mu_bd = po_dot(P->w[b - 1], wd);
    double t_end;
    int np = po_ray_pieces(s, P->x[b], wd, dist, W->pc, W->tb, &t_end);
    double tau_c = po_tau(s, bt, W->pc, np);
    double r2 = dist * dist * s->voxel_km * s->voxel_km;
    double Wd = 1.0 / omega[(size_t)d * cm->width * cm->height + pix];
    double logc = pre->logf + log(po_fs(s, bt, P->v[b], mu_bd)) - tau_c - log(r2) + log(Wd) - pre->logmu;
    e.pix = pix;
    e.c = exp(logc);
    e.mu_bd = mu_bd;
    e.np = np;
    return e;
}

static double* po_solid_angles(const po_cams* cm)
{
    size_t npx = (size_t)cm->width * cm->height;
    double* om = (double*)malloc(sizeof(double) * npx * (size_t)cm->n);
    for (int d = 0; d < cm->n; ++d) prto_pixel_solid_angles(cm->f_px[d], cm->width, cm->height, om + npx * d);
    return om;
}

/* ----------------------------------------------------------- render */

/* Recycled forward model F(beta_t | beta_ref) (Eq. forward_simualtion_recycling
   with local estimation): images[d][p] = (1/N) sum_paths sum_b c_{b,d} 1[pix=p].
   counters: [0] voxel-segments (free-flight + in-image connections), [1] local
   estimates.  Paths are given in CSR form (off[n+1]). */
int prto_render(const po_scene* s, const po_cams* cm, const double* beta_t, const double* beta_ref,
                int64_t n_total, int64_t n, const int64_t* off, const float* xyz, const int32_t* vox,
                const int32_t* B, int32_t Brender, double* images, int64_t* counters)
{
    const size_t npx = (size_t)cm->width * cm->height * (size_t)cm->n;
    double* omega = po_solid_angles(cm);
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double* priv = (double*)calloc(npx * (size_t)nth, sizeof(double));
    int64_t* cnt = (int64_t*)calloc(2 * (size_t)nth, sizeof(int64_t));
    int err = 0;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* img = priv + npx * (size_t)tid;
        po_work W;
        po_work_init(s, &W);
        po_path* P = (po_path*)malloc(sizeof(po_path));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            if (po_load_path(s, off, xyz, vox, B, i, Brender, P) != 0) { err = 1; continue; }
            if (P->Br == 0) continue;
            cnt[2 * tid] += po_segments(s, beta_t, beta_ref, P, P->Br, &W);
            for (int b = 1; b <= P->Br; ++b) {
                po_prefix pre = po_prefix_terms(s, beta_t, beta_ref, P, b, &W);
                for (int d = 0; d < cm->n; ++d) {
                    po_le e = po_local_estimate(s, cm, beta_t, P, b, d, &pre, omega, &W);
                    if (e.pix < 0) continue;
                    img[(size_t)d * cm->width * cm->height + e.pix] += e.c;
                    cnt[2 * tid] += e.np;
                    cnt[2 * tid + 1] += 1;
                }
            }
        }
        free(P);
        po_work_free(&W);
    }
    for (size_t p = 0; p < npx; ++p) {
        double acc = 0.0;
        for (int t = 0; t < nth; ++t) acc += priv[npx * (size_t)t + p];
        images[p] = acc / (double)n_total;
    }
    if (counters) {
        counters[0] = counters[1] = 0;
        for (int t = 0; t < nth; ++t) { counters[0] += cnt[2 * t]; counters[1] += cnt[2 * t + 1]; }
    }
    free(priv); free(cnt); free(omega);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------- grad */

/* Vertex term of the tomography PSF (App. C, Eq. fs_deriv):
   (beta_c,v + (w_a f_a(mu)/(w_c f_c(mu))) beta_a)^-1 */
static double po_psf_vertex(const po_scene* s, const double* bt, int v, double mu)
{
    double ratio = (s->albedo_air * prto_phase_rayleigh(mu)) / (s->albedo_cloud * prto_phase_hg(mu, s->g));
    return 1.0 / (bt[v] + ratio * s->beta_air);
}

/* Loss gradient (Eq. loss_gradient with the recycled derivative estimator,
   Eq. gradient_simualtion_recycling):
   grad[v] = sum_{d,p} residual[d][p] * (1/N) sum_paths sum_b c_{b,d} 1[pix=p] S_v(b,d),
   with S_v the tomography PSF of the local-estimate sub-path x_0..x_b -> camera:
   S_v = -sum_{segments incl. the connection} l_v [km]
         + sum_{k=1..b} 1[x_k in voxel v] (beta_c,v + w_a f_a/(w_c f_c) beta_a)^-1,
   where the cosine at x_b is the one toward the camera. */
int prto_grad(const po_scene* s, const po_cams* cm, const double* beta_t, const double* beta_ref,
              int64_t n_total, int64_t n, const int64_t* off, const float* xyz, const int32_t* vox,
              const int32_t* B, const double* residual, double* grad)
{
    const size_t nu = (size_t)s->nx * s->ny * s->nz;
    double* omega = po_solid_angles(cm);
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double* priv = (double*)calloc(nu * (size_t)nth, sizeof(double));
    int err = 0;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* g = priv + nu * (size_t)tid;
        po_work W;
        po_work_init(s, &W);
        po_path* P = (po_path*)malloc(sizeof(po_path));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            if (po_load_path(s, off, xyz, vox, B, i, s->max_order, P) != 0) { err = 1; continue; }
            if (P->Br == 0) continue;
            po_segments(s, beta_t, beta_ref, P, P->Br, &W);
            for (int b = 1; b <= P->Br; ++b) {
                po_prefix pre = po_prefix_terms(s, beta_t, beta_ref, P, b, &W);
                for (int d = 0; d < cm->n; ++d) {
                    po_le e = po_local_estimate(s, cm, beta_t, P, b, d, &pre, omega, &W);
                    if (e.pix < 0) continue;
                    double wgt = residual[(size_t)d * cm->width * cm->height + e.pix] * e.c;
                    if (wgt == 0.0) continue;
                    /* -l over the free-flight segments 0..b-1 */
                    for (int k = 0; k < b; ++k) {
                        const po_piece* pk = W.seg_pc + (size_t)k * W.pcap;
                        for (int j = 0; j < W.seg_np[k]; ++j) g[pk[j].v] -= wgt * pk[j].l * s->voxel_km;
                    }
                    /* -l over the connection */
                    for (int j = 0; j < e.np; ++j) g[W.pc[j].v] -= wgt * W.pc[j].l * s->voxel_km;
                    /* scatter vertices 1..b */
                    for (int k = 1; k <= b; ++k) {
                        double mu = (k < b) ? po_dot(P->w[k - 1], P->w[k]) : e.mu_bd;
                        g[P->v[k]] += wgt * po_psf_vertex(s, beta_t, P->v[k], mu);
                    }
                }
            }
        }
        free(P);
        po_work_free(&W);
    }
    for (size_t v = 0; v < nu; ++v) {
        double acc = 0.0;
        for (int t = 0; t < nth; ++t) acc += priv[nu * (size_t)t + v];
        grad[v] = acc / (double)n_total;
    }
    free(priv); free(omega);
    return err ? -1 : 0;
}

/* --------------------------------------------------------- reweight */

/* log of the full sampled-path pdf (Eq. final_mu, with the escape probability
   of the last segment when the path left the box and the direction pdf at
   every scatter that has a successor vertex), up to the source factor 1/A
   which cancels in the ratio.  The pdf carries the extinction beta(x_k) of
   every scatter vertex, so it is zero (log = -inf) when one of them is zero,
   whatever the phase function there. */
static double po_log_full_pdf(const po_scene* s, const double* bc, const po_path* P, po_work* W)
{
    double lp = 0.0;
    for (int k = 1; k <= P->B; ++k) {
        double b = po_beta(s, bc, P->v[k]);
        if (!(b > 0.0)) return -INFINITY;
        lp += log(b);
    }
    for (int k = 0; k + 1 < P->nv; ++k) {
        double t_end;
        int np = po_ray_pieces(s, P->x[k], P->w[k], P->len[k], W->pc, W->tb, &t_end);
        lp -= po_tau(s, bc, W->pc, np);
    }
    for (int k = 1; k + 1 < P->nv; ++k) {
        double mu = po_dot(P->w[k - 1], P->w[k]);
        lp += log(po_fs(s, bc, P->v[k], mu)) - log(po_beta_s(s, bc, P->v[k]));
    }
    return lp;
}

/* Per-path log of the recycling correction factor r = mu(x|beta_t)/mu(x|beta_ref)
   (Eq. correction factor) over the whole sampled path. */
int prto_reweight(const po_scene* s, const double* beta_t, const double* beta_ref, int64_t n,
                  const int64_t* off, const float* xyz, const int32_t* vox, const int32_t* B, double* logr)
{
    int err = 0;
#pragma omp parallel
    {
        po_work W;
        po_work_init(s, &W);
        po_path* P = (po_path*)malloc(sizeof(po_path));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            if (po_load_path(s, off, xyz, vox, B, i, s->max_order, P) != 0) { err = 1; continue; }
            logr[i] = po_log_full_pdf(s, beta_t, P, &W) - po_log_full_pdf(s, beta_ref, P, &W);
        }
        free(P);
        po_work_free(&W);
    }
    return err ? -1 : 0;
}

/* ----------------------------------------------------- space carving */

/* Photo-hull initialisation (Sec. 6.1, space carving after Kutulakos &
   Seitz): a voxel is removed when some camera sees its centre on a pixel
   whose value is at most that camera's threshold; a camera that does not see
   the centre (behind it or outside its image) removes nothing.  mask[v] = 1
   for the voxels kept. */
void prto_space_carve(const po_scene* s, const po_cams* cm, const double* images, const double* threshold,
                      uint8_t* mask)
{
    const size_t npx = (size_t)cm->width * cm->height;
    for (int iz = 0; iz < s->nz; ++iz)
        for (int iy = 0; iy < s->ny; ++iy)
            for (int ix = 0; ix < s->nx; ++ix) {
                double xkm[3] = {(ix + 0.5) * s->voxel_km, (iy + 0.5) * s->voxel_km, (iz + 0.5) * s->voxel_km};
                int keep = 1;
                for (int d = 0; d < cm->n; ++d) {
                    int pix = po_project(cm, d, xkm);
                    if (pix >= 0 && images[npx * (size_t)d + (size_t)pix] <= threshold[d]) keep = 0;
                }
                mask[ix + (size_t)s->nx * (iy + (size_t)s->ny * iz)] = (uint8_t)keep;
            }
}

int prto_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
