// Device-side building blocks shared by the gfx950 kernels: scene/camera
// parameter blocks, Philox4x32-10, phase functions, the orthonormal basis,
// and the incremental 3-D DDA voxel walkers (Amanatides & Woo style).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace prt {

constexpr int kWave = 64;
constexpr int kMaxCams = 24;
constexpr int kMaxOrder = 64;
constexpr double kPi = 3.14159265358979323846;

// Scene constants in the units the kernels use (grid units for lengths).
struct DevScene {
    int nx, ny, nz, max_order;
    double vk;              // voxel edge [km]
    double beta_air;        // 1/km
    double w_c, w_a;        // single-scattering albedos
    double g;               // HG asymmetry
    double hg_num;          // (1 - g^2) / (4 pi)
    double sun[3];          // propagation direction of the sun's rays
    double a_top, a_x, a_y; // projected areas of the lit faces [km^2]
    double w0;              // source weight F0 * projected box area
    double x_face, y_face;  // grid coordinate of the lit x / y face
    double inv_nx, inv_ny, inv_nxy; // 1 / nx, 1 / ny and 1 / (nx * ny), for voxel_ijk
};

// Cameras with positions converted to grid units.
struct DevCams {
    int n, W, H;
    int outside;  // every camera lies outside the grid box: connections end at the box boundary
    double pos[kMaxCams][3];
    double rot[kMaxCams][9];
    double f[kMaxCams];
};

// ------------------------------------------------------------ Philox4x32-10

__device__ __forceinline__ void philox4x32_10(uint32_t k0, uint32_t k1, uint32_t& x0, uint32_t& x1,
                                              uint32_t& x2, uint32_t& x3)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
        const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
        const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
}

// Four uniforms in (0,1) for (path, event): (x + 1/2) 2^-32, exact in FP64.
__device__ __forceinline__ void uniforms4(uint64_t seed, uint64_t path, uint32_t event, double u[4])
{
    uint32_t x0 = (uint32_t)path, x1 = (uint32_t)(path >> 32), x2 = event, x3 = 0u;
    philox4x32_10((uint32_t)seed, (uint32_t)(seed >> 32), x0, x1, x2, x3);
    u[0] = ((double)x0 + 0.5) * 0x1p-32;
    u[1] = ((double)x1 + 0.5) * 0x1p-32;
    u[2] = ((double)x2 + 0.5) * 0x1p-32;
    u[3] = ((double)x3 + 0.5) * 0x1p-32;
}

// ---------------------------------------------------------- phase functions

__device__ __forceinline__ double phase_hg(const DevScene& s, double mu)
{
    const double d = 1.0 + s.g * s.g - 2.0 * s.g * mu;
    return s.hg_num / (d * sqrt(d));
}

__device__ __forceinline__ double phase_rayleigh(double mu)
{
    return (3.0 / (16.0 * kPi)) * (1.0 + mu * mu);
}

// (the sampling helpers below run in the event precision E of the sampler:
// double in the all-FP64 mode, float with FP32 traversal)
__device__ __forceinline__ void sincos_e(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sincos_e(float x, float* s, float* c) { sincosf(x, s, c); }
template <typename E>
__device__ __forceinline__ E sample_hg(E u, E g)
{
    E mu;
    if (fabs(g) < (E)1e-6) {
        mu = (E)2 * u - (E)1;
    } else {
        const E s = ((E)1 - g * g) / ((E)1 - g + (E)2 * g * u);
        mu = ((E)1 + g * g - s * s) / ((E)2 * g);
    }
    return fmin((E)1, fmax((E)-1, mu));
}

// Rayleigh: the cubic mu^3 + 3 mu + 4 - 8u = 0 has the single real root s - 1/s,
// s = cbrt(q + sqrt(q^2 + 1)), q = 4u - 2.
template <typename E>
__device__ __forceinline__ E sample_rayleigh(E u)
{
    const E q = (E)4 * u - (E)2;
    const E s = cbrt(q + sqrt(q * q + (E)1));
    return fmin((E)1, fmax((E)-1, s - (E)1 / s));
}

// New direction at cosine mu, azimuth phi about n, in the branchless
// orthonormal basis of Duff et al. (JCGT 2017); renormalised.
template <typename E>
__device__ __forceinline__ void scatter_direction(const E n[3], E mu, E phi, E out[3])
{
    const E sgn = n[2] >= (E)0 ? (E)1 : (E)-1;
    const E a = (E)-1 / (sgn + n[2]);
    const E b = n[0] * n[1] * a;
    const E e1x = (E)1 + sgn * n[0] * n[0] * a, e1y = sgn * b, e1z = -sgn * n[0];
    const E e2x = b, e2y = sgn + n[1] * n[1] * a, e2z = -n[1];
    const E st = sqrt(fmax((E)0, (E)1 - mu * mu));
    E sp, cp;
    sincos_e(phi, &sp, &cp);
    const E wx = mu * n[0] + st * (cp * e1x + sp * e2x);
    const E wy = mu * n[1] + st * (cp * e1y + sp * e2y);
    const E wz = mu * n[2] + st * (cp * e1z + sp * e2z);
    const E inv = (E)1 / sqrt(wx * wx + wy * wy + wz * wz);
    out[0] = wx * inv;
    out[1] = wy * inv;
    out[2] = wz * inv;
}

// Scattering "directional function" f_s = w_c beta_c f_HG + w_a beta_a f_R.
__device__ __forceinline__ double fs_mix(const DevScene& s, double beta_c, double hg, double ray)
{
    return s.w_c * beta_c * hg + s.w_a * s.beta_air * ray;
}

// -------------------------------------------------------------- projection

// FP64 pinhole projection of a grid-unit point; returns pixel or -1.
__device__ __forceinline__ int project(const DevCams& c, int d, double x, double y, double z, double vk)
{
    const double* R = c.rot[d];
    const double qx = (x - c.pos[d][0]) * vk, qy = (y - c.pos[d][1]) * vk, qz = (z - c.pos[d][2]) * vk;
    const double px = R[0] * qx + R[1] * qy + R[2] * qz;
    const double py = R[3] * qx + R[4] * qy + R[5] * qz;
    const double pz = R[6] * qx + R[7] * qy + R[8] * qz;
    if (!(pz > 0.0)) return -1;
    const double iz = 1.0 / pz;
    const double u = c.f[d] * px * iz + 0.5 * c.W;
    const double v = c.f[d] * py * iz + 0.5 * c.H;
    if (!(u >= 0.0 && u < c.W && v >= 0.0 && v < c.H)) return -1;
    const int col = min((int)floor(u), c.W - 1);
    const int row = min((int)floor(v), c.H - 1);
    return row * c.W + col;
}

// ------------------------------------------------------------ LDS fills

// dst[i] = value(i) for i < n by the workgroup's threads, kFillLoads values
// per thread loaded before any is stored (the loads of a plain loop wait one
// at a time); value is called with an index clamped to n - 1, so every load
// stays in bounds.
constexpr int kFillLoads = 8;

template <typename T, typename F>
__device__ __forceinline__ void lds_fill(T* dst, int n, F&& value)
{
    const int step = (int)blockDim.x;
    for (int i0 = (int)threadIdx.x; i0 < n; i0 += kFillLoads * step) {
        T v[kFillLoads];
#pragma unroll
        for (int j = 0; j < kFillLoads; ++j) v[j] = value(min(i0 + j * step, n - 1));
#pragma unroll
        for (int j = 0; j < kFillLoads; ++j)
            if (i0 + j * step < n) dst[i0 + j * step] = v[j];
    }
}

// ------------------------------------------------------------- DDA walker

// Steps of the incremental voxel walk along p + t w, from voxel (ix,iy,iz)
// at parameter t (grid units) up to tmax, inside the box [0,nx) x [0,ny) x
// [z0,z1) (all layers, or a slab of z layers).  The functor is called as
// f(voxel, t_start, length) for every piece in order, with length >= 0
// (zero for a degenerate piece, e.g. when p sits on a voxel face) and the
// voxel numbered inside the box (ix + nx*(iy + ny*(iz - z0))); it returns
// false to stop the walk.  Returns the parameter t reached (the box exit,
// tmax, or where the functor stopped) and adds the number of pieces visited
// to *pieces.
//
// The step is branchless: the axis of the nearest face is chosen with
// selects, and each axis carries the number of faces left before the box
// boundary, so leaving the box needs no index bound checks.  Every
// iteration uses up one face of one axis and leaves the loop when an axis
// has none left, so the walk ends after at most (faces left) + 1 pieces for
// any input, including non-finite directions (whose components are treated
// as zero).  Face parameters are always measured from p, so a walk that
// starts part way (t > 0) produces the same pieces as one started at p.
// The step loop shared by every walk: R packs the faces left before the
// boundary along x, y and z in 10-bit fields that start at 512 + faces (a
// step past the last face of an axis clears that field's bit 9; dimensions
// are at most 512 voxels), v is the voxel index, dvx/dvy/dvz the index steps.
template <typename Real, bool kBounded, typename F>
__device__ __forceinline__ Real dda_loop(int R, int v, int dvx, int dvy, int dvz, Real tnx, Real tny, Real tnz,
                                         Real dtx, Real dty, Real dtz, Real t, Real tmax, uint32_t& pieces, F&& f)
{
    constexpr int kGuard = (1 << 9) | (1 << 19) | (1 << 29);
    const int R0 = R;
    for (;;) {
        const Real tn = fmin(tnx, fmin(tny, tnz));
        const bool go = !kBounded || tn < tmax;
        // the face parameters only grow, so te never decreases along the walk
        const Real te = kBounded ? (go ? tn : tmax) : tn;
        if (!f(v, t, te - t)) break;
        t = te;
        const bool bx = tnx == tn;
        const bool by = !bx && tny == tn;
        const bool bz = !bx && !by;
        R -= bx ? 1 : (by ? 1 << 10 : 1 << 20);
        v += bx ? dvx : (by ? dvy : dvz);
        tnx += bx ? dtx : (Real)0;
        tny += by ? dty : (Real)0;
        tnz += bz ? dtz : (Real)0;
        if ((kBounded && !go) || (R & kGuard) != kGuard) break;
    }
    // every piece (but one stopped by the functor) used up one face count
    const int used = (R0 & 1023) + ((R0 >> 10) & 1023) + (R0 >> 20) - (R & 1023) - ((R >> 10) & 1023) - (R >> 20);
    pieces += (uint32_t)used;
    return t;
}

// Face parameter of the next face along one axis (direction sign s, inverse
// component iv) from voxel i, clamped to the start t so that no piece is
// negative.
template <typename Real>
__device__ __forceinline__ Real dda_first_face(int s, int i, Real p, Real iv, Real t)
{
    return fmax(s > 0 ? ((Real)(i + 1) - p) * iv : (s < 0 ? ((Real)i - p) * iv : (Real)INFINITY), t);
}

template <typename Real, bool kBounded = true, typename F>
__device__ __forceinline__ Real dda_steps(int nx, int ny, int z0, int z1, Real px, Real py, Real pz, int ix, int iy,
                                          int iz, int sx, int sy, int sz, Real ivx, Real ivy, Real ivz, Real t,
                                          Real tmax, uint32_t& pieces, F&& f)
{
    const int rx = sx > 0 ? nx - 1 - ix : ix;
    const int ry = sy > 0 ? ny - 1 - iy : iy;
    const int rz = sz > 0 ? z1 - 1 - iz : iz - z0;
    const int R = (rx + 512) | (ry + 512) << 10 | (rz + 512) << 20;
    return dda_loop<Real, kBounded>(R, ix + nx * (iy + ny * (iz - z0)), sx, sy * nx, sz * nx * ny,
                                    dda_first_face(sx, ix, px, ivx, t), dda_first_face(sy, iy, py, ivy, t),
                                    dda_first_face(sz, iz, pz, ivz, t), (Real)sx * ivx, (Real)sy * ivy,
                                    (Real)sz * ivz, t, tmax, pieces, f);
}

// Inverse of a direction component: FP32 walks take the hardware reciprocal
// (within 1 ulp; the walk's pieces need no correctly rounded inverse, and its
// face counts, not the face parameters, bound it), FP64 walks the division.
__device__ __forceinline__ float dda_inv(float w) { return __builtin_amdgcn_rcpf(w); }
__device__ __forceinline__ double dda_inv(double w) { return 1.0 / w; }

// Direction signs and inverse components; false when w has no nonzero
// component.
template <typename Real>
__device__ __forceinline__ bool dda_dir(Real wx, Real wy, Real wz, int& sx, int& sy, int& sz, Real& ivx, Real& ivy,
                                        Real& ivz)
{
    sx = wx > (Real)0 ? 1 : (wx < (Real)0 ? -1 : 0);
    sy = wy > (Real)0 ? 1 : (wy < (Real)0 ? -1 : 0);
    sz = wz > (Real)0 ? 1 : (wz < (Real)0 ? -1 : 0);
    ivx = sx ? dda_inv(wx) : (Real)0;
    ivy = sy ? dda_inv(wy) : (Real)0;
    ivz = sz ? dda_inv(wz) : (Real)0;
    return sx != 0 || sy != 0 || sz != 0;
}

// Walk over the whole grid from p (in voxel (ix,iy,iz)) until the ray leaves
// the grid (or the functor stops it); no length bound, so the loop tests only
// the face counts.
template <typename Real, typename F>
__device__ __forceinline__ Real dda_walk(int nx, int ny, int nz, Real px, Real py, Real pz, int ix, int iy,
                                         int iz, Real wx, Real wy, Real wz, F&& f)
{
    int sx, sy, sz;
    Real ivx, ivy, ivz;
    if (!dda_dir(wx, wy, wz, sx, sy, sz, ivx, ivy, ivz)) return (Real)0;
    uint32_t pieces = 0;
    return dda_steps<Real, false>(nx, ny, 0, nz, px, py, pz, ix, iy, iz, sx, sy, sz, ivx, ivy, ivz, (Real)0,
                                  (Real)INFINITY, pieces, f);
}

// As dda_walk for t in [0, tmax] (unbounded without kBounded), adding the
// number of pieces visited to *pieces.
template <typename Real, bool kBounded = true, typename F>
__device__ __forceinline__ Real dda_walk_counted(int nx, int ny, int nz, Real px, Real py, Real pz, int ix, int iy,
                                                 int iz, Real wx, Real wy, Real wz, Real tmax, uint32_t& pieces,
                                                 F&& f)
{
    int sx, sy, sz;
    Real ivx, ivy, ivz;
    if (!dda_dir(wx, wy, wz, sx, sy, sz, ivx, ivy, ivz)) return (Real)0;
    return dda_steps<Real, kBounded>(nx, ny, 0, nz, px, py, pz, ix, iy, iz, sx, sy, sz, ivx, ivy, ivz, (Real)0, tmax,
                                     pieces, f);
}

// Sum of value(voxel) * length over the pieces of the walk of
// dda_walk_counted, t in [0, tmax] (unbounded without kBounded), with U
// pieces formed before their U values are fetched: a lane then has U loads
// in flight, which hides the latency of a grid in global memory.  The pieces
// and the order of the additions are those of the plain walk (a step past the
// end of the walk repeats the last voxel with length 0 and adds nothing), so
// the sum equals the plain walk's bit for bit; pieces are counted as there.
//
// kTileZ: value() takes voxel indices of the z-tiled layout (tile_index):
// a step along z moves by one inside a tile of kTileZ layers and by a tile
// row between tiles.
constexpr int kTileZ = 4;

__host__ __device__ inline int64_t tile_index(int ix, int iy, int iz, int nx, int ny)
{
    return (((int64_t)(iz / kTileZ) * ny + iy) * nx + ix) * kTileZ + iz % kTileZ;
}

// Linear voxel index (ix + nx (iy + ny iz)) of z-tiled index t; the
// divisions by nx and ny as in voxel_ijk.
__device__ __forceinline__ int tile_to_linear(int t, int nx, int ny, double inv_nx, double inv_ny)
{
    const int r = t / kTileZ;  // ((iz / kTileZ) * ny + iy) * nx + ix
    const int row = (int)floor(((double)r + 0.5) * inv_nx);
    const int ix = r - row * nx;
    const int tz = (int)floor(((double)row + 0.5) * inv_ny);
    const int iy = row - tz * ny;
    return ix + nx * (iy + ny * (tz * kTileZ + t % kTileZ));
}

// Voxel index of a walk, stepped with the walk: linear, or z-tiled; times
// kScale (e.g. the element size, so that the walk steps a byte offset).
template <bool kTiled, int kScale = 1>
struct WalkIndex {
    int v, dvx, dvy, dz_in, dz_out;
    int zl;  // z steps left before the tile boundary in the walk's direction
    __device__ __forceinline__ WalkIndex(int nx, int ny, int ix, int iy, int iz, int sx, int sy, int sz)
    {
        dvx = kScale * (kTiled ? sx * kTileZ : sx);
        dvy = kScale * (kTiled ? sy * nx * kTileZ : sy * nx);
        // a z step inside a tile, and one onto the next tile (the same as the
        // first without tiles)
        dz_in = kScale * (kTiled ? sz : sz * nx * ny);
        dz_out = kTiled ? kScale * sz * (nx * ny * kTileZ - (kTileZ - 1)) : dz_in;
        // opaque to the compiler: it would otherwise fold the step's choice
        // between sz and sz * X into a multiplication by a chosen factor
        // (a quarter-rate integer multiply per step, in a branch)
        if (kTiled) asm volatile("" : "+v"(dz_in), "+v"(dz_out));
        zl = kTiled ? (sz > 0 ? kTileZ - 1 - iz % kTileZ : iz % kTileZ) : 1;
        v = kScale * (kTiled ? (int)tile_index(ix, iy, iz, nx, ny) : ix + nx * (iy + ny * iz));
    }
    // the step along x, y or z (one of bx, by, bz), taken when `next`
    __device__ __forceinline__ void step(bool next, bool bx, bool by, bool bz)
    {
        const int dvz = kTiled && zl == 0 ? dz_out : dz_in;
        if (kTiled) zl = next && bz ? (zl == 0 ? kTileZ - 1 : zl - 1) : zl;
        v = next ? v + (bx ? dvx : (by ? dvy : dvz)) : v;
    }
};

// kScale: value() takes the voxel index times kScale (sizeof(Real): a byte
// offset into the grid).
template <int U, typename Real, bool kBounded, bool kTiled = false, int kScale = 1, typename G>
__device__ __forceinline__ Real dda_sum(int nx, int ny, int nz, Real px, Real py, Real pz, int ix, int iy, int iz,
                                        Real wx, Real wy, Real wz, Real tmax, uint32_t& pieces, G&& value)
{
    int sx, sy, sz;
    Real ivx, ivy, ivz;
    if (!dda_dir(wx, wy, wz, sx, sy, sz, ivx, ivy, ivz)) return (Real)0;
    constexpr int kGuard = (1 << 9) | (1 << 19) | (1 << 29);
    Real t = (Real)0;
    Real tnx = dda_first_face(sx, ix, px, ivx, t), tny = dda_first_face(sy, iy, py, ivy, t),
         tnz = dda_first_face(sz, iz, pz, ivz, t);
    const Real dtx = (Real)sx * ivx, dty = (Real)sy * ivy, dtz = (Real)sz * ivz;
    const int rx = sx > 0 ? nx - 1 - ix : ix;
    const int ry = sy > 0 ? ny - 1 - iy : iy;
    const int rz = sz > 0 ? nz - 1 - iz : iz;
    int R = (rx + 512) | (ry + 512) << 10 | (rz + 512) << 20;
    WalkIndex<kTiled, kScale> vi(nx, ny, ix, iy, iz, sx, sy, sz);
    bool alive = true;
    uint32_t n = 0;
    Real acc = (Real)0;
    for (;;) {
        int vv[U];
        Real ll[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const Real tn = fmin(tnx, fmin(tny, tnz));
            const bool go = !kBounded || tn < tmax;
            const Real te = kBounded ? (go ? tn : tmax) : tn;
            vv[k] = vi.v;
            ll[k] = alive ? te - t : (Real)0;
            n += alive ? 1u : 0u;
            const bool bx = tnx == tn;
            const bool by = !bx && tny == tn;
            const bool bz = !bx && !by;
            const int Rn = R - (bx ? 1 : (by ? 1 << 10 : 1 << 20));
            const bool next = alive && (!kBounded || go) && (Rn & kGuard) == kGuard;
            // the last piece's voxel stays: no step leaves the box
            R = next ? Rn : R;
            vi.step(next, bx, by, bz);
            t = next ? te : t;
            tnx = next && bx ? tnx + dtx : tnx;
            tny = next && by ? tny + dty : tny;
            tnz = next && bz ? tnz + dtz : tnz;
            alive = next;
        }
        Real bb[U];
#pragma unroll
        for (int k = 0; k < U; ++k) bb[k] = value((uint32_t)vv[k]);
#pragma unroll
        for (int k = 0; k < U; ++k) acc += bb[k] * ll[k];
        if (!alive) break;
    }
    pieces += n;
    return acc;
}

// The free flight of the sampler: the walk of dda_walk (unbounded, to the box
// exit) accumulating value(voxel) * length until the optical depth tau is
// passed, with U pieces formed before their U values are fetched (as
// dda_sum).  Returns the voxel of the piece in which the accumulated depth
// first exceeds tau (strictly: tau < acc + value * length), setting *acc to
// the depth before that piece and *t0 to the piece's start, or -1 when the
// ray leaves the box first, setting *t0 to the exit parameter.  The pieces,
// the order of the additions and the comparisons are those of a dda_walk
// functor doing the same, so both give the same result.  kTiled: voxel
// indices (value's argument and the result) of the z-tiled layout; both
// times kScale (sizeof(Real): byte offsets).
template <int U, typename Real, bool kTiled = false, int kScale = 1, typename G>
__device__ __forceinline__ int dda_first_hit(int nx, int ny, int nz, Real px, Real py, Real pz, int ix, int iy, int iz,
                                             Real wx, Real wy, Real wz, Real tau, G&& value, Real* acc_out,
                                             Real* t0_out)
{
    int sx, sy, sz;
    Real ivx, ivy, ivz;
    *acc_out = (Real)0;
    *t0_out = (Real)0;
    if (!dda_dir(wx, wy, wz, sx, sy, sz, ivx, ivy, ivz)) return -1;
    constexpr int kGuard = (1 << 9) | (1 << 19) | (1 << 29);
    Real t = (Real)0;
    Real tnx = dda_first_face(sx, ix, px, ivx, t), tny = dda_first_face(sy, iy, py, ivy, t),
         tnz = dda_first_face(sz, iz, pz, ivz, t);
    const Real dtx = (Real)sx * ivx, dty = (Real)sy * ivy, dtz = (Real)sz * ivz;
    const int rx = sx > 0 ? nx - 1 - ix : ix;
    const int ry = sy > 0 ? ny - 1 - iy : iy;
    const int rz = sz > 0 ? nz - 1 - iz : iz;
    int R = (rx + 512) | (ry + 512) << 10 | (rz + 512) << 20;
    WalkIndex<kTiled, kScale> vi(nx, ny, ix, iy, iz, sx, sy, sz);
    bool alive = true;
    Real acc = (Real)0;
    for (;;) {
        int vv[U];
        Real ll[U], ts[U];
        bool live[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const Real tn = fmin(tnx, fmin(tny, tnz));
            vv[k] = vi.v;
            ts[k] = t;
            ll[k] = tn - t;
            live[k] = alive;
            const bool bx = tnx == tn;
            const bool by = !bx && tny == tn;
            const bool bz = !bx && !by;
            const int Rn = R - (bx ? 1 : (by ? 1 << 10 : 1 << 20));
            const bool next = alive && (Rn & kGuard) == kGuard;
            // the exit parameter advances with the last piece; its voxel stays
            t = alive ? tn : t;
            R = next ? Rn : R;
            vi.step(next, bx, by, bz);
            tnx = next && bx ? tnx + dtx : tnx;
            tny = next && by ? tny + dty : tny;
            tnz = next && bz ? tnz + dtz : tnz;
            alive = next;
        }
        Real bb[U];
#pragma unroll
        for (int k = 0; k < U; ++k) bb[k] = value((uint32_t)vv[k]);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (!live[k]) break;
            const Real dt = bb[k] * ll[k];
            if (tau < acc + dt) {
                *acc_out = acc;
                *t0_out = ts[k];
                return vv[k];
            }
            acc += dt;
        }
        if (!alive) break;
    }
    *acc_out = acc;
    *t0_out = t;
    return -1;
}

// The part of that walk inside the slab of z layers [z0, z1) (pieces counted
// as in dda_walk_counted): the pieces
// are those of the whole-grid walk that fall in the slab, with voxels
// numbered inside the slab.  When p lies outside the slab the walk enters
// it through the near z face (if the ray reaches that face inside the box
// before tmax); the entry voxel is taken from the entry point, so a piece
// next to the entry can differ from the whole-grid walk by rounding only.
template <typename Real, bool kBounded = true, typename F>
__device__ __forceinline__ void dda_walk_slab(int nx, int ny, int z0, int z1, Real px, Real py, Real pz, int ix,
                                              int iy, int iz, Real wx, Real wy, Real wz, Real tmax,
                                              uint32_t& pieces, F&& f)
{
    int sx, sy, sz;
    Real ivx, ivy, ivz;
    if (!dda_dir(wx, wy, wz, sx, sy, sz, ivx, ivy, ivz)) return;
    Real t = (Real)0;
    if (iz < z0 || iz >= z1) {
        const bool below = iz < z0;
        if (below ? sz <= 0 : sz >= 0) return;
        t = ((Real)(below ? z0 : z1) - pz) * ivz;
        if (!(t < tmax)) return;
        const Real x = px + t * wx, y = py + t * wy;
        if (!(x >= (Real)0 && x <= (Real)nx && y >= (Real)0 && y <= (Real)ny)) return;
        ix = min((int)x, nx - 1);
        iy = min((int)y, ny - 1);
        iz = below ? z0 : z1 - 1;
        t = fmax(t, (Real)0);
    }
    dda_steps<Real, kBounded>(nx, ny, z0, z1, px, py, pz, ix, iy, iz, sx, sy, sz, ivx, ivy, ivz, t, tmax, pieces, f);
}

// An axis-aligned block of the grid, voxels [lo[a], hi[a]) along axis a,
// numbered inside the block as sum over a of (i_a - lo[a]) * st[a].
struct SubBox {
    int lo[3], hi[3];
    int st[3];
};

// The part of the walk from p (in voxel (ix,iy,iz)) along w, t in [0, tmax]
// (unbounded without kBounded), that lies in the block b: the pieces of the
// whole-grid walk that fall in it, voxels numbered inside the block, pieces
// counted as in dda_walk_counted.  When p lies outside the block the walk
// enters it where the ray meets the block (if it does before tmax); the
// entry voxel is taken from the entry point, so a piece next to the entry can
// differ from the whole-grid walk by rounding only.
// (v0 is added to every voxel index the functor sees.)
template <typename Real, bool kBounded = true, typename F>
__device__ __forceinline__ void dda_walk_box(const SubBox& b, Real px, Real py, Real pz, int ix, int iy, int iz,
                                             Real wx, Real wy, Real wz, Real tmax, uint32_t& pieces, F&& f,
                                             int v0 = 0)
{
    int sx, sy, sz;
    Real ivx, ivy, ivz;
    if (!dda_dir(wx, wy, wz, sx, sy, sz, ivx, ivy, ivz)) return;
    Real t = (Real)0;
    const bool inside = ix >= b.lo[0] && ix < b.hi[0] && iy >= b.lo[1] && iy < b.hi[1] && iz >= b.lo[2] &&
                        iz < b.hi[2];
    if (!inside) {
        // slab clipping of the ray against the block (selects, no branches:
        // an axis the ray does not move along only has to hold the start)
        Real tn = (Real)0, tf = kBounded ? tmax : (Real)INFINITY;
        const int s[3] = {sx, sy, sz}, i[3] = {ix, iy, iz};
        const Real p[3] = {px, py, pz}, iv[3] = {ivx, ivy, ivz};
        bool miss = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const Real t1 = ((Real)b.lo[a] - p[a]) * iv[a], t2 = ((Real)b.hi[a] - p[a]) * iv[a];
            const bool still = s[a] == 0;
            miss = miss || (still && (i[a] < b.lo[a] || i[a] >= b.hi[a]));
            tn = still ? tn : fmax(tn, fmin(t1, t2));
            tf = still ? tf : fmin(tf, fmax(t1, t2));
        }
        if (miss || !(tn < tf)) return;
        t = tn;
        ix = min(max((int)floor(px + t * wx), b.lo[0]), b.hi[0] - 1);
        iy = min(max((int)floor(py + t * wy), b.lo[1]), b.hi[1] - 1);
        iz = min(max((int)floor(pz + t * wz), b.lo[2]), b.hi[2] - 1);
    }
    const int rx = sx > 0 ? b.hi[0] - 1 - ix : ix - b.lo[0];
    const int ry = sy > 0 ? b.hi[1] - 1 - iy : iy - b.lo[1];
    const int rz = sz > 0 ? b.hi[2] - 1 - iz : iz - b.lo[2];
    const int R = (rx + 512) | (ry + 512) << 10 | (rz + 512) << 20;
    const int v = v0 + (ix - b.lo[0]) * b.st[0] + (iy - b.lo[1]) * b.st[1] + (iz - b.lo[2]) * b.st[2];
    dda_loop<Real, kBounded>(R, v, sx * b.st[0], sy * b.st[1], sz * b.st[2], dda_first_face(sx, ix, px, ivx, t),
                             dda_first_face(sy, iy, py, ivy, t), dda_first_face(sz, iz, pz, ivz, t),
                             (Real)sx * ivx, (Real)sy * ivy, (Real)sz * ivz, t, tmax, pieces, f);
}

// Spatial sort key of a path (the store orders paths by size B, then by this
// key): the Morton code of the coarse cell (8 cells per axis) holding the
// path's first vertex after the source (its first scatter, or its entry
// point when it has none).  Paths next to each other in the store then start
// near each other, so their walks have similar lengths.
constexpr int kCellBits = 3;
constexpr int kCells = 1 << (3 * kCellBits);
__host__ __device__ inline uint32_t cell_key(int v, int nx, int ny, int nz)
{
    const int ix = v % nx, iy = (v / nx) % ny, iz = v / (nx * ny);
    const uint32_t cx = (uint32_t)(ix * (1 << kCellBits) / nx), cy = (uint32_t)(iy * (1 << kCellBits) / ny),
                   cz = (uint32_t)(iz * (1 << kCellBits) / nz);
    uint32_t m = 0;
    for (int k = 0; k < kCellBits; ++k)
        m |= ((cx >> k) & 1u) << (3 * k) | ((cy >> k) & 1u) << (3 * k + 1) | ((cz >> k) & 1u) << (3 * k + 2);
    return m;
}

// Voxel index components of a linear voxel id.
__device__ __forceinline__ void voxel_ijk(int v, int nx, int ny, int& ix, int& iy, int& iz)
{
    ix = v % nx;
    const int r = v / nx;
    iy = r % ny;
    iz = r / ny;
}

// The same from the scene's reciprocals: floor((v + 1/2) / d) computed as
// ((double)v + 0.5) * (1/d) is exact for 0 <= v < 2^31 and d <= 2^18 (the
// rounding errors stay below 2^-20 while the quotient lies at least 1/(2d)
// from an integer), and takes a few FP64 operations instead of an integer
// division each.
__device__ __forceinline__ void voxel_ijk(const DevScene& s, int v, int& ix, int& iy, int& iz)
{
    iz = (int)floor(((double)v + 0.5) * s.inv_nxy);
    const int r = v - iz * (s.nx * s.ny);
    iy = (int)floor(((double)r + 0.5) * s.inv_nx);
    ix = r - iy * s.nx;
}

__device__ __forceinline__ int vox_of(const float4& r) { return __float_as_int(r.w); }

}  // namespace prt
