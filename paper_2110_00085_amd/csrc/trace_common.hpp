// Device helpers of the kernels on stored paths (trace.hip, ablation.hip):
// vertex records, walks that sum or scatter along a ray, the FP32 phase
// function, the recycled vertex factor, the slab blocks of the binned
// gradient, and the task counters of the persistent kernels.
#pragma once

#include "launch.hpp"

namespace prt {
namespace trace {


struct Vtx {
    double x, y, z;
    int v;
};

__device__ __forceinline__ Vtx load_vtx(const float4* __restrict__ V, int k)
{
    const float4 r = V[(int64_t)k * kWave];
    return Vtx{(double)r.x, (double)r.y, (double)r.z, vox_of(r)};
}

// Unit direction from a to b and the distance (grid units).
__device__ __forceinline__ double seg_dir(const Vtx& a, const Vtx& b, double w[3])
{
    const double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
    const double L = sqrt(dx * dx + dy * dy + dz * dz);
    const double inv = L > 0.0 ? 1.0 / L : 0.0;
    w[0] = dx * inv;
    w[1] = dy * inv;
    w[2] = dz * inv;
    return L;
}

__device__ __forceinline__ int clamp_vox(int v, int nu) { return min(max(v, 0), nu - 1); }

// Sum of beta(v) * length over the walk from vertex p (voxel p.v) along w
// for length tmax (grid units); adds the number of pieces to count.  With
// U > 1 the walk forms U pieces before fetching their values (for grids in
// global memory; same sum).
template <typename Real, bool kBounded = true, int U = 1, bool kTiled = false, int kScale = 1, typename G>
__device__ __forceinline__ Real walk_sum(const DevScene& s, G&& beta, const Vtx& p, const double w[3], double tmax,
                                         uint64_t& count)
{
    int ix, iy, iz;
    voxel_ijk(s, clamp_vox(p.v, s.nx * s.ny * s.nz), ix, iy, iz);
    static_assert((!kTiled && kScale == 1) || U > 1, "the z-tiled layout and byte offsets are walked by dda_sum");
    if constexpr (U > 1) {
        uint32_t n = 0;
        const Real acc = dda_sum<U, Real, kBounded, kTiled, kScale>(s.nx, s.ny, s.nz, (Real)p.x, (Real)p.y, (Real)p.z, ix, iy,
                                                            iz, (Real)w[0], (Real)w[1], (Real)w[2], (Real)tmax, n,
                                                            beta);
        count += n;
        return acc;
    }
    Real acc = (Real)0;
    uint32_t n = 0;
    dda_walk_counted<Real, kBounded>(s.nx, s.ny, s.nz, (Real)p.x, (Real)p.y, (Real)p.z, ix, iy, iz, (Real)w[0], (Real)w[1],
                           (Real)w[2], (Real)tmax, n, [&](int v, Real, Real l) {
                               acc += beta((uint32_t)v) * l;
                               return true;
                           });
    count += n;
    return acc;
}

// Calls add(v, scale * length) for every piece of the walk that lies in the
// slab of z layers [z0, z1), v numbered inside the slab (zero-length pieces
// add zero).
template <typename Real, bool kBounded = true, typename A>
__device__ __forceinline__ void walk_scatter(const DevScene& s, A&& add, const Vtx& p, const double w[3], double tmax,
                                             double scale, uint64_t& count, int z0, int z1)
{
    int ix, iy, iz;
    voxel_ijk(s, clamp_vox(p.v, s.nx * s.ny * s.nz), ix, iy, iz);
    uint32_t n = 0;
    dda_walk_slab<Real, kBounded>(s.nx, s.ny, z0, z1, (Real)p.x, (Real)p.y, (Real)p.z, ix, iy, iz, (Real)w[0], (Real)w[1],
                        (Real)w[2], (Real)tmax, n, [&](int v, Real, Real l) {
                            add((uint32_t)v, scale * (double)l);
                            return true;
                        });
    count += n;
}

// As walk_scatter for the part of the walk inside the block b (voxels
// numbered inside the block).
template <typename Real, bool kBounded = true, typename A>
__device__ __forceinline__ void walk_scatter_box(const DevScene& s, A&& add, const Vtx& p, const double w[3],
                                                 double tmax, double scale, uint64_t& count, const SubBox& b)
{
    int ix, iy, iz;
    voxel_ijk(s, clamp_vox(p.v, s.nx * s.ny * s.nz), ix, iy, iz);
    uint32_t n = 0;
    dda_walk_box<Real, kBounded>(b, (Real)p.x, (Real)p.y, (Real)p.z, ix, iy, iz, (Real)w[0], (Real)w[1], (Real)w[2],
                                 (Real)tmax, n, [&](int v, Real, Real l) {
                                     add((uint32_t)v, scale * (double)l);
                                     return true;
                                 });
    count += n;
}

// As walk_scatter_box for an FP32 walk given in floats: from point (px,py,pz)
// in voxel v along the unit direction (wx,wy,wz) up to tmax.
template <bool kBounded = true, typename A>
__device__ __forceinline__ void walk_scatter_box_f(const DevScene& s, A&& add, float px, float py, float pz, int v,
                                                   float wx, float wy, float wz, float tmax, double scale,
                                                   uint64_t& count, const SubBox& b)
{
    int ix, iy, iz;
    voxel_ijk(s, clamp_vox(v, s.nx * s.ny * s.nz), ix, iy, iz);
    uint32_t n = 0;
    dda_walk_box<float, kBounded>(b, px, py, pz, ix, iy, iz, wx, wy, wz, tmax, n, [&](int u, float, float l) {
        add((uint32_t)u, scale * (double)l);
        return true;
    });
    count += n;
}

// An FP64 tally in LDS addressed in bytes: walks over it step the byte
// address itself (strides times 8 from the tally's start), which saves the
// index-to-address arithmetic of every piece.
typedef __attribute__((address_space(3))) double lds_double;

struct LdsTally {
    uint32_t base;  // byte address of element 0
    SubBox box;     // the block, with strides in bytes
    __device__ __forceinline__ LdsTally(double* tally, const SubBox& b) : box(b)
    {
        base = (uint32_t)(uintptr_t)(lds_double*)tally;
#pragma unroll
        for (int k = 0; k < 3; ++k) box.st[k] = b.st[k] * (int)sizeof(double);
    }
    __device__ __forceinline__ static void add_at(uint32_t addr, double x)
    {
        __hip_atomic_fetch_add((lds_double*)(uintptr_t)addr, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
};

// As walk_scatter_box_f, adding scale * length into the LDS tally t.
template <bool kBounded = true>
__device__ __forceinline__ void walk_tally_box_f(const DevScene& s, const LdsTally& t, float px, float py, float pz,
                                                 int v, float wx, float wy, float wz, float tmax, double scale,
                                                 uint64_t& count)
{
    int ix, iy, iz;
    voxel_ijk(s, clamp_vox(v, s.nx * s.ny * s.nz), ix, iy, iz);
    uint32_t n = 0;
    dda_walk_box<float, kBounded>(
        t.box, px, py, pz, ix, iy, iz, wx, wy, wz, tmax, n,
        [&](int a, float, float l) {
            LdsTally::add_at((uint32_t)a, scale * (double)l);
            return true;
        },
        (int)t.base);
    count += n;
}

// Slab `slab` of the binned gradient as a block of the grid, numbered with
// the slab axis slowest (its voxels are contiguous in the slab tally).
// (selects rather than indexing by the runtime axis, so that the block stays
// in registers)
__device__ __forceinline__ SubBox slab_box(const DevScene& s, int axis, int layers, int slab)
{
    const int n[3] = {s.nx, s.ny, s.nz};
    const int nb = axis == 0 ? s.ny : s.nx;                 // first other axis
    const int nc = axis == 2 ? s.ny : s.nz;                 // second other axis
    SubBox b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const bool on = k == axis;
        const bool first_other = k == (axis == 0 ? 1 : 0);
        b.lo[k] = on ? slab * layers : 0;
        b.hi[k] = on ? min(n[k], slab * layers + layers) : n[k];
        b.st[k] = on ? nb * nc : (first_other ? 1 : nb);
    }
    return b;
}

// Index of grid voxel v inside block b, or -1 outside it.
__device__ __forceinline__ int box_index(const SubBox& b, int v, const DevScene& s)
{
    int i[3];
    voxel_ijk(s, v, i[0], i[1], i[2]);
    int u = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (i[k] < b.lo[k] || i[k] >= b.hi[k]) return -1;
        u += (i[k] - b.lo[k]) * b.st[k];
    }
    return u;
}

// Layer (along the slab axis) of a point at coordinate x on that axis in
// voxel layer i, widened by eps on both sides: [lo, hi] grows to cover it.
constexpr int kNoLayer = 0x7fffffff;

__device__ __forceinline__ void layer_span(float x, int i, int& lo, int& hi)
{
    constexpr float eps = 1e-3f;
    lo = min(lo, min(i, (int)floorf(x - eps)));
    hi = max(hi, max(i, (int)floorf(x + eps)));
}

// Henyey-Greenstein phase function in FP32, 1 + g^2 - 2 g mu written as
// (1-g)^2 + 2 g (1-mu) (no cancellation near mu = 1); the hardware square
// root and reciprocal (each within 1 ulp) stand in for the correctly rounded
// ones, since the FP32 contribution carries ~1e-7 relative error anyway.
__device__ __forceinline__ float phase_hg_f32_om(const DevScene& s, float one_minus_mu)
{
    const float g = (float)s.g;
    const float d = (1.f - g) * (1.f - g) + 2.f * g * one_minus_mu;
    return (float)s.hg_num * __builtin_amdgcn_rcpf(d * __builtin_amdgcn_sqrtf(d));
}

__device__ __forceinline__ float phase_hg_f32(const DevScene& s, float mu) { return phase_hg_f32_om(s, 1.f - mu); }

// Factor of scatter vertex k (1 <= k < b) in the recycled contribution:
// albedo_ref(x_k) * f_s,t(x_k, mu_k) / f_s,ref(x_k, mu_k).
__device__ __forceinline__ double vertex_ratio(const DevScene& s, double bct, double bcr, double mu)
{
    const double hg = phase_hg(s, mu), ra = phase_rayleigh(mu);
    const double fst = fs_mix(s, bct, hg, ra), fsr = fs_mix(s, bcr, hg, ra);
    const double bsr = s.w_c * bcr + s.w_a * s.beta_air, btr = bcr + s.beta_air;
    return (bsr / btr) * (fst / fsr);
}

// Counter of this wavefront in a task-counter set.
__device__ __forceinline__ unsigned int task_counter()
{
    return (blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) % kTaskCounters;
}

// Next task for this wavefront from counter c (lane 0 takes it).
__device__ __forceinline__ unsigned int next_task(unsigned int* work, unsigned int c)
{
    unsigned int t = 0;
    if (threadIdx.x % kWave == 0) t = atomicAdd(work + c * kTaskStride, 1u);
    return __shfl(t, 0) * kTaskCounters + c;
}

__device__ __forceinline__ void flush_counts(unsigned long long* c, uint64_t seg, uint64_t le, uint64_t ovh)
{
    if (seg) atomicAdd(&c[0], (unsigned long long)seg);
    if (le) atomicAdd(&c[1], (unsigned long long)le);
    if (ovh) atomicAdd(&c[3], (unsigned long long)ovh);
}


}  // namespace trace
}  // namespace prt
