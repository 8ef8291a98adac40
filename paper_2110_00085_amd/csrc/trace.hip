// Hot path on stored paths: recycled rendering with local estimation
// (Sec. 5.2 + Sec. 3.4.3), the loss gradient through the tomography path
// score function (Sec. 4.4, App. C), and the correction-factor statistics.
//
// One lane per stored path; a wavefront holds a batch of 64 paths of
// (nearly) equal size B thanks to the sort, so lanes leave the scatter loop
// together.  The voxel walk runs in Real (float or double); projection,
// path weights and all tallies are FP64.  With FP32 traversal the factors of
// a stored contribution after the projection (phase function, transmittance,
// 1/r^2) and the gradient weights are FP32, as they are stored in FP32.
#include <algorithm>
#include <cmath>

#include "launch.hpp"
#include "trace_common.hpp"

namespace prt {

using namespace trace;

// ------------------------------------------------------------------ render


// Persistent launch: each workgroup of kBlock threads sets up its LDS (image
// tallies, extinction grid), then its wavefronts take (batch, camera group)
// tasks from a device counter, heaviest batches first.
constexpr int kBlock = 1024;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr size_t kLdsBudget = 128 * 1024;       // grids
constexpr int64_t kMaxGradSlabs = 8;            // LDS gradient slabs when each slab recomputes the weights
constexpr int64_t kMaxTapeGradSlabs = 64;       // LDS gradient slabs when the weights come from the tape
constexpr size_t kTapeImageLds = 64 * 1024;     // FP64 image of one camera, images formed from the tape
constexpr int kWalkLoads = 4;                   // pieces formed before their grid loads, grids in global memory
constexpr int kRenderWalkLoads = 4;             // the same for the render's connection walks

// The field beta_t - beta_ref for a persistent workgroup: formed in LDS from
// beta_t and beta_ref (kGridLds), else the one prepared in global memory.
template <typename Real, bool kGridLds>
__device__ __forceinline__ const Real* delta_grid(const TraceArgs& a, unsigned char* smem)
{
    if (!kGridLds) return (const Real*)a.grid_dlt;
    Real* sg = reinterpret_cast<Real*>(smem);
    const int nu = a.s.nx * a.s.ny * a.s.nz;
    lds_fill(sg, nu, [&](int i) { return (Real)((double)a.bc_t[i] - (double)a.st.beta_ref[i]); });
    __syncthreads();
    return sg;
}

bool delta_grid_lds(int fp64, int64_t nu) { return (size_t)nu * (fp64 ? 8 : 4) <= kLdsBudget; }

// Sum of the delta grid gd (from delta_grid) times length along a free-flight
// segment: one piece at a time in LDS, else kWalkLoads pieces per batch of
// loads from global memory, walked in byte offsets.
template <typename Real, bool kGridLds>
__device__ __forceinline__ Real delta_walk(const DevScene& s, const Real* gd, const Vtx& p0, const double w[3],
                                           double L, uint64_t& count)
{
    if constexpr (kGridLds) {
        return walk_sum<Real, true>(s, [&](uint32_t v) { return gd[v]; }, p0, w, L, count);
    } else {
        const unsigned char* g = reinterpret_cast<const unsigned char*>(gd);
        return walk_sum<Real, true, kWalkLoads, false, (int)sizeof(Real)>(
            s, [&](uint32_t off) { return *reinterpret_cast<const Real*>(g + off); }, p0, w, L, count);
    }
}

// Prefix weights, one wavefront per task (batch, b) with the field
// beta_t - beta_ref cached in LDS when it fits (persistent workgroups): a lane
// holds one path of the batch at its scatter b <= brender and stores
// q_b = base_b / base_{b-1} (base_0 = 1), where
// base_b = P_b / (beta_ref(x_b) + beta_air) with P_b = w0 prod_{k<b}
// exp(-(tau_t - tau_ref)(segment k)) prod_{1<=k<b} albedo_ref f_s,t / f_s,ref (x_k):
// every local estimate at x_b is base_b f_s,t(x_b, mu_bd) exp(-tau_t(connection)) / r^2,
// and the render forms base_b as the running product of q_1..q_b.  The
// factor of scatter b needs only the segment x_{b-1} -> x_b and the vertex
// x_{b-1}, so the segments of a path are walked by different wavefronts.
template <typename Real, bool kGridLds>
__global__ void __launch_bounds__(kBlock) render_prefix_kernel(TraceArgs a, VertexLevels lv)
{
    extern __shared__ unsigned char smem[];
    // the render kernel that follows takes its tasks from zeroed counters
    if (blockIdx.x == 0 && threadIdx.x < kTaskCounters) a.work[threadIdx.x * kTaskStride] = 0u;
    if (a.copy_beta) {
        const int nu_ = a.s.nx * a.s.ny * a.s.nz;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nu_; i += gridDim.x * blockDim.x)
            a.copy_beta[i] = a.bc_t[i];
    }
    const Real* gd = delta_grid<Real, kGridLds>(a, smem);
    const DevScene& s = a.s;
    const int nu = s.nx * s.ny * s.nz;
    const int64_t nb = a.st.n_slots / kWave;
    const int lane = threadIdx.x % kWave;
    const uint32_t waves = gridDim.x * kWavesPerBlock;
    uint64_t nseg = 0;
    int b = lv.bmax;
    for (uint32_t task = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; task < lv.total; task += waves) {
        // levels are contiguous task ranges in falling b (wavefront-uniform)
        while (task >= lv.start[b] + (uint32_t)(nb - lv.first_batch[b])) --b;
        const int64_t bt = lv.first_batch[b] + (int64_t)(task - lv.start[b]);
        const int64_t slot = bt * kWave + lane;
        if (b > min((int)a.st.B[slot], a.brender)) continue;
        const float4* __restrict__ V = a.st.vtx + a.st.batch_off[bt] + lane;
        const Vtx p0 = load_vtx(V, b - 1), p1 = load_vtx(V, b);
        double w[3];
        const double L = seg_dir(p0, p1, w);
        // free-flight segment b-1: transmittance ratio exp(-(tau_t - tau_ref))
        const Real dt = delta_walk<Real, kGridLds>(s, gd, p0, w, L, nseg);
        double q = exp(-(double)dt * s.vk);
        if (b == 1) {
            q *= s.w0;
        } else {
            // albedo_ref f_s,t / f_s,ref at x_{b-1} times base_{b-1}'s denominator
            const Vtx pm = load_vtx(V, b - 2);
            double wp[3];
            seg_dir(pm, p0, wp);
            const int v = clamp_vox(p0.v, nu);
            const double bct = (double)a.bc_t[v], bcr = (double)a.st.beta_ref[v];
            const double mu = wp[0] * w[0] + wp[1] * w[1] + wp[2] * w[2];
            const double hg = phase_hg(s, mu), ra = phase_rayleigh(mu);
            q *= (s.w_c * bcr + s.w_a * s.beta_air) * (fs_mix(s, bct, hg, ra) / fs_mix(s, bcr, hg, ra));
        }
        a.pbase[(a.st.batch_off[bt] - a.tape_base) + lane + (int64_t)b * kWave] =
            q / ((double)a.st.beta_ref[clamp_vox(p1.v, nu)] + s.beta_air);
    }
    flush_counts(a.counters, nseg, 0, 0);
}

// Persistent launch with the delta grid in LDS when it fits.
template <typename K, typename... Args>
static hipError_t launch_delta_kernel(hipStream_t st, K k, bool lds_grid, size_t grid_bytes, int n_wg,
                                      const Args&... args)
{
    const size_t lds = lds_grid ? grid_bytes : 0;
    if (lds) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k<<<dim3(n_wg), dim3(kBlock), lds, st>>>(args...);
    return hipGetLastError();
}

hipError_t launch_render_prefix(hipStream_t st, int fp64, const TraceArgs& a, const VertexLevels& lv, int n_cu)
{
    if (lv.total == 0) return hipSuccess;
    const size_t grid_bytes = (size_t)a.s.nx * a.s.ny * a.s.nz * (fp64 ? 8 : 4);
    const bool lds = grid_bytes <= kLdsBudget;
    const int n_wg = (int)std::max<int64_t>(
        1, std::min<int64_t>(((int64_t)lv.total + kWavesPerBlock - 1) / kWavesPerBlock, n_cu));
    if (fp64)
        return lds ? launch_delta_kernel(st, render_prefix_kernel<double, true>, true, grid_bytes, n_wg, a, lv)
                   : launch_delta_kernel(st, render_prefix_kernel<double, false>, false, grid_bytes, n_wg, a, lv);
    return lds ? launch_delta_kernel(st, render_prefix_kernel<float, true>, true, grid_bytes, n_wg, a, lv)
               : launch_delta_kernel(st, render_prefix_kernel<float, false>, false, grid_bytes, n_wg, a, lv);
}

// Local estimates from the stored paths.  Tasks are (batch, camera group),
// heaviest batches first; per scatter b the task reads base_b and, for every
// camera of its group, projects x_b, evaluates f_s,t and walks the
// connection for its transmittance.
// kGridLds: the total-extinction grid is cached in LDS.  kImg: with
// kImgGlobal every contribution is an FP64 atomic on the output image; with
// kImgFromTape there is no tally here (the images are formed from the tape
// afterwards, in FP64, which leaves the LDS to the grid).
// kTape: every contribution is recorded on the tape.
constexpr int kImgGlobal = 0, kImgFromTape = 2;

template <typename Real, bool kGridLds, int kImg, bool kTape>
__global__ void __launch_bounds__(kBlock) render_kernel(TraceArgs a, DevCams cams)
{
    extern __shared__ unsigned char smem[];
    const DevScene& s = a.s;
    const int nu = s.nx * s.ny * s.nz;
    const int npix = cams.W * cams.H;
    Real* __restrict__ sgrid = reinterpret_cast<Real*>(smem);
    // a grid in global memory is walked in its z-tiled copy: a walk's next
    // pieces share cache lines along z as well as x
    const Real* __restrict__ gtile = (const Real*)a.grid_tile;
    if (kGridLds) {
        lds_fill(sgrid, nu, [&](int i) { return (Real)((double)a.bc_t[i] + s.beta_air); });
        __syncthreads();
    }
    auto beta_tot = [&](uint32_t v) -> Real { return sgrid[v]; };
    // (the tiled copy is walked in byte offsets: no index arithmetic per piece)
    auto beta_tile = [&](uint32_t off) -> Real {
        return *reinterpret_cast<const Real*>(reinterpret_cast<const unsigned char*>(gtile) + off);
    };
    uint64_t nseg = 0, nle = 0;
    // the connection's optical depth (in grid units) from p1 along u up to tm;
    // with every camera outside the box the walk ends at the box boundary,
    // before the camera, so it needs no length bound
    auto walk_conn = [&](const Vtx& p1, const double u[3], double tm) -> Real {
        if constexpr (kGridLds) {
            return cams.outside ? walk_sum<Real, false>(s, beta_tot, p1, u, tm, nseg)
                                : walk_sum<Real, true>(s, beta_tot, p1, u, tm, nseg);
        } else {
            return cams.outside
                       ? walk_sum<Real, false, kRenderWalkLoads, true, (int)sizeof(Real)>(s, beta_tile, p1, u, tm, nseg)
                       : walk_sum<Real, true, kRenderWalkLoads, true, (int)sizeof(Real)>(s, beta_tile, p1, u, tm, nseg);
        }
    };
    const double r2scale = 1.0 / (s.vk * s.vk);
    const float vkf = (float)s.vk, wc_f = (float)s.w_c;
    const float wab = (float)(s.w_a * s.beta_air), ray_k = (float)(3.0 / (16.0 * kPi));
    const int lane = threadIdx.x % kWave;
    const int64_t nb = a.st.n_slots / kWave;
    const int G = a.groups, cpg = (cams.n + G - 1) / G;
    const unsigned int n_tasks = (unsigned int)(nb - a.st.first_slot / kWave) * (unsigned int)G;
    const unsigned int tc = task_counter();
    for (unsigned int task = next_task(a.work, tc); task < n_tasks; task = next_task(a.work, tc)) {
        const int64_t bt = nb - 1 - (int64_t)(task / G);
        const int g = (int)(task % G);
        const int d_lo = g * cpg, d_hi = min(cams.n, d_lo + cpg);
        const int64_t slot = bt * kWave + lane;
        const int Br = min((int)a.st.B[slot], a.brender);
        if (Br <= 0) continue;
        const float4* __restrict__ V = a.st.vtx + a.st.batch_off[bt] + lane;
        const double* __restrict__ Pb = a.pbase + (a.st.batch_off[bt] - a.tape_base) + lane;
        float2* __restrict__ T = kTape ? a.tape + (a.st.batch_off[bt] - a.tape_base) * cams.n + lane : nullptr;
        Vtx p0 = load_vtx(V, 0);
        double base = 1.0;
        for (int b = 1; b <= Br; ++b) {
            const Vtx p1 = load_vtx(V, b);
            double w[3];
            seg_dir(p0, p1, w);
            const int v1 = clamp_vox(p1.v, nu);
            const double bct = (double)a.bc_t[v1];
            base *= Pb[(int64_t)b * kWave];
            const float wcb = wc_f * (float)bct;
            for (int d = d_lo; d < d_hi; ++d) {
                const int pix = project(cams, d, p1.x, p1.y, p1.z, s.vk);
                if (pix < 0) {
                    if (kTape) T[(int64_t)(b * cams.n + d) * kWave] = make_float2(0.f, __int_as_float(-1));
                    continue;
                }
                const double ex = cams.pos[d][0] - p1.x, ey = cams.pos[d][1] - p1.y, ez = cams.pos[d][2] - p1.z;
                double c;
                if constexpr (sizeof(Real) == 4) {
                    // FP32 traversal: the contribution is kept in FP32 (tape), so
                    // the phase function, transmittance and 1/r^2 are
                    // FP32; the direction and 1 - mu stay FP64 (a forward-peaked
                    // phase function is sensitive to 1 - mu near mu = 1).
                    const double d2 = ex * ex + ey * ey + ez * ez;
                    double id = (double)rsqrtf((float)d2);
                    id = id * (1.5 - 0.5 * d2 * id * id);  // one Newton step: ~1e-14 relative
                    const double u[3] = {ex * id, ey * id, ez * id};
                    const double mu = w[0] * u[0] + w[1] * u[1] + w[2] * u[2];
                    const float muf = (float)mu;
                    const float hg = phase_hg_f32_om(s, (float)(1.0 - mu));
                    const float fst = wcb * hg + wab * ray_k * (1.f + muf * muf);
                    const Real tc = walk_conn(p1, u, d2 * id);
                    c = base * (double)(fst * expf(-(float)tc * vkf) * (float)(r2scale * id * id));
                } else {
                    const double dist2 = ex * ex + ey * ey + ez * ez;
                    const double dist = sqrt(dist2);
                    const double id = 1.0 / dist;
                    const double u[3] = {ex * id, ey * id, ez * id};
                    const double mu = w[0] * u[0] + w[1] * u[1] + w[2] * u[2];
                    const double fst = fs_mix(s, bct, phase_hg(s, mu), phase_rayleigh(mu));
                    const Real tc = walk_conn(p1, u, dist);
                    c = base * fst * exp(-(double)tc * s.vk) * (r2scale / dist2);
                }
                if (kTape) T[(int64_t)(b * cams.n + d) * kWave] = make_float2((float)c, __int_as_float(pix));
                if (kImg == kImgGlobal) unsafeAtomicAdd(&a.img[(int64_t)d * npix + pix], c);
                ++nle;
            }
            p0 = p1;
        }
    }
    flush_counts(a.counters, nseg, nle, 0);
}

// Exact pixel solid angle: F(x,y) = atan(xy / (f sqrt(x^2+y^2+f^2))) is the
// solid angle of [0,x]x[0,y] on the image plane at distance f.
__device__ __forceinline__ double pixel_solid_angle(double f, int W, int H, int row, int col)
{
    auto F = [f](double x, double y) { return atan(x * y / (f * sqrt(x * x + y * y + f * f))); };
    const double x1 = col - 0.5 * W, x2 = x1 + 1.0, y1 = row - 0.5 * H, y2 = y1 + 1.0;
    return F(x2, y2) - F(x1, y2) - F(x2, y1) + F(x1, y1);
}

// Factor turning pixel i's tally into radiance: scale / Omega_p.
__device__ __forceinline__ double pixel_scale(const DevCams& c, int64_t i, double scale)
{
    const int64_t npix = (int64_t)c.W * c.H;
    const int d = (int)(i / npix), p = (int)(i % npix);
    return scale / pixel_solid_angle(c.f[d], c.W, c.H, p / c.W, p % c.W);
}

template <typename Real, bool kGridLds, int kImg, bool kTape>
static hipError_t launch_render_t(hipStream_t st, const TraceArgs& a, const DevCams& c, int n_wg)
{
    const size_t nu = (size_t)a.s.nx * a.s.ny * a.s.nz;
    const size_t lds = kGridLds ? nu * sizeof(Real) : 0;
    if (lds) {
        hipError_t e = hipFuncSetAttribute((const void*)render_kernel<Real, kGridLds, kImg, kTape>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    render_kernel<Real, kGridLds, kImg, kTape><<<dim3(n_wg), dim3(kBlock), lds, st>>>(a, c);
    return hipGetLastError();
}

// Images from the tape: workgroup (x, d) adds the contributions c_{b,d} of
// every scatter of a strided share of the batches into an FP64 LDS image of
// camera d and writes it to partial[d][x]; tape_image_reduce_kernel adds the
// partials of each pixel in a fixed order.  The groups x are as many as fit
// the chip at once (kTapeImageBlocksPerCU workgroups per CU over all cameras),
// and a wavefront issues the tape loads of up to kTapeImageLoads scatters of
// its batch before it adds them, with the next batch's sizes already loading.
constexpr int kTapeImageBlocksPerCU = 2;
constexpr int kTapeImageLoads = 8;

int tape_image_groups(int n_cu, int n_cams)
{
    return std::max(1, kTapeImageBlocksPerCU * n_cu / std::max(1, n_cams));
}

__global__ void __launch_bounds__(kBlock) tape_image_kernel(TraceArgs a, DevCams cams, double* __restrict__ partial)
{
    extern __shared__ unsigned char smem[];
    double* __restrict__ simg = reinterpret_cast<double*>(smem);
    const int npix = cams.W * cams.H;
    const int d = blockIdx.y;
    for (int i = threadIdx.x; i < npix; i += blockDim.x) simg[i] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x % kWave;
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    const int64_t nb = a.st.n_slots / kWave;
    const int64_t stride = (int64_t)cams.n * kWave;
    int64_t bt = a.st.first_slot / kWave + (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    int Br = bt < nb ? min((int)a.st.B[bt * kWave + lane], a.brender) : 0;
    for (; bt < nb; bt += waves) {
        const int64_t btn = bt + waves;
        const int Bnext = btn < nb ? min((int)a.st.B[btn * kWave + lane], a.brender) : 0;
        const float2* __restrict__ T = a.tape + (a.st.batch_off[bt] - a.tape_base) * cams.n + d * kWave + lane;
        for (int b0 = 1; b0 <= Br; b0 += kTapeImageLoads) {
            float2 t[kTapeImageLoads];
#pragma unroll
            for (int j = 0; j < kTapeImageLoads; ++j)
                t[j] = b0 + j <= Br ? T[(int64_t)(b0 + j) * stride] : make_float2(0.f, __int_as_float(-1));
#pragma unroll
            for (int j = 0; j < kTapeImageLoads; ++j) {
                const int pix = __float_as_int(t[j].y);
                if (pix >= 0) atomicAdd(&simg[pix], (double)t[j].x);
            }
        }
        Br = Bnext;
    }
    __syncthreads();
    double* __restrict__ out = partial + ((int64_t)d * gridDim.x + blockIdx.x) * npix;
    for (int i = threadIdx.x; i < npix; i += blockDim.x) out[i] = simg[i];
}

__global__ void __launch_bounds__(256) tape_image_reduce_kernel(const double* __restrict__ partial, int groups,
                                                                int npix, int64_t n, DevCams c, double scale,
                                                                double* __restrict__ img)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t d = i / npix, p = i % npix;
    double acc = 0.0;
    // the groups in order, kTapeImageLoads loads in flight
    for (int x0 = 0; x0 < groups; x0 += kTapeImageLoads) {
        double t[kTapeImageLoads];
#pragma unroll
        for (int j = 0; j < kTapeImageLoads; ++j)
            t[j] = x0 + j < groups ? partial[(d * groups + x0 + j) * npix + p] : 0.0;
#pragma unroll
        for (int j = 0; j < kTapeImageLoads; ++j) acc += t[j];
    }
    img[i] = acc * pixel_scale(c, i, scale);
}

// Workgroups for a persistent launch over the batches that hold scattered paths.
static int persistent_groups(int64_t n_slots, int64_t first_slot, int n_cu, int per_cu)
{
    const int64_t batches = (n_slots - first_slot + kWave - 1) / kWave;
    const int64_t need = (batches + kWavesPerBlock - 1) / kWavesPerBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)n_cu * per_cu));
}

RenderPlan plan_render(int fp64, int64_t nu, const DevCams& c, bool tape, int64_t n_slots, int64_t first_slot,
                       int n_cu)
{
    RenderPlan p;
    const int64_t npix = (int64_t)c.W * c.H, nimg = npix * c.n;
    const int64_t grid_bytes = nu * (fp64 ? 8 : 4);
    if (tape && !fp64 && npix * 8 <= (int64_t)kTapeImageLds) {
        // images from the tape: the LDS holds only the grid
        p.img_tape = true;
        p.grid_lds = grid_bytes <= (int64_t)kLdsBudget;
        p.n_wg = persistent_groups(n_slots, first_slot, n_cu, p.grid_lds ? 1 : 2);
        p.img_groups = tape_image_groups(n_cu, c.n);
        p.partial_bytes = (size_t)nimg * p.img_groups * sizeof(double);
        return p;
    }
    // otherwise every contribution is an FP64 atomic on the output images
    p.grid_lds = grid_bytes <= (int64_t)kLdsBudget;
    p.n_wg = persistent_groups(n_slots, first_slot, n_cu, p.grid_lds ? 1 : 2);
    return p;
}

hipError_t launch_render(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c, const RenderPlan& p)
{
    if (a.st.n_slots - a.st.first_slot <= 0) return hipSuccess;
    if (fp64) {  // the all-FP64 mode records no FP32 tape
        if (p.grid_lds) return launch_render_t<double, true, kImgGlobal, false>(st, a, c, p.n_wg);
        return launch_render_t<double, false, kImgGlobal, false>(st, a, c, p.n_wg);
    }
    const bool tape = a.tape != nullptr;
    if (p.img_tape) {
        if (p.grid_lds) return launch_render_t<float, true, kImgFromTape, true>(st, a, c, p.n_wg);
        return launch_render_t<float, false, kImgFromTape, true>(st, a, c, p.n_wg);
    }
    if (p.grid_lds)
        return tape ? launch_render_t<float, true, kImgGlobal, true>(st, a, c, p.n_wg)
                    : launch_render_t<float, true, kImgGlobal, false>(st, a, c, p.n_wg);
    return tape ? launch_render_t<float, false, kImgGlobal, true>(st, a, c, p.n_wg)
                : launch_render_t<float, false, kImgGlobal, false>(st, a, c, p.n_wg);
}

hipError_t launch_render_reduce(hipStream_t st, const TraceArgs& a, const DevCams& c, const RenderPlan& p,
                                const void* partial, double scale, double* img)
{
    const int64_t npix = (int64_t)c.W * c.H, nimg = npix * c.n;
    const unsigned blocks = (unsigned)((nimg + 255) / 256);
    if (!p.img_tape) return hipSuccess;
    {
        const size_t lds = (size_t)npix * sizeof(double);
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void*)tape_image_kernel,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        tape_image_kernel<<<dim3(p.img_groups, c.n), dim3(kBlock), lds, st>>>(a, c, (double*)partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        tape_image_reduce_kernel<<<dim3(blocks), dim3(256), 0, st>>>((const double*)partial, p.img_groups,
                                                                      (int)npix, nimg, c, scale, img);
        return hipGetLastError();
    }
}



// images = tallies / (N Omega_p)
__global__ void __launch_bounds__(256) render_finalize_kernel(double* __restrict__ img, DevCams c, double scale)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npix = (int64_t)c.W * c.H;
    if (i >= npix * c.n) return;
    img[i] *= pixel_scale(c, i, scale);
}

hipError_t launch_render_finalize(hipStream_t st, double* img, const DevCams& c, double scale)
{
    const int64_t n = (int64_t)c.W * c.H * c.n;
    render_finalize_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(img, c, scale);
    return hipGetLastError();
}

// rho = residual / (N Omega_p)
__global__ void __launch_bounds__(256) grad_prep_kernel(const double* __restrict__ res, double* __restrict__ rho,
                                                        DevCams c, double scale, int* __restrict__ flag,
                                                        unsigned int* __restrict__ work)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && flag) *flag = 1;
    if (i < 2 * kTaskCounters) work[(i / 2) * kTaskStride + i % 2] = 0u;
    if (i == 0) work[kBinChunkWord] = 0u;
    const int64_t npix = (int64_t)c.W * c.H;
    if (i >= npix * c.n) return;
    rho[i] = res[i] * pixel_scale(c, i, scale);
}

hipError_t launch_grad_prep(hipStream_t st, const double* residual, double* rho, const DevCams& c, double scale,
                            int* flag, unsigned int* work)
{
    const int64_t n = std::max<int64_t>((int64_t)c.W * c.H * c.n, 2 * kTaskCounters);
    grad_prep_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(residual, rho, c, scale, flag, work);
    return hipGetLastError();
}

// -------------------------------------------------------------------- grad

// The gradient is sum_{b,d} w_{b,d} S(b,d), with w = c rho_{d,p} and S the
// tomography PSF of the local-estimate sub-path (Sec. 4.4, App. C): -l in
// every voxel of the sub-path's segments and connection, plus the vertex
// terms at its scatters.  Summing over d first gives R_b = sum_d w_{b,d};
// free-flight segment k is then shared by every estimate at a later vertex,
// so it takes -A_k l with A_k = sum_{b>k} R_b, and the scatter at x_k takes
// A_k times its vertex term.
//
// Tally: one launch covers the slab of z layers [z0, z1) and adds only the
// score terms of voxels in it (the walks are clipped to the slab).  With
// kLds the workgroup accumulates the slab in LDS in FP64 (LDS FP64 adds are
// several times faster than FP32 ones on this chip) and writes its partial
// sums to partial[blockIdx.x][v]; a second kernel adds the partials in a
// fixed order.  Without kLds the launch covers all layers and every update
// is an FP64 atomic on the output.

// Slab tally: sg in LDS (kLds) or the output gradient, numbered inside the slab.
template <bool kLds>
struct SlabTally {
    double* __restrict__ out;
    int vlo, nsv;
    __device__ __forceinline__ void add(uint32_t v, double x) const
    {
        if (kLds) atomicAdd(&out[v], x);
        else unsafeAtomicAdd(&out[v], x);
    }
    // v is a grid voxel, added only when it lies in the slab
    __device__ __forceinline__ void add_vox(int v, double x) const
    {
        const int u = v - vlo;
        if ((unsigned)u < (unsigned)nsv) add((uint32_t)u, x);
    }
};

template <bool kLds>
__device__ __forceinline__ SlabTally<kLds> slab_tally_begin(const TraceArgs& a, int z0, int z1, unsigned char* smem)
{
    const int layer = a.s.nx * a.s.ny;
    SlabTally<kLds> t;
    t.vlo = z0 * layer;
    t.nsv = (z1 - z0) * layer;
    if (kLds) {
        t.out = reinterpret_cast<double*>(smem);
        for (int i = threadIdx.x; i < t.nsv; i += kBlock) t.out[i] = 0.0;
        __syncthreads();
    } else {
        t.out = a.grad + t.vlo;
    }
    return t;
}

template <bool kLds>
__device__ __forceinline__ void slab_tally_end(const SlabTally<kLds>& t, double* __restrict__ partial)
{
    if (!kLds) return;
    __syncthreads();
    double* __restrict__ out = partial + (int64_t)blockIdx.x * t.nsv;
    for (int i = threadIdx.x; i < t.nsv; i += kBlock) out[i] = t.out[i];
}

// Weights from the transmittance tape, one wavefront per task (batch, b): a
// lane holds one path of the batch at its scatter b and writes, for every
// camera d, w_{b,d} = c_{b,d} rho_{d,p} with c and the pixel p from the tape
// (0 when x_b projects outside camera d), and for the vertex R_b, the
// connection vertex term sum_d w_{b,d} w_c f_HG / f_s,t at x_b, and the
// coefficient w_c f_HG / f_s,t of the scatter at x_b between segments b-1 and
// b.  The vertices of a path are independent here, so a path's vertices go to
// different wavefronts and their loads overlap.  Runs only when the tape
// matches beta_t (FP32 traversal mode): the per-camera phase functions are
// evaluated in FP32, like the stored weights.

constexpr int kGwCams = 5;
// cameras per camera group: at most 3 groups of the kMaxCams cameras
constexpr int kGroupCams = (kMaxCams + 2) / 3;
constexpr int kGwBlock = 256;
constexpr int kGwBlocksPerCU = 8;

__global__ void __launch_bounds__(kGwBlock) grad_weights_kernel(TraceArgs a, DevCams cams, VertexLevels lv)
{
    if (*a.tape_flag == 0) return;
    __shared__ unsigned long long wg_le;
    if (threadIdx.x == 0) wg_le = 0;
    __syncthreads();
    const DevScene& s = a.s;
    const int nu = s.nx * s.ny * s.nz;
    const int npix = cams.W * cams.H;
    const int64_t nb = a.st.n_slots / kWave;
    const int lane = threadIdx.x % kWave;
    const uint32_t waves = gridDim.x * (kGwBlock / kWave);
    const float wc = (float)s.w_c, wab = (float)(s.w_a * s.beta_air), ray_k = (float)(3.0 / (16.0 * kPi));
    uint64_t nle = 0;
    int b = lv.bmax;
    for (uint32_t task = blockIdx.x * (kGwBlock / kWave) + threadIdx.x / kWave; task < lv.total; task += waves) {
        // levels are contiguous task ranges in falling b (wavefront-uniform)
        while (task >= lv.start[b] + (uint32_t)(nb - lv.first_batch[b])) --b;
        // the batch index is wavefront-uniform: its offsets come from scalar loads
        const int64_t bt = __builtin_amdgcn_readfirstlane((int)(lv.first_batch[b] + (int64_t)(task - lv.start[b])));
        const int64_t slot = bt * kWave + lane;
        const int64_t rec0 = a.st.batch_off[bt] - a.tape_base;
        const float4* __restrict__ V = a.st.vtx + a.st.batch_off[bt] + lane;
        const float2* __restrict__ Tp = a.tape + rec0 * cams.n + lane;
        float* __restrict__ Wp = a.wtape + rec0 * cams.n + lane;
        // Rows b-1 and b of the vertices and row b of the tape exist for every
        // lane of a batch on level b (some lane has B >= b), so they load
        // together with the lane's B; a lane with B < b computes on its padding
        // or stale rows and neither gathers nor stores.
        const Vtx p0 = load_vtx(V, b - 1), p1 = load_vtx(V, b);
        const int Bn = (int)a.st.B[slot];
        const bool act = b <= Bn;
        // binned gradient: layers along the slab axis reached by the walks of
        // this (batch, b), per camera group and for segment b-1
        const bool bins = a.trange != nullptr;
        const int ax = a.bin_axis;
        const int G = a.groups, cpg = (cams.n + G - 1) / G;
        const float p1a = (float)(ax == 0 ? p1.x : (ax == 1 ? p1.y : p1.z));
        int p1i;
        {
            int i0, i1, i2;
            voxel_ijk(s, clamp_vox(p1.v, nu), i0, i1, i2);
            p1i = ax == 0 ? i0 : (ax == 1 ? i1 : i2);
        }
        const float nbox[3] = {(float)s.nx, (float)s.ny, (float)s.nz};
        // ranges of the camera groups (at most 3) and of the segment walk,
        // updated by selects so that they stay in registers
        int rlo[4] = {kNoLayer, kNoLayer, kNoLayer, kNoLayer}, rhi[4] = {-1, -1, -1, -1};
        // tape records of kGwCams cameras from d0 on, one group ahead of its
        // arithmetic (a camera index past the last loads the last camera's
        // record, in bounds and without a branch, and is masked below)
        float2 tn[kGwCams];
        auto load_group = [&](int d0) {
#pragma unroll
            for (int j = 0; j < kGwCams; ++j) tn[j] = Tp[(int64_t)(b * cams.n + min(d0 + j, cams.n - 1)) * kWave];
        };
        load_group(0);
        double w[3];
        seg_dir(p0, p1, w);
        const int v1 = clamp_vox(p1.v, nu);
        const double bct = (double)a.bc_t[v1];
        const float wcb = wc * (float)bct;
        const float wf0 = (float)w[0], wf1 = (float)w[1], wf2 = (float)w[2];
        float Rb = 0.f, vert = 0.f;
        // cameras in groups of kGwCams: all tape loads of a group, then all
        // residual gathers, then the arithmetic, so the loads overlap
        for (int d0 = 0; d0 < cams.n; d0 += kGwCams) {
            float2 tt[kGwCams];
            double rr[kGwCams];
#pragma unroll
            for (int j = 0; j < kGwCams; ++j) tt[j] = tn[j];
            if (d0 + kGwCams < cams.n) load_group(d0 + kGwCams);
#pragma unroll
            for (int j = 0; j < kGwCams; ++j) {
                if (!act || d0 + j >= cams.n) tt[j].y = __int_as_float(-1);
                const int pix = __float_as_int(tt[j].y);
                rr[j] = pix >= 0 ? a.rho[(int64_t)(d0 + j) * npix + pix] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < kGwCams; ++j) {
                const int d = d0 + j;
                if (d >= cams.n) break;
                const int pix = __float_as_int(tt[j].y);
                float wf = 0.f;
                if (pix >= 0) {
                    wf = tt[j].x * (float)rr[j];
                    const float ex = (float)(cams.pos[d][0] - p1.x), ey = (float)(cams.pos[d][1] - p1.y),
                                ez = (float)(cams.pos[d][2] - p1.z);
                    static_assert(kMaxBinSlabs <= 255, "slab ranges pack two 8-bit slab indices");
                    uint16_t rpack = 0xffffu;
                    if (bins && wf != 0.f) {
                        // the connection runs from x_b to where it leaves the box
                        // (or reaches the camera): parameter t in [0, 1] along e
                        const float e[3] = {ex, ey, ez};
                        const float q[3] = {(float)p1.x, (float)p1.y, (float)p1.z};
                        float tend = 1.f;
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            if (e[k] != 0.f) tend = fminf(tend, ((e[k] > 0.f ? nbox[k] : 0.f) - q[k]) / e[k]);
                        tend = fmaxf(tend, 0.f);
                        const float ea = ax == 0 ? ex : (ax == 1 ? ey : ez);
                        int lo = kNoLayer, hi = -1;
                        layer_span(p1a, p1i, lo, hi);
                        layer_span(p1a + tend * ea, p1i, lo, hi);
                        const int gi = d / cpg;
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            rlo[k] = gi == k ? min(rlo[k], lo) : rlo[k];
                            rhi[k] = gi == k ? max(rhi[k], hi) : rhi[k];
                        }
                        const int na = ax == 0 ? s.nx : (ax == 1 ? s.ny : s.nz);
                        rpack = (uint16_t)((max(lo, 0) / a.bin_layers) | (min(hi, na - 1) / a.bin_layers) << 8);
                    }
                    if (bins && act) a.rtape[rec0 * cams.n + lane + (int64_t)(b * cams.n + d) * kWave] = rpack;
                    const float mu = (wf0 * ex + wf1 * ey + wf2 * ez) * rsqrtf(ex * ex + ey * ey + ez * ez);
                    const float hg = phase_hg_f32(s, mu);
                    const float fst = wcb * hg + wab * ray_k * (1.f + mu * mu);
                    Rb += wf;
                    if (fst > 0.f) vert += wf * (wc * hg / fst);
                    ++nle;
                }
                if (act) Wp[(int64_t)(b * cams.n + d) * kWave] = wf;
                if (bins && act && pix < 0) a.rtape[rec0 * cams.n + lane + (int64_t)(b * cams.n + d) * kWave] = 0xffffu;
            }
        }
        if (bins) {
            int slo = kNoLayer, shi = -1;
            if (act) {
                // segment b-1 of the free-flight walk
                int i0, i1, i2;
                voxel_ijk(s, clamp_vox(p0.v, nu), i0, i1, i2);
                const float p0a = (float)(ax == 0 ? p0.x : (ax == 1 ? p0.y : p0.z));
                layer_span(p0a, ax == 0 ? i0 : (ax == 1 ? i1 : i2), slo, shi);
                layer_span(p1a, p1i, slo, shi);
            }
            // wavefront minimum and maximum, then one atomic pair per kind
            const int nsl = (a.st.n_slots / kWave), kinds = G + 1;
            const int na = ax == 0 ? s.nx : (ax == 1 ? s.ny : s.nz);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k >= kinds) break;
                int lo = k == G ? slo : rlo[k], hi = k == G ? shi : rhi[k];
                for (int o = kWave / 2; o > 0; o >>= 1) {
                    lo = min(lo, __shfl_xor(lo, o));
                    hi = max(hi, __shfl_xor(hi, o));
                }
                if (lane == 0 && lo <= hi) {
                    const int64_t t = (int64_t)(nsl - 1 - bt) * kinds + k;
                    atomicMin(&a.trange[2 * t], max(lo, 0) / a.bin_layers);
                    atomicMax(&a.trange[2 * t + 1], min(hi, na - 1) / a.bin_layers);
                }
                if (lane == 0 && k < G)
                    a.brange[((rec0 >> 6) + b) * G + k] =
                        lo <= hi ? (uint32_t)(max(lo, 0) / a.bin_layers) |
                                       (uint32_t)(min(hi, na - 1) / a.bin_layers) << 16
                                 : 0xffffu;
            }
        }
        if (!act) continue;
        // the scatter at x_b turns segment b-1 (direction w) into segment b
        double coef = 0.0;
        if (b < Bn) {
            const Vtx p2 = load_vtx(V, b + 1);
            double wn[3];
            seg_dir(p1, p2, wn);
            const double mu = w[0] * wn[0] + w[1] * wn[1] + w[2] * wn[2];
            const double hg = phase_hg(s, mu);
            const double fst = fs_mix(s, bct, hg, phase_rayleigh(mu));
            if (fst > 0.0) coef = s.w_c * hg / fst;
        }
        a.vaux[rec0 + lane + (int64_t)b * kWave] = make_float4(Rb, vert, (float)coef, 0.f);
    }
    // one counter update per workgroup
    if (nle) atomicAdd(&wg_le, (unsigned long long)nle);
    __syncthreads();
    if (threadIdx.x == 0 && wg_le) atomicAdd(&a.counters[1], wg_le);
}

hipError_t launch_grad_weights(hipStream_t st, const TraceArgs& a, const DevCams& c, const VertexLevels& lv, int n_cu)
{
    if (lv.total == 0) return hipSuccess;
    const uint32_t per_wg = kGwBlock / kWave;
    const int64_t blocks = std::min<int64_t>(((int64_t)lv.total + per_wg - 1) / per_wg, (int64_t)n_cu * kGwBlocksPerCU);
    grad_weights_kernel<<<dim3((unsigned)blocks), dim3(kGwBlock), 0, st>>>(a, c, lv);
    return hipGetLastError();
}

// Walks on the stored weights (tape case).  Tasks are (batch, kind), heaviest
// batches first: kind g < groups walks the connections of camera group g
// (kind 0 also adds the connection vertex terms), kind == groups walks the
// free-flight segments with the suffix sums A_k and adds their vertex terms.
template <bool kLds>
__global__ void __launch_bounds__(kBlock) grad_walk_kernel(TraceArgs a, DevCams cams, int z0, int z1,
                                                           double* __restrict__ partial)
{
    if (*a.tape_flag == 0) return;
    extern __shared__ unsigned char smem[];
    const SlabTally<kLds> tally = slab_tally_begin<kLds>(a, z0, z1, smem);
    auto add = [&](uint32_t v, double x) { tally.add(v, x); };
    const DevScene& s = a.s;
    const int nu = s.nx * s.ny * s.nz;
    const int lane = threadIdx.x % kWave;
    const int64_t nb = a.st.n_slots / kWave;
    const int G = a.groups, K = G + 1, cpg = (cams.n + G - 1) / G;
    const unsigned int n_tasks = (unsigned int)(nb - a.st.first_slot / kWave) * (unsigned int)K;
    uint64_t nseg = 0;
    const unsigned int tc = task_counter();
    for (unsigned int task = next_task(a.work, tc); task < n_tasks; task = next_task(a.work, tc)) {
        const int64_t bt = nb - 1 - (int64_t)(task / K);
        const int kind = (int)(task % K);
        const int64_t slot = bt * kWave + lane;
        const int Bn = (int)a.st.B[slot];
        if (Bn <= 0) continue;
        const int64_t rec0 = a.st.batch_off[bt] - a.tape_base;
        const float4* __restrict__ V = a.st.vtx + a.st.batch_off[bt] + lane;
        const float4* __restrict__ X = a.vaux + rec0 + lane;
        if (kind < G) {
            const int d_lo = kind * cpg, nd = min(cams.n, d_lo + cpg) - d_lo;
            const float* __restrict__ Wp = a.wtape + rec0 * cams.n + d_lo * kWave + lane;
            // the vertex and the group's weights of scatter b+1 load while
            // scatter b walks
            Vtx pn = load_vtx(V, 1);
            float wn[kGroupCams];
#pragma unroll
            for (int j = 0; j < kGroupCams; ++j) wn[j] = j < nd ? Wp[(int64_t)(cams.n + j) * kWave] : 0.f;
            for (int b = 1; b <= Bn; ++b) {
                const Vtx p1 = pn;
                float wc[kGroupCams];
#pragma unroll
                for (int j = 0; j < kGroupCams; ++j) wc[j] = wn[j];
                if (b < Bn) {
                    pn = load_vtx(V, b + 1);
#pragma unroll
                    for (int j = 0; j < kGroupCams; ++j)
                        wn[j] = j < nd ? Wp[(int64_t)((b + 1) * cams.n + j) * kWave] : 0.f;
                }
                for (int j = 0; j < nd; ++j) {
                    const int d = d_lo + j;
                    const double wgt = (double)wc[j];
                    if (wgt == 0.0) continue;
                    // the walk runs in FP32: its direction and length are formed in
                    // FP32 from the FP64 offset (hardware reciprocal square root)
                    const float ex = (float)(cams.pos[d][0] - p1.x), ey = (float)(cams.pos[d][1] - p1.y),
                                ez = (float)(cams.pos[d][2] - p1.z);
                    const float d2 = ex * ex + ey * ey + ez * ez;
                    const float id = __builtin_amdgcn_rsqf(d2);
                    const double u[3] = {(double)(ex * id), (double)(ey * id), (double)(ez * id)};
                    const double dist = (double)(d2 * id);
                    if (cams.outside)
                        walk_scatter<float, false>(s, add, p1, u, dist, -wgt * s.vk, nseg, z0, z1);
                    else
                        walk_scatter<float>(s, add, p1, u, dist, -wgt * s.vk, nseg, z0, z1);
                }
                if (kind == 0) {
                    const double vert = (double)X[(int64_t)b * kWave].y;
                    if (vert != 0.0) tally.add_vox(clamp_vox(p1.v, nu), vert);
                }
            }
        } else {
            double A = 0.0;
            Vtx pk1 = load_vtx(V, Bn);
            for (int k = Bn - 1; k >= 0; --k) {
                A += (double)X[(int64_t)(k + 1) * kWave].x;
                const Vtx pk = load_vtx(V, k);
                double w[3];
                const double L = seg_dir(pk, pk1, w);
                if (A != 0.0) {
                    walk_scatter<float>(s, add, pk, w, L, -A * s.vk, nseg, z0, z1);
                    if (k >= 1) tally.add_vox(clamp_vox(pk.v, nu), A * (double)X[(int64_t)k * kWave].z);
                }
                pk1 = pk;
            }
        }
    }
    flush_counts(a.counters, nseg, 0, 0);
    slab_tally_end<kLds>(tally, partial);
}

// ------------------------------------------------------- binned gradient
//
// The walks on the stored weights again, without repeating every walk once
// per slab: each gradient task (batch, kind) carries the range of slabs its
// walks reach (set by the weights kernel); the tasks are listed slab after
// slab, and one persistent launch takes chunks of that list.  A workgroup
// tallies the slab of its chunk in LDS in FP64, walking each listed task
// clipped to the slab, and writes the slab's sums as the chunk's partial; a
// second kernel adds, for every voxel, the partials of its slab's chunks in
// chunk order.  Every voxel piece of a walk lies in exactly one slab.

constexpr int kBinChunksPerWg = 16;  // chunks of the list per workgroup (load balance)
constexpr int kBinMinChunk = 64;    // smallest chunk (each chunk zeroes and writes out a slab)
constexpr int kBinReduceLoads = 8;
constexpr int kBinQueue = 128;      // per-wavefront queue of connection walks (power of two, >= 2 * 64)

// trange = empty ranges, grad = 0.
__global__ void __launch_bounds__(256) grad_bin_init_kernel(int* __restrict__ trange, int64_t n_tasks,
                                                            double* __restrict__ grad, int64_t nu)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_tasks) {
        trange[2 * i] = kNoLayer;
        trange[2 * i + 1] = -1;
    }
    if (i < nu) grad[i] = 0.0;
}

// cnt[s * n_blocks + block] = tasks of the block whose range holds slab s.
__global__ void __launch_bounds__(kBinTasks) grad_bin_count_kernel(const int* __restrict__ trange, GradBins g,
                                                                   const int* __restrict__ flag)
{
    if (*flag == 0) return;
    __shared__ unsigned int hist[kMaxBinSlabs];
    for (int i = threadIdx.x; i < g.n_slabs; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kBinTasks + threadIdx.x;
    if (t < g.n_tasks) {
        const int lo = trange[2 * t], hi = trange[2 * t + 1];
        for (int s = lo; s <= hi; ++s) atomicAdd(&hist[s], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < g.n_slabs; i += blockDim.x) g.cnt[(int64_t)i * g.n_blocks + blockIdx.x] = hist[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) g.cnt[(int64_t)g.n_slabs * g.n_blocks] = 0u;
}

// After the scan: every task is written to the list of each slab of its range.
__global__ void __launch_bounds__(kBinTasks) grad_bin_fill_kernel(const int* __restrict__ trange, GradBins g,
                                                                  const int* __restrict__ flag)
{
    if (*flag == 0) return;
    __shared__ unsigned int cur[kMaxBinSlabs];
    for (int i = threadIdx.x; i < g.n_slabs; i += blockDim.x) cur[i] = g.cnt[(int64_t)i * g.n_blocks + blockIdx.x];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * kBinTasks + threadIdx.x;
    if (t < g.n_tasks) {
        const int lo = trange[2 * t], hi = trange[2 * t + 1];
        for (int s = lo; s <= hi; ++s) {
            const unsigned int pos = atomicAdd(&cur[s], 1u);
            if ((int64_t)pos < g.list_cap) g.list[pos] = (uint32_t)t;
        }
    }
}

// One listed task of slab box b: the walks of kind `kind` of batch bt,
// clipped to the block, added to the LDS tally.
__device__ __forceinline__ void grad_bin_task(const TraceArgs& a, const DevCams& cams, const double* cpos,
                                              const SubBox& box, int slab, double* __restrict__ tally,
                                              uint32_t* queue, int64_t bt, int kind, uint64_t& nseg)
{
    const DevScene& s = a.s;
    const int nu = s.nx * s.ny * s.nz;
    const int lane = threadIdx.x % kWave;
    const int G = a.groups, cpg = (cams.n + G - 1) / G;
    const int64_t slot = bt * kWave + lane;
    const int Bn = (int)a.st.B[slot];
    // (lanes without scatters stay: the connection walks are shared across lanes)
    if (kind >= G && Bn <= 0) return;
    auto add = [&](uint32_t v, double x) { atomicAdd(&tally[v], x); };
    const LdsTally lt(tally, box);
    const int64_t rec0 = a.st.batch_off[bt] - a.tape_base;
    const float4* __restrict__ V = a.st.vtx + a.st.batch_off[bt] + lane;
    const float4* __restrict__ X = a.vaux + rec0 + lane;
    if (kind < G) {
        // connections: every lane tests its (scatter, camera) walks against
        // the slab (range tape), the hits are queued in LDS, and 64 queued
        // walks at a time are walked, one per lane
        const int d_lo = kind * cpg, nd = min(cams.n, d_lo + cpg) - d_lo;
        const uint16_t* __restrict__ Rp = a.rtape + rec0 * cams.n + d_lo * kWave + lane;
        const float4* __restrict__ Vb = a.st.vtx + a.st.batch_off[bt];
        const float* __restrict__ Wb = a.wtape + rec0 * cams.n + d_lo * kWave;
        const uint32_t sl = (uint32_t)slab;
        uint32_t wq = 0, rq = 0;
        // (the camera positions come from LDS: lanes index them by their own
        // queued camera)
        auto walk_entry = [&](uint32_t e) {
            const int L = (int)(e & 63u), b = (int)((e >> 6) & 127u), j = (int)(e >> 13);
            const float4 r = Vb[(int64_t)b * kWave + L];
            const double wgt = (double)Wb[(int64_t)(b * cams.n + j) * kWave + L];
            const double* c = cpos + 3 * (d_lo + j);
            const float ex = (float)(c[0] - (double)r.x), ey = (float)(c[1] - (double)r.y),
                        ez = (float)(c[2] - (double)r.z);
            const float d2 = ex * ex + ey * ey + ez * ez;
            const float id = __builtin_amdgcn_rsqf(d2);
            if (cams.outside)
                walk_tally_box_f<false>(s, lt, r.x, r.y, r.z, vox_of(r), ex * id, ey * id, ez * id, d2 * id,
                                        -wgt * s.vk, nseg);
            else
                walk_tally_box_f(s, lt, r.x, r.y, r.z, vox_of(r), ex * id, ey * id, ez * id, d2 * id, -wgt * s.vk,
                                 nseg);
        };
        int bmax = Bn;
        for (int o = kWave / 2; o > 0; o >>= 1) bmax = max(bmax, __shfl_xor(bmax, o));
        // the union of a row's ranges skips rows without a walk in this slab
        // (their vertex terms are zero too: a vertex term comes with a
        // weighted connection, whose range holds the vertex's own layer)
        const uint32_t* __restrict__ BR = a.brange + (rec0 >> 6) * G + kind;
        for (int b = 1; b <= bmax; ++b) {
            const uint32_t br = BR[(int64_t)b * G];
            if (sl < (br & 0xffffu) || sl > (br >> 16)) continue;
            uint32_t rr[kGroupCams];
#pragma unroll
            for (int j = 0; j < kGroupCams; ++j)
                rr[j] = (j < nd && b <= Bn) ? (uint32_t)Rp[(int64_t)(b * cams.n + j) * kWave] : 0xffffu;
#pragma unroll
            for (int j = 0; j < kGroupCams; ++j) {
                const bool hit = (rr[j] & 0xffu) <= sl && sl <= (rr[j] >> 8);
                const uint64_t m = __ballot(hit);
                if (hit) {
                    const uint32_t pos = wq + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    queue[pos & (kBinQueue - 1)] = (uint32_t)lane | (uint32_t)b << 6 | (uint32_t)j << 13;
                }
                wq += (uint32_t)__popcll(m);
                if (wq - rq >= (uint32_t)kWave) {
                    __builtin_amdgcn_wave_barrier();
                    walk_entry(queue[(rq + lane) & (kBinQueue - 1)]);
                    rq += kWave;
                }
            }
            if (kind == 0 && b <= Bn) {
                const double vert = (double)X[(int64_t)b * kWave].y;
                const int u = vert != 0.0 ? box_index(box, clamp_vox(vox_of(V[(int64_t)b * kWave]), nu), s) : -1;
                if (u >= 0) add((uint32_t)u, vert);
            }
        }
        if (wq > rq) {
            __builtin_amdgcn_wave_barrier();
            if ((uint32_t)lane < wq - rq) walk_entry(queue[(rq + lane) & (kBinQueue - 1)]);
        }
    } else {
        // a segment whose bounding box (widened by a voxel: a walk starts in
        // its stored voxel, which rounding can put next to the position's)
        // misses the block has no piece in it, and its start vertex no term:
        // both are skipped before the direction is formed
        auto near = [&](double lo, double hi, int a) { return hi >= (double)box.lo[a] - 1.0 && lo <= (double)box.hi[a] + 1.0; };
        double A = 0.0;
        Vtx pk1 = load_vtx(V, Bn);
        for (int k = Bn - 1; k >= 0; --k) {
            A += (double)X[(int64_t)(k + 1) * kWave].x;
            const Vtx pk = load_vtx(V, k);
            const bool seg_near = near(fmin(pk.x, pk1.x), fmax(pk.x, pk1.x), 0) &&
                                  near(fmin(pk.y, pk1.y), fmax(pk.y, pk1.y), 1) &&
                                  near(fmin(pk.z, pk1.z), fmax(pk.z, pk1.z), 2);
            if (A != 0.0 && seg_near) {
                double w[3];
                const double L = seg_dir(pk, pk1, w);
                walk_tally_box_f(s, lt, (float)pk.x, (float)pk.y, (float)pk.z, pk.v, (float)w[0], (float)w[1],
                                 (float)w[2], (float)L, -A * s.vk, nseg);
                const int u = k >= 1 ? box_index(box, clamp_vox(pk.v, nu), s) : -1;
                if (u >= 0) add((uint32_t)u, A * (double)X[(int64_t)k * kWave].z);
            }
            pk1 = pk;
        }
    }
}

// Chunks of the slab lists: chunk size C = max(kBinMinChunk, total / (chunks
// per workgroup * workgroups)); slab s holds chunks [chunks[s], chunks[s+1]),
// chunks[n_slabs] = their number, chunks[n_slabs+1] = C.  One workgroup.
__global__ void __launch_bounds__(256) grad_bin_chunks_kernel(GradBins g, int n_wg, const int* __restrict__ flag)
{
    if (*flag == 0) return;
    if (threadIdx.x != 0) return;
    const uint32_t total = g.cnt[(int64_t)g.n_slabs * g.n_blocks];
    const uint32_t want = (uint32_t)kBinChunksPerWg * (uint32_t)n_wg;
    const uint32_t C = max((uint32_t)kBinMinChunk, (total + want - 1) / want);
    uint32_t k = 0;
    for (int s = 0; s < g.n_slabs; ++s) {
        g.chunks[s] = k;
        const uint32_t a0 = g.cnt[(int64_t)s * g.n_blocks];
        const uint32_t a1 = s + 1 < g.n_slabs ? g.cnt[(int64_t)(s + 1) * g.n_blocks] : total;
        k += (a1 - a0 + C - 1) / C;
    }
    g.chunks[g.n_slabs] = k;
    g.chunks[g.n_slabs + 1] = C;
}

// Persistent: a workgroup takes chunk c of slab s, tallies its tasks' walks
// clipped to the slab in LDS (FP64) and writes the slab's sums to
// partial[c * slab_voxels + i].
__global__ void __launch_bounds__(kBlock) grad_bin_walk_kernel(TraceArgs a, DevCams cams, GradBins g)
{
    if (*a.tape_flag == 0) return;
    extern __shared__ unsigned char smem[];
    double* __restrict__ tally = reinterpret_cast<double*>(smem);
    __shared__ unsigned int s_chunk, s_item;
    __shared__ uint32_t wave_queue[kWavesPerBlock][kBinQueue];
    __shared__ double cpos[3 * kMaxCams];
    for (int i = threadIdx.x; i < 3 * cams.n; i += kBlock) cpos[i] = cams.pos[i / 3][i % 3];
    const DevScene& s = a.s;
    const int per_layer = g.axis == 0 ? s.ny * s.nz : (g.axis == 1 ? s.nx * s.nz : s.nx * s.ny);
    const int64_t nb = a.st.n_slots / kWave;
    const int kinds = a.groups + 1;
    const uint32_t total = g.cnt[(int64_t)g.n_slabs * g.n_blocks];
    const uint32_t n_chunks = g.chunks[g.n_slabs];
    const uint32_t C = g.chunks[g.n_slabs + 1];
    const int64_t slab_vox = (int64_t)g.layers * per_layer;
    uint64_t nseg = 0;
    for (;;) {
        if (threadIdx.x == 0) s_chunk = atomicAdd(a.work + kBinChunkWord, 1u);
        __syncthreads();
        const uint32_t c = s_chunk;
        if (c >= n_chunks) break;
        // the slab of chunk c: the last slab whose chunks start at or before it
        int lo = 0, hi = g.n_slabs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (g.chunks[mid] <= c) lo = mid;
            else hi = mid - 1;
        }
        const int sl = lo;
        const uint32_t a0 = g.cnt[(int64_t)sl * g.n_blocks];
        const uint32_t a1 = sl + 1 < g.n_slabs ? g.cnt[(int64_t)(sl + 1) * g.n_blocks] : total;
        const uint32_t i0 = a0 + (c - g.chunks[sl]) * C;
        const uint32_t i1 = min(a1, i0 + C);
        const SubBox box = slab_box(s, g.axis, g.layers, sl);
        const int nsv = (sl * g.layers + g.layers <= (g.axis == 0 ? s.nx : (g.axis == 1 ? s.ny : s.nz))
                             ? g.layers
                             : (g.axis == 0 ? s.nx : (g.axis == 1 ? s.ny : s.nz)) - sl * g.layers) *
                        per_layer;
        for (int i = threadIdx.x; i < nsv; i += kBlock) tally[i] = 0.0;
        if (threadIdx.x == 0) s_item = i0;
        __syncthreads();
        for (;;) {
            unsigned int it = 0;
            if (threadIdx.x % kWave == 0) it = atomicAdd(&s_item, 1u);
            it = __shfl(it, 0);
            if (it >= i1) break;
            const uint32_t t = g.list[it];
            grad_bin_task(a, cams, cpos, box, sl, tally, wave_queue[threadIdx.x / kWave],
                          nb - 1 - (int64_t)(t / kinds), (int)(t % kinds), nseg);
        }
        __syncthreads();
        double* __restrict__ out = g.partial + (int64_t)c * slab_vox;
        for (int i = threadIdx.x; i < nsv; i += kBlock) out[i] = tally[i];
        __syncthreads();
    }
    flush_counts(a.counters, nseg, 0, 0);
}

// grad[v] = sum over the chunks of v's slab, in chunk order, of the
// partials; one thread per slab voxel (slab after slab).
__global__ void __launch_bounds__(256) grad_bin_reduce_kernel(GradBins g, int nx, int ny, int nz,
                                                              double* __restrict__ grad,
                                                              const int* __restrict__ flag)
{
    if (*flag == 0) return;
    const int per_layer = g.axis == 0 ? ny * nz : (g.axis == 1 ? nx * nz : nx * ny);
    const int na = g.axis == 0 ? nx : (g.axis == 1 ? ny : nz);
    const int64_t slab_vox = (int64_t)g.layers * per_layer;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int sl = (int)(q / slab_vox);
    const int64_t i = q % slab_vox;
    if (sl >= g.n_slabs) return;
    const int la = (int)(i / per_layer);
    if (sl * g.layers + la >= na) return;
    const int r = (int)(i % per_layer);
    const int nb = g.axis == 0 ? ny : nx;
    const int ib = r % nb, ic = r / nb, ia = sl * g.layers + la;
    // (x, y, z) from the slab axis and the two others in increasing order
    const int x = g.axis == 0 ? ia : ib;
    const int y = g.axis == 0 ? ib : (g.axis == 1 ? ia : ic);
    const int z = g.axis == 2 ? ia : ic;
    double acc = 0.0;
    const uint32_t c0 = g.chunks[sl], c1 = g.chunks[sl + 1];
    for (uint32_t c = c0; c < c1; c += kBinReduceLoads) {
        double t[kBinReduceLoads];
#pragma unroll
        for (uint32_t j = 0; j < kBinReduceLoads; ++j) t[j] = c + j < c1 ? g.partial[(int64_t)(c + j) * slab_vox + i] : 0.0;
#pragma unroll
        for (int j = 0; j < kBinReduceLoads; ++j) acc += t[j];
    }
    grad[x + (int64_t)nx * (y + (int64_t)ny * z)] = acc;
}

GradBins choose_grad_bins(const DevScene& s, const DevCams& c, int64_t n_tasks)
{
    const int n[3] = {s.nx, s.ny, s.nz};
    // the slab axis along which the walks move least: the directions from the
    // box centre to the cameras and the sun's direction, summed per axis
    double spread[3] = {0.0, 0.0, 0.0};
    const double ctr[3] = {0.5 * s.nx, 0.5 * s.ny, 0.5 * s.nz};
    for (int d = 0; d < c.n; ++d) {
        double e[3], l2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            e[k] = c.pos[d][k] - ctr[k];
            l2 += e[k] * e[k];
        }
        const double il = l2 > 0.0 ? 1.0 / std::sqrt(l2) : 0.0;
        for (int k = 0; k < 3; ++k) spread[k] += std::fabs(e[k]) * il;
    }
    for (int k = 0; k < 3; ++k) spread[k] += std::fabs(s.sun[k]);
    GradBins g{};
    g.axis = 0;
    for (int k = 1; k < 3; ++k)
        if (spread[k] < spread[g.axis]) g.axis = k;
    const int ob = g.axis == 0 ? 1 : 0, oc = g.axis == 2 ? 1 : 2;
    const int64_t layer_bytes = (int64_t)n[ob] * n[oc] * (int64_t)sizeof(double);
    g.layers = (int)std::max<int64_t>(1, std::min<int64_t>(n[g.axis], (int64_t)kLdsBudget / layer_bytes));
    g.n_slabs = (n[g.axis] + g.layers - 1) / g.layers;
    g.n_tasks = n_tasks;
    g.n_blocks = (n_tasks + kBinTasks - 1) / kBinTasks;
    return g;
}

bool grad_bins_fit(const DevScene& s, const GradBins& g)
{
    const int n[3] = {s.nx, s.ny, s.nz};
    const int ob = g.axis == 0 ? 1 : 0, oc = g.axis == 2 ? 1 : 2;
    return (int64_t)n[ob] * n[oc] * (int64_t)sizeof(double) <= (int64_t)kLdsBudget && g.n_slabs <= kMaxBinSlabs;
}

hipError_t launch_grad_bin_init(hipStream_t st, const TraceArgs& a, const GradBins& g)
{
    const int64_t nu = (int64_t)a.s.nx * a.s.ny * a.s.nz;
    const int64_t n = std::max<int64_t>(std::max<int64_t>(g.n_tasks, nu), 1);
    grad_bin_init_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(a.trange, g.n_tasks, a.grad, nu);
    return hipGetLastError();
}

hipError_t launch_grad_bin_lists(hipStream_t st, const TraceArgs& a, const GradBins& g, uint32_t* scan_scratch)
{
    if (g.n_tasks <= 0) return hipSuccess;
    grad_bin_count_kernel<<<dim3((unsigned)g.n_blocks), dim3(kBinTasks), 0, st>>>(a.trange, g, a.tape_flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_scan_u32(st, g.cnt, (int64_t)g.n_slabs * g.n_blocks + 1, scan_scratch)) != hipSuccess) return e;
    grad_bin_fill_kernel<<<dim3((unsigned)g.n_blocks), dim3(kBinTasks), 0, st>>>(a.trange, g, a.tape_flag);
    return hipGetLastError();
}

hipError_t launch_grad_bin_walk(hipStream_t st, const TraceArgs& a, const DevCams& c, const GradBins& g, int n_cu)
{
    if (g.n_tasks <= 0) return hipSuccess;
    hipError_t e;
    grad_bin_chunks_kernel<<<dim3(1), dim3(256), 0, st>>>(g, n_cu, a.tape_flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int n[3] = {a.s.nx, a.s.ny, a.s.nz};
    const int ob = g.axis == 0 ? 1 : 0, oc = g.axis == 2 ? 1 : 2;
    const size_t lds = (size_t)g.layers * n[ob] * n[oc] * sizeof(double);
    if ((e = hipFuncSetAttribute((const void*)grad_bin_walk_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds)) != hipSuccess)
        return e;
    grad_bin_walk_kernel<<<dim3(n_cu), dim3(kBlock), lds, st>>>(a, c, g);
    return hipGetLastError();
}

hipError_t launch_grad_bin_reduce(hipStream_t st, const TraceArgs& a, const GradBins& g)
{
    if (g.n_tasks <= 0) return hipSuccess;
    const int n[3] = {a.s.nx, a.s.ny, a.s.nz};
    const int ob = g.axis == 0 ? 1 : 0, oc = g.axis == 2 ? 1 : 2;
    const int64_t cells = (int64_t)g.n_slabs * g.layers * n[ob] * n[oc];
    grad_bin_reduce_kernel<<<dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st>>>(g, a.s.nx, a.s.ny, a.s.nz,
                                                                                       a.grad, a.tape_flag);
    return hipGetLastError();
}

size_t grad_bin_partial_bytes(const DevScene& s, const GradBins& g, int n_cu)
{
    const int n[3] = {s.nx, s.ny, s.nz};
    const int ob = g.axis == 0 ? 1 : 0, oc = g.axis == 2 ? 1 : 2;
    const size_t chunks = (size_t)kBinChunksPerWg * n_cu + g.n_slabs;
    return chunks * (size_t)g.layers * n[ob] * n[oc] * sizeof(double);
}

// Recomputing variant (no valid tape, or all-FP64 mode), per path: pass 1
// recomputes every contribution c_{b,d} and its weight w, adds the connection
// part of the score and keeps R_b; pass 2 walks the free-flight segments
// backwards with the suffix sums A_k.  Camera groups split a path's local
// estimates; pass 2 is linear in R_b, so each group runs it with its own
// partial sums and the totals add up.  With a tape flag it runs only when
// the tape does not match beta_t.
template <typename Real, bool kLds>
__global__ void __launch_bounds__(kBlock) grad_kernel(TraceArgs a, DevCams cams, int z0, int z1,
                                                      double* __restrict__ partial)
{
    if (a.tape_flag && *a.tape_flag != 0) return;
    extern __shared__ unsigned char smem[];
    const SlabTally<kLds> tally = slab_tally_begin<kLds>(a, z0, z1, smem);
    auto add = [&](uint32_t v, double x) { tally.add(v, x); };
    const DevScene& s = a.s;
    const int nu = s.nx * s.ny * s.nz;
    const Real* __restrict__ gtot = (const Real*)a.grid_tot;
    const Real* __restrict__ gd = (const Real*)a.grid_dlt;
    const int npix = cams.W * cams.H;
    const double r2scale = 1.0 / (s.vk * s.vk);
    const int lane = threadIdx.x % kWave;
    const int64_t nb = a.st.n_slots / kWave;
    const int G = a.groups, cpg = (cams.n + G - 1) / G;
    const unsigned int n_tasks = (unsigned int)(nb - a.st.first_slot / kWave) * (unsigned int)G;
    // algorithmic work is counted once, in the launch of the first slab
    const bool count = z0 == 0;
    uint64_t nseg = 0, novh = 0;
    double R[kMaxOrder + 1];
    const unsigned int tc = task_counter();
    for (unsigned int task = next_task(a.work, tc); task < n_tasks; task = next_task(a.work, tc)) {
        const int64_t bt = nb - 1 - (int64_t)(task / G);
        const int g = (int)(task % G);
        const int d_lo = g * cpg, d_hi = min(cams.n, d_lo + cpg);
        const int64_t slot = bt * kWave + lane;
        const int Bn = (int)a.st.B[slot];
        if (Bn <= 0) continue;
        uint64_t& segc = g == 0 ? nseg : novh;
        uint64_t& cseg = count ? nseg : novh;
        const float4* __restrict__ V = a.st.vtx + a.st.batch_off[bt] + lane;
        Vtx p0 = load_vtx(V, 0);
        double P = s.w0;
        double wprev[3] = {0.0, 0.0, 0.0};
        for (int b = 1; b <= Bn; ++b) {
            const Vtx p1 = load_vtx(V, b);
            double w[3];
            const double L = seg_dir(p0, p1, w);
            const Real dt = walk_sum<Real, true, kWalkLoads>(s, [&](uint32_t v) { return gd[v]; }, p0, w, L, novh);
            P *= exp(-(double)dt * s.vk);
            if (b >= 2) {
                const int v = clamp_vox(p0.v, nu);
                P *= vertex_ratio(s, (double)a.bc_t[v], (double)a.st.beta_ref[v],
                                  wprev[0] * w[0] + wprev[1] * w[1] + wprev[2] * w[2]);
            }
            const int v1 = clamp_vox(p1.v, nu);
            const double bct = (double)a.bc_t[v1];
            const double base = P / ((double)a.st.beta_ref[v1] + s.beta_air);
            double Rb = 0.0, vert = 0.0;
            for (int d = d_lo; d < d_hi; ++d) {
                const int pix = project(cams, d, p1.x, p1.y, p1.z, s.vk);
                if (pix < 0) continue;
                const double rho = a.rho[(int64_t)d * npix + pix];
                if (rho == 0.0) continue;
                const double ex = cams.pos[d][0] - p1.x, ey = cams.pos[d][1] - p1.y, ez = cams.pos[d][2] - p1.z;
                const double dist2 = ex * ex + ey * ey + ez * ez;
                const double dist = sqrt(dist2);
                const double id = 1.0 / dist;
                const double u[3] = {ex * id, ey * id, ez * id};
                const double mu = w[0] * u[0] + w[1] * u[1] + w[2] * u[2];
                const double hg = phase_hg(s, mu);
                const double fst = fs_mix(s, bct, hg, phase_rayleigh(mu));
                const Real tc = walk_sum<Real, true, kWalkLoads>(s, [&](uint32_t v) { return gtot[v]; }, p1, u, dist, cseg);
                const double c = base * fst * exp(-(double)tc * s.vk) * (r2scale / dist2);
                const double wgt = c * rho;
                Rb += wgt;
                // vertex term at x_b: w * w_c f_HG / f_s,t
                if (fst > 0.0) vert += wgt * (s.w_c * hg / fst);
                walk_scatter<Real>(s, add, p1, u, dist, -wgt * s.vk, novh, z0, z1);
            }
            if (vert != 0.0) tally.add_vox(v1, vert);
            R[b] = Rb;
            wprev[0] = w[0]; wprev[1] = w[1]; wprev[2] = w[2];
            p0 = p1;
        }
        // pass 2: segments k = Bn-1 .. 0 with suffix weights
        double A = 0.0;
        Vtx pk1 = load_vtx(V, Bn);
        for (int k = Bn - 1; k >= 0; --k) {
            A += R[k + 1];
            const Vtx pk = load_vtx(V, k);
            double w[3];
            const double L = seg_dir(pk, pk1, w);
            if (A != 0.0) {
                walk_scatter<Real>(s, add, pk, w, L, -A * s.vk, segc, z0, z1);
                const int v = clamp_vox(pk.v, nu);
                if (k >= 1 && (unsigned)(v - tally.vlo) < (unsigned)tally.nsv) {
                    const Vtx pm = load_vtx(V, k - 1);
                    double wm[3];
                    seg_dir(pm, pk, wm);
                    const double mu = wm[0] * w[0] + wm[1] * w[1] + wm[2] * w[2];
                    const double hg = phase_hg(s, mu);
                    const double fst = fs_mix(s, (double)a.bc_t[v], hg, phase_rayleigh(mu));
                    if (fst > 0.0) tally.add((uint32_t)(v - tally.vlo), A * (s.w_c * hg / fst));
                }
            }
            pk1 = pk;
        }
    }
    flush_counts(a.counters, nseg, 0, novh);
    slab_tally_end<kLds>(tally, partial);
}

// grad[v] = sum over workgroups of partial[w][v] in a fixed order: a
// workgroup covers 64 voxels, its wavefront c sums the partials of the c-th
// contiguous share of the workgroups (kReduceChunks shares, kReduceLoads loads
// in flight per lane), and the shares are added in order.
constexpr int kReduceChunks = 8;
constexpr int kReduceLoads = 8;

__global__ void __launch_bounds__(kReduceChunks * kWave) grad_reduce_kernel(const double* __restrict__ partial,
                                                                           int n_wg, int64_t nv,
                                                                           double* __restrict__ grad,
                                                                           unsigned int* __restrict__ work,
                                                                           const int* __restrict__ skip)
{
    __shared__ double red[kReduceChunks][kWave];
    // zeroes the task counters of the next slab's launch
    if (blockIdx.x == 0 && threadIdx.x < 2 * kTaskCounters)
        work[(threadIdx.x / 2) * kTaskStride + threadIdx.x % 2] = 0u;
    // the binned walk on the tape has written the gradient
    if (skip && *skip != 0) return;
    const int lane = threadIdx.x % kWave, c = threadIdx.x / kWave;
    const int64_t v = (int64_t)blockIdx.x * kWave + lane;
    const int cs = (n_wg + kReduceChunks - 1) / kReduceChunks;
    const int w0 = c * cs, w1 = min(n_wg, w0 + cs);
    double acc = 0.0;
    if (v < nv) {
        for (int w = w0; w < w1; w += kReduceLoads) {
            double x[kReduceLoads];
#pragma unroll
            for (int j = 0; j < kReduceLoads; ++j) x[j] = w + j < w1 ? partial[(int64_t)(w + j) * nv + v] : 0.0;
#pragma unroll
            for (int j = 0; j < kReduceLoads; ++j) acc += x[j];
        }
    }
    red[c][lane] = acc;
    __syncthreads();
    if (c == 0 && v < nv) {
        double t = 0.0;
        for (int k = 0; k < kReduceChunks; ++k) t += red[k][lane];
        grad[v] = t;
    }
}

template <typename Kern>
static hipError_t launch_persistent(hipStream_t st, Kern k, int n_wg, size_t lds, const TraceArgs& a,
                                   const DevCams& c, int z0, int z1, double* partial)
{
    if (lds) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k<<<dim3(n_wg), dim3(kBlock), lds, st>>>(a, c, z0, z1, partial);
    return hipGetLastError();
}

// The walk kernel on stored weights (when a tape flag is given; task counter
// work[0]) and the recomputing kernel (work[1]); exactly one of them does work.
template <typename Real, bool kLds>
static hipError_t launch_grad_t(hipStream_t st, const TraceArgs& a, const DevCams& c, const GradPlan& p, int z0,
                                int z1, double* partial, bool walk_on_tape)
{
    const size_t lds = kLds ? (size_t)(z1 - z0) * a.s.nx * a.s.ny * sizeof(double) : 0;
    hipError_t e = hipSuccess;
    const bool tape = sizeof(Real) == 4 && a.tape_flag && a.tape && a.wtape && a.vaux;
    const bool walk = tape && walk_on_tape;
    if (walk) e = launch_persistent(st, grad_walk_kernel<kLds>, p.n_wg, lds, a, c, z0, z1, partial);
    if (e != hipSuccess) return e;
    // without a tape the recomputing kernel must run whatever the flag says;
    // with one it runs only when the tape does not match beta_t
    TraceArgs b = a;
    b.work = a.work + 1;
    if (!tape) b.tape_flag = nullptr;
    return launch_persistent(st, grad_kernel<Real, kLds>, p.n_wg, lds, b, c, z0, z1, partial);
}

GradPlan plan_grad(int nx, int ny, int nz, int64_t n_slots, int64_t first_slot, int n_cu, bool tape)
{
    GradPlan p;
    const int64_t layer_bytes = (int64_t)nx * ny * (int64_t)sizeof(double);
    const int64_t layers = std::min<int64_t>(nz, (int64_t)kLdsBudget / layer_bytes);
    const int64_t slabs = layers > 0 ? (nz + layers - 1) / layers : 0;
    // Without the tape every slab recomputes the contributions, so past a few
    // slabs FP64 atomics on the output are cheaper; with it a slab only walks,
    // and LDS tallies stay cheaper than global FP64 atomics (~1600 clocks per
    // wavefront instruction) up to many slabs.
    p.lds = layers > 0 && slabs <= (tape ? kMaxTapeGradSlabs : kMaxGradSlabs);
    p.slab_layers = p.lds ? (int)layers : nz;
    p.n_slabs = p.lds ? (int)slabs : 1;
    const int64_t batches = (n_slots - first_slot + kWave - 1) / kWave;
    const int64_t need = std::max<int64_t>(1, (batches + kWavesPerBlock - 1) / kWavesPerBlock);
    p.n_wg = (int)std::min<int64_t>(need, (int64_t)n_cu * (p.lds ? 1 : 2));
    p.partial_bytes = p.lds ? (size_t)p.n_wg * (size_t)(p.slab_layers * layer_bytes) : 0;
    return p;
}

void grad_slab(const GradPlan& p, int nz, int i, int* z0, int* z1)
{
    *z0 = i * p.slab_layers;
    *z1 = std::min(nz, *z0 + p.slab_layers);
}

hipError_t launch_grad(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c, const GradPlan& p, int slab,
                       void* partial, bool walk_on_tape)
{
    if (a.st.n_slots - a.st.first_slot <= 0) return hipSuccess;
    int z0, z1;
    grad_slab(p, a.s.nz, slab, &z0, &z1);
    if (fp64) {
        if (p.lds) return launch_grad_t<double, true>(st, a, c, p, z0, z1, (double*)partial, walk_on_tape);
        return launch_grad_t<double, false>(st, a, c, p, z0, z1, nullptr, walk_on_tape);
    }
    if (p.lds) return launch_grad_t<float, true>(st, a, c, p, z0, z1, (double*)partial, walk_on_tape);
    return launch_grad_t<float, false>(st, a, c, p, z0, z1, nullptr, walk_on_tape);
}

hipError_t launch_grad_reduce(hipStream_t st, const GradPlan& p, int nx, int ny, int nz, int slab,
                              const void* partial, double* grad, unsigned int* work, const int* skip)
{
    if (!p.lds) return hipSuccess;
    int z0, z1;
    grad_slab(p, nz, slab, &z0, &z1);
    const int64_t layer = (int64_t)nx * ny, nv = (int64_t)(z1 - z0) * layer;
    grad_reduce_kernel<<<dim3((unsigned)std::max<int64_t>(1, (nv + kWave - 1) / kWave)), dim3(kReduceChunks * kWave),
                         0, st>>>((const double*)partial, p.n_wg, nv, grad + z0 * layer, work, skip);
    return hipGetLastError();
}

// flag = 1 when two fields are bitwise equal (the tape's beta and beta_t).
__global__ void __launch_bounds__(256) equal_flag_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                         int64_t n, int* __restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && __float_as_int(x[i]) != __float_as_int(y[i])) *flag = 0;
}


hipError_t launch_equal_flag(hipStream_t st, const float* x, const float* y, int64_t n, int* flag)
{
    equal_flag_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(x, y, n, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------- reweight

// log r = log mu(x|beta_t) - log mu(x|beta_ref) over the whole stored path:
// every segment's optical-depth difference (the exit segment included), the
// extinction ratio at every scatter, and the direction-pdf ratio
// f_p = f_s / beta_s at every scatter that has a successor vertex.  The sum is
// taken in log space in FP64: each scatter adds the log of its own factor
// (extinction ratio times direction-pdf ratio), so no running product can
// overflow or underflow.  A path that beta_t cannot produce (zero extinction,
// or zero directional function, at one of its scatters) has r = 0: the
// sampling pdf of Eq. final_mu carries beta(x_k) at every scatter vertex.  One
// lane per path in persistent workgroups (the field beta_t - beta_ref cached
// in LDS when it fits); per-workgroup sums of r and r^2 go to partial[2*wg].
template <typename Real, bool kGridLds>
__global__ void __launch_bounds__(kBlock) reweight_kernel(TraceArgs a)
{
    extern __shared__ unsigned char smem[];
    __shared__ double red[2][kWavesPerBlock];
    const Real* gd = delta_grid<Real, kGridLds>(a, smem);
    const DevScene& s = a.s;
    const int nu = s.nx * s.ny * s.nz;
    double rs = 0.0, r2s = 0.0;
    uint64_t cnt = 0;
    // slots in batch order from the heaviest batch (the end of the store) down
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < a.st.n_slots;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t slot = (a.st.n_slots / kWave - 1 - q / kWave) * kWave + q % kWave;
        const int nv = (int)a.st.nv[slot];
        const int Bn = (int)a.st.B[slot];
        if (nv <= 0) continue;
        const float4* __restrict__ V = a.st.vtx + a.st.batch_off[slot / kWave] + (slot % kWave);
        double lr = 0.0;     // log r
        bool possible = true;  // false once some factor of mu(x|beta_t) is zero
        Vtx p0 = load_vtx(V, 0);
        double wprev[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k + 1 < nv; ++k) {
            const Vtx p1 = load_vtx(V, k + 1);
            double w[3];
            const double L = seg_dir(p0, p1, w);
            lr -= (double)delta_walk<Real, kGridLds>(s, gd, p0, w, L, cnt) * s.vk;
            if (k >= 1) {
                // scatter k (it has the successor k+1): extinction ratio and
                // direction-pdf ratio f_s,t bs_ref / (f_s,ref bs_t)
                const int v = clamp_vox(p0.v, nu);
                const double bct = (double)a.bc_t[v], bcr = (double)a.st.beta_ref[v];
                const double mu = wprev[0] * w[0] + wprev[1] * w[1] + wprev[2] * w[2];
                const double hg = phase_hg(s, mu), ra = phase_rayleigh(mu);
                const double bst = s.w_c * bct + s.w_a * s.beta_air, bsr = s.w_c * bcr + s.w_a * s.beta_air;
                const double fst = fs_mix(s, bct, hg, ra), fsr = fs_mix(s, bcr, hg, ra);
                if (fst > 0.0 && bst > 0.0)
                    lr += log(((bct + s.beta_air) * fst * bsr) / ((bcr + s.beta_air) * fsr * bst));
                else
                    possible = false;
            }
            wprev[0] = w[0]; wprev[1] = w[1]; wprev[2] = w[2];
            p0 = p1;
        }
        // the last scatter of a path capped at max_order has no successor: its
        // extinction ratio alone
        if (Bn > 0 && Bn + 1 == nv) {
            const int v = clamp_vox(vox_of(V[(int64_t)Bn * kWave]), nu);
            const double bt = (double)a.bc_t[v] + s.beta_air;
            if (bt > 0.0)
                lr += log(bt / ((double)a.st.beta_ref[v] + s.beta_air));
            else
                possible = false;
        }
        const double r = possible ? exp(lr) : 0.0;
        rs += r;
        r2s += r * r;
    }
    // workgroup sums in a fixed order: within each wavefront, then over wavefronts
    for (int o = kWave / 2; o > 0; o >>= 1) {
        rs += __shfl_down(rs, o);
        r2s += __shfl_down(r2s, o);
    }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (lane == 0) {
        red[0][wave] = rs;
        red[1][wave] = r2s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            t0 += red[0][w];
            t1 += red[1][w];
        }
        a.partial[2 * blockIdx.x] = t0;
        a.partial[2 * blockIdx.x + 1] = t1;
    }
}

int64_t reweight_blocks(int64_t n_slots, int n_cu)
{
    return std::max<int64_t>(1, std::min<int64_t>((n_slots + kBlock - 1) / kBlock, n_cu));
}

hipError_t launch_reweight(hipStream_t st, int fp64, const TraceArgs& a, int n_cu, int64_t* n_blocks)
{
    const size_t grid_bytes = (size_t)a.s.nx * a.s.ny * a.s.nz * (fp64 ? 8 : 4);
    const bool lds = grid_bytes <= kLdsBudget;
    const int n_wg = (int)reweight_blocks(a.st.n_slots, n_cu);
    *n_blocks = n_wg;
    if (fp64)
        return lds ? launch_delta_kernel(st, reweight_kernel<double, true>, true, grid_bytes, n_wg, a)
                   : launch_delta_kernel(st, reweight_kernel<double, false>, false, grid_bytes, n_wg, a);
    return lds ? launch_delta_kernel(st, reweight_kernel<float, true>, true, grid_bytes, n_wg, a)
               : launch_delta_kernel(st, reweight_kernel<float, false>, false, grid_bytes, n_wg, a);
}

}  // namespace prt
