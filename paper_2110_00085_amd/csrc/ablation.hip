// Path-sorting ablation (Sec. 5.3): the paper's GPU design, one thread per
// stored path that walks all of that path's scatters and cameras, run on a
// per-path (CSR) copy of a store in one of two orders -- sorted by path size
// B (Alg. 2 "Sort") or in the order the paths were drawn -- so that the only
// difference between the two runs is which paths share a wavefront.
//
// The numbers computed are those of the production kernels (trace.hip): the
// recycled local estimates of Eq. forward_simualtion_recycling and the
// gradient of Eq. gradient_simualtion_recycling through the tomography path
// score function; only the work decomposition differs.  Images are tallied
// with FP64 atomics on the output, the gradient per workgroup in FP64 LDS
// slabs of z layers (reduced by grad_reduce_kernel) or with FP64 atomics
// when the grid needs too many slabs.
#include <algorithm>

#include "launch.hpp"
#include "trace_common.hpp"

namespace prt {

using namespace trace;

namespace {

constexpr int kTppBlock = 1024;

// Path q of the CSR copy: its records rec[off[q] .. off[q+1]) and its size.
__device__ __forceinline__ Vtx csr_vtx(const float4* __restrict__ V, int k)
{
    const float4 r = V[k];
    return Vtx{(double)r.x, (double)r.y, (double)r.z, vox_of(r)};
}

}  // namespace

// Sizes of the paths in the chosen order: qnv[q] (records) and qB[q].
__global__ void __launch_bounds__(256) tpp_sizes_kernel(StoreView st, int64_t n, const int32_t* __restrict__ inv,
                                                        int64_t* __restrict__ qnv, uint8_t* __restrict__ qB)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q > n) return;
    if (q == n) {
        qnv[n] = 0;  // the scan's last element becomes the record total
        return;
    }
    const int64_t slot = inv ? inv[q] : q;
    qnv[q] = st.nv[slot];
    qB[q] = st.B[slot];
}

// inv[perm[s]] = s: path id -> sorted slot.
__global__ void __launch_bounds__(256) tpp_inverse_kernel(const int32_t* __restrict__ perm, int64_t n,
                                                          int32_t* __restrict__ inv)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) inv[perm[s]] = (int32_t)s;
}

// rec[off[q] + k] = vertex k of path q (from the store's batch layout).
__global__ void __launch_bounds__(256) tpp_copy_kernel(StoreView st, int64_t n, const int32_t* __restrict__ inv,
                                                       const int64_t* __restrict__ off, float4* __restrict__ rec)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int64_t slot = inv ? inv[q] : q;
    const float4* __restrict__ V = st.vtx + st.batch_off[slot / kWave] + slot % kWave;
    const int nv = (int)(off[q + 1] - off[q]);
    for (int k = 0; k < nv; ++k) rec[off[q] + k] = V[(int64_t)k * kWave];
}

// One thread per path (static assignment, q = thread + k * threads): the
// recycled prefix weight is carried along the path and every (scatter,
// camera) contribution goes to the image as an FP64 atomic.
template <typename Real, bool kGridLds>
__global__ void __launch_bounds__(kTppBlock) tpp_render_kernel(TraceArgs a, DevCams cams, TppView v)
{
    extern __shared__ unsigned char smem[];
    const DevScene& s = a.s;
    const int nu = s.nx * s.ny * s.nz;
    const int npix = cams.W * cams.H;
    Real* __restrict__ sgrid = reinterpret_cast<Real*>(smem);
    const Real* __restrict__ gtot = (const Real*)a.grid_tot;
    const Real* __restrict__ gd = (const Real*)a.grid_dlt;
    if (kGridLds) {
        lds_fill(sgrid, nu, [&](int i) { return (Real)((double)a.bc_t[i] + s.beta_air); });
        __syncthreads();
    }
    auto beta_tot = [&](uint32_t u) -> Real { return kGridLds ? sgrid[u] : gtot[u]; };
    const double r2scale = 1.0 / (s.vk * s.vk);
    uint64_t nseg = 0, nle = 0, novh = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < v.n; q += (int64_t)gridDim.x * blockDim.x) {
        const int Br = min((int)v.B[q], a.brender);
        if (Br <= 0) continue;
        const float4* __restrict__ V = v.rec + v.off[q];
        Vtx p0 = csr_vtx(V, 0);
        double P = s.w0;
        double wprev[3] = {0.0, 0.0, 0.0};
        for (int b = 1; b <= Br; ++b) {
            const Vtx p1 = csr_vtx(V, b);
            double w[3];
            const double L = seg_dir(p0, p1, w);
            const Real dt = walk_sum<Real>(s, [&](uint32_t u) { return gd[u]; }, p0, w, L, novh);
            P *= exp(-(double)dt * s.vk);
            if (b >= 2) {
                const int u = clamp_vox(p0.v, nu);
                P *= vertex_ratio(s, (double)a.bc_t[u], (double)a.st.beta_ref[u],
                                  wprev[0] * w[0] + wprev[1] * w[1] + wprev[2] * w[2]);
            }
            const int v1 = clamp_vox(p1.v, nu);
            const double bct = (double)a.bc_t[v1];
            const double base = P / ((double)a.st.beta_ref[v1] + s.beta_air);
            for (int d = 0; d < cams.n; ++d) {
                const int pix = project(cams, d, p1.x, p1.y, p1.z, s.vk);
                if (pix < 0) continue;
                const double ex = cams.pos[d][0] - p1.x, ey = cams.pos[d][1] - p1.y, ez = cams.pos[d][2] - p1.z;
                const double dist2 = ex * ex + ey * ey + ez * ez;
                const double dist = sqrt(dist2);
                const double id = 1.0 / dist;
                const double u[3] = {ex * id, ey * id, ez * id};
                const double mu = w[0] * u[0] + w[1] * u[1] + w[2] * u[2];
                const double fst = fs_mix(s, bct, phase_hg(s, mu), phase_rayleigh(mu));
                const Real tc = cams.outside ? walk_sum<Real, false>(s, beta_tot, p1, u, dist, nseg)
                                             : walk_sum<Real>(s, beta_tot, p1, u, dist, nseg);
                const double c = base * fst * exp(-(double)tc * s.vk) * (r2scale / dist2);
                unsafeAtomicAdd(&a.img[(int64_t)d * npix + pix], c);
                ++nle;
            }
            wprev[0] = w[0]; wprev[1] = w[1]; wprev[2] = w[2];
            p0 = p1;
        }
    }
    flush_counts(a.counters, nseg, nle, novh);
}

// One thread per path: pass 1 recomputes every contribution c_{b,d}, its
// weight w = c rho and adds the connection part of the score (clipped to the
// slab [z0, z1)) and the vertex terms, keeping R_b = sum_d w_{b,d}; pass 2
// walks the free-flight segments backwards with the suffix sums A_k.
template <typename Real, bool kLds>
__global__ void __launch_bounds__(kTppBlock) tpp_grad_kernel(TraceArgs a, DevCams cams, TppView v, int z0, int z1,
                                                             double* __restrict__ partial)
{
    extern __shared__ unsigned char smem[];
    const DevScene& s = a.s;
    const int nu = s.nx * s.ny * s.nz;
    const int layer = s.nx * s.ny;
    const int vlo = z0 * layer, nsv = (z1 - z0) * layer;
    double* __restrict__ tally = kLds ? reinterpret_cast<double*>(smem) : a.grad + vlo;
    if (kLds) {
        for (int i = threadIdx.x; i < nsv; i += blockDim.x) tally[i] = 0.0;
        __syncthreads();
    }
    auto add = [&](uint32_t u, double x) {
        if (kLds) atomicAdd(&tally[u], x);
        else unsafeAtomicAdd(&tally[u], x);
    };
    auto add_vox = [&](int u, double x) {
        const int r = u - vlo;
        if ((unsigned)r < (unsigned)nsv) add((uint32_t)r, x);
    };
    const Real* __restrict__ gtot = (const Real*)a.grid_tot;
    const Real* __restrict__ gd = (const Real*)a.grid_dlt;
    const int npix = cams.W * cams.H;
    const double r2scale = 1.0 / (s.vk * s.vk);
    // algorithmic work is counted once, in the launch of the first slab
    const bool count = z0 == 0;
    uint64_t nseg = 0, novh = 0;
    double R[kMaxOrder + 1];
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < v.n; q += (int64_t)gridDim.x * blockDim.x) {
        const int Bn = (int)v.B[q];
        if (Bn <= 0) continue;
        uint64_t& cseg = count ? nseg : novh;
        const float4* __restrict__ V = v.rec + v.off[q];
        Vtx p0 = csr_vtx(V, 0);
        double P = s.w0;
        double wprev[3] = {0.0, 0.0, 0.0};
        for (int b = 1; b <= Bn; ++b) {
            const Vtx p1 = csr_vtx(V, b);
            double w[3];
            const double L = seg_dir(p0, p1, w);
            const Real dt = walk_sum<Real>(s, [&](uint32_t u) { return gd[u]; }, p0, w, L, novh);
            P *= exp(-(double)dt * s.vk);
            if (b >= 2) {
                const int u = clamp_vox(p0.v, nu);
                P *= vertex_ratio(s, (double)a.bc_t[u], (double)a.st.beta_ref[u],
                                  wprev[0] * w[0] + wprev[1] * w[1] + wprev[2] * w[2]);
            }
            const int v1 = clamp_vox(p1.v, nu);
            const double bct = (double)a.bc_t[v1];
            const double base = P / ((double)a.st.beta_ref[v1] + s.beta_air);
            double Rb = 0.0, vert = 0.0;
            for (int d = 0; d < cams.n; ++d) {
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
                const Real tc = walk_sum<Real>(s, [&](uint32_t uu) { return gtot[uu]; }, p1, u, dist, novh);
                const double c = base * fst * exp(-(double)tc * s.vk) * (r2scale / dist2);
                const double wgt = c * rho;
                Rb += wgt;
                if (fst > 0.0) vert += wgt * (s.w_c * hg / fst);
                walk_scatter<Real>(s, add, p1, u, dist, -wgt * s.vk, cseg, z0, z1);
            }
            if (vert != 0.0) add_vox(v1, vert);
            R[b] = Rb;
            wprev[0] = w[0]; wprev[1] = w[1]; wprev[2] = w[2];
            p0 = p1;
        }
        double A = 0.0;
        Vtx pk1 = csr_vtx(V, Bn);
        for (int k = Bn - 1; k >= 0; --k) {
            A += R[k + 1];
            const Vtx pk = csr_vtx(V, k);
            double w[3];
            const double L = seg_dir(pk, pk1, w);
            if (A != 0.0) {
                walk_scatter<Real>(s, add, pk, w, L, -A * s.vk, cseg, z0, z1);
                const int u = clamp_vox(pk.v, nu);
                if (k >= 1 && (unsigned)(u - vlo) < (unsigned)nsv) {
                    const Vtx pm = csr_vtx(V, k - 1);
                    double wm[3];
                    seg_dir(pm, pk, wm);
                    const double mu = wm[0] * w[0] + wm[1] * w[1] + wm[2] * w[2];
                    const double hg = phase_hg(s, mu);
                    const double fst = fs_mix(s, (double)a.bc_t[u], hg, phase_rayleigh(mu));
                    if (fst > 0.0) add((uint32_t)(u - vlo), A * (s.w_c * hg / fst));
                }
            }
            pk1 = pk;
        }
    }
    flush_counts(a.counters, nseg, 0, novh);
    if (kLds) {
        __syncthreads();
        double* __restrict__ out = partial + (int64_t)blockIdx.x * nsv;
        for (int i = threadIdx.x; i < nsv; i += blockDim.x) out[i] = tally[i];
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_tpp_layout(hipStream_t st, const StoreView& sv, int64_t n, const int32_t* perm, int order,
                             int32_t* inv, int64_t* off, uint8_t* qB, void* scan_scratch)
{
    const unsigned blocks = (unsigned)((n + 1 + 255) / 256);
    const int32_t* pinv = nullptr;
    if (order == 1) {
        tpp_inverse_kernel<<<dim3(blocks), dim3(256), 0, st>>>(perm, n, inv);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        pinv = inv;
    }
    tpp_sizes_kernel<<<dim3(blocks), dim3(256), 0, st>>>(sv, n, pinv, off, qB);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_scan_i64(st, off, n + 1, (int64_t*)scan_scratch);
}

hipError_t launch_tpp_copy(hipStream_t st, const StoreView& sv, int64_t n, const int32_t* inv, int order,
                           const int64_t* off, float4* rec)
{
    tpp_copy_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(sv, n, order == 1 ? inv : nullptr,
                                                                          off, rec);
    return hipGetLastError();
}

template <typename K>
static hipError_t set_dynamic_lds(K k, size_t lds)
{
    if (!lds) return hipSuccess;
    return hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename Real, bool kGridLds>
static hipError_t run_tpp_render(hipStream_t st, const TraceArgs& a, const DevCams& c, const TppView& v, int n_wg,
                                 size_t lds)
{
    hipError_t e = set_dynamic_lds(tpp_render_kernel<Real, kGridLds>, lds);
    if (e != hipSuccess) return e;
    tpp_render_kernel<Real, kGridLds><<<dim3(n_wg), dim3(kTppBlock), lds, st>>>(a, c, v);
    return hipGetLastError();
}

hipError_t launch_tpp_render(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c, const TppView& v,
                             int n_cu)
{
    if (v.n <= 0) return hipSuccess;
    const size_t nu = (size_t)a.s.nx * a.s.ny * a.s.nz;
    const size_t grid_bytes = nu * (fp64 ? 8 : 4);
    const bool lds = grid_bytes <= 128 * 1024;
    const int n_wg = (int)std::max<int64_t>(1, std::min<int64_t>((v.n + kTppBlock - 1) / kTppBlock, n_cu));
    if (fp64)
        return lds ? run_tpp_render<double, true>(st, a, c, v, n_wg, grid_bytes)
                   : run_tpp_render<double, false>(st, a, c, v, n_wg, 0);
    return lds ? run_tpp_render<float, true>(st, a, c, v, n_wg, grid_bytes)
               : run_tpp_render<float, false>(st, a, c, v, n_wg, 0);
}

template <typename Real, bool kLds>
static hipError_t run_tpp_grad(hipStream_t st, const TraceArgs& a, const DevCams& c, const TppView& v, int n_wg,
                               size_t lds, int z0, int z1, double* partial)
{
    hipError_t e = set_dynamic_lds(tpp_grad_kernel<Real, kLds>, lds);
    if (e != hipSuccess) return e;
    tpp_grad_kernel<Real, kLds><<<dim3(n_wg), dim3(kTppBlock), lds, st>>>(a, c, v, z0, z1, partial);
    return hipGetLastError();
}

hipError_t launch_tpp_grad(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c, const TppView& v,
                           const GradPlan& p, int slab, double* partial)
{
    if (v.n <= 0) return hipSuccess;
    int z0, z1;
    grad_slab(p, a.s.nz, slab, &z0, &z1);
    const size_t lds = p.lds ? (size_t)(z1 - z0) * a.s.nx * a.s.ny * sizeof(double) : 0;
    if (fp64)
        return p.lds ? run_tpp_grad<double, true>(st, a, c, v, p.n_wg, lds, z0, z1, partial)
                     : run_tpp_grad<double, false>(st, a, c, v, p.n_wg, 0, z0, z1, nullptr);
    return p.lds ? run_tpp_grad<float, true>(st, a, c, v, p.n_wg, lds, z0, z1, partial)
                 : run_tpp_grad<float, false>(st, a, c, v, p.n_wg, 0, z0, z1, nullptr);
}

}  // namespace prt
