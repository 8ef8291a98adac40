// Hot path on stored paths: recycled rendering with local estimation
// (Sec. 5.2 + Sec. 3.4.3), the loss gradient through the tomography path
// score function (Sec. 4.4, App. C), and the correction-factor statistics.
//
// One lane per stored path; a wavefront holds a batch of 64 paths of
// (nearly) equal size B thanks to the sort, so lanes leave the scatter loop
// together.  The voxel walk runs in Real (float or double); projection,
// phase functions, path weights and all tallies are FP64.
#include "launch.hpp"

namespace prt {

namespace {

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

// Sum of grid[v] * length over the walk from vertex p (voxel p.v) along w for
// length tmax; returns the sum (grid units) and adds the pieces to *count.
template <typename Real>
__device__ __forceinline__ Real walk_sum(const DevScene& s, const Real* __restrict__ grid, const Vtx& p,
                                         const double w[3], double tmax, uint64_t& count)
{
    int ix, iy, iz;
    voxel_ijk(clamp_vox(p.v, s.nx * s.ny * s.nz), s.nx, s.ny, ix, iy, iz);
    Real acc = (Real)0;
    dda_walk<Real>(s.nx, s.ny, s.nz, (Real)p.x, (Real)p.y, (Real)p.z, ix, iy, iz, (Real)w[0], (Real)w[1],
                   (Real)w[2], (Real)tmax, [&](int v, Real, Real l) {
                       acc += grid[v] * l;
                       ++count;
                       return true;
                   });
    return acc;
}

// Adds scale * length (km) to grad[v] for every piece of the walk.
template <typename Real>
__device__ __forceinline__ void walk_scatter(const DevScene& s, double* __restrict__ grad, const Vtx& p,
                                             const double w[3], double tmax, double scale, uint64_t& count)
{
    int ix, iy, iz;
    voxel_ijk(clamp_vox(p.v, s.nx * s.ny * s.nz), s.nx, s.ny, ix, iy, iz);
    dda_walk<Real>(s.nx, s.ny, s.nz, (Real)p.x, (Real)p.y, (Real)p.z, ix, iy, iz, (Real)w[0], (Real)w[1],
                   (Real)w[2], (Real)tmax, [&](int v, Real, Real l) {
                       unsafeAtomicAdd(&grad[v], scale * (double)l);
                       ++count;
                       return true;
                   });
}

// Factor of scatter vertex k (1 <= k < b) in the recycled contribution:
// albedo_ref(x_k) * f_s,t(x_k, mu_k) / f_s,ref(x_k, mu_k).
__device__ __forceinline__ double vertex_ratio(const DevScene& s, double bct, double bcr, double mu)
{
    const double hg = phase_hg(s, mu), ra = phase_rayleigh(mu);
    const double fst = fs_mix(s, bct, hg, ra), fsr = fs_mix(s, bcr, hg, ra);
    const double bsr = s.w_c * bcr + s.w_a * s.beta_air, btr = bcr + s.beta_air;
    return (bsr / btr) * (fst / fsr);
}

__device__ __forceinline__ void flush_counts(unsigned long long* c, uint64_t seg, uint64_t le, uint64_t ovh)
{
    if (seg) atomicAdd(&c[0], (unsigned long long)seg);
    if (le) atomicAdd(&c[1], (unsigned long long)le);
    if (ovh) atomicAdd(&c[3], (unsigned long long)ovh);
}

}  // namespace

// ------------------------------------------------------------------ render

template <typename Real>
__global__ void __launch_bounds__(256) render_kernel(TraceArgs a, DevCams cams)
{
    const int64_t slot = a.st.first_slot + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= a.st.n_slots) return;
    const int Br = min((int)a.st.B[slot], a.brender);
    if (Br <= 0) return;
    const DevScene& s = a.s;
    const Real* __restrict__ gt = (const Real*)a.grid_tot;
    const Real* __restrict__ gd = (const Real*)a.grid_dlt;
    const float4* __restrict__ V = a.st.vtx + a.st.batch_off[slot / kWave] + (slot % kWave);
    const int nu = s.nx * s.ny * s.nz;
    const int npix = cams.W * cams.H;
    const double r2scale = 1.0 / (s.vk * s.vk);
    uint64_t nseg = 0, nle = 0;

    Vtx p0 = load_vtx(V, 0);
    double P = s.w0;           // running f/mu of the prefix (without the last vertex)
    double wprev[3] = {0.0, 0.0, 0.0};
    for (int b = 1; b <= Br; ++b) {
        const Vtx p1 = load_vtx(V, b);
        double w[3];
        const double L = seg_dir(p0, p1, w);
        // free-flight segment b-1: transmittance ratio exp(-(tau_t - tau_ref))
        const Real dt = walk_sum<Real>(s, gd, p0, w, L, nseg);
        P *= exp(-(double)dt * s.vk);
        if (b >= 2) {
            const int v = clamp_vox(p0.v, nu);
            P *= vertex_ratio(s, (double)a.bc_t[v], (double)a.st.beta_ref[v],
                              wprev[0] * w[0] + wprev[1] * w[1] + wprev[2] * w[2]);
        }
        // local estimates from x_b to every camera
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
            const Real tc = walk_sum<Real>(s, gt, p1, u, dist, nseg);
            const double c = base * fst * exp(-(double)tc * s.vk) * (r2scale / dist2);
            unsafeAtomicAdd(&a.img[(int64_t)d * npix + pix], c);
            ++nle;
        }
        wprev[0] = w[0]; wprev[1] = w[1]; wprev[2] = w[2];
        p0 = p1;
    }
    flush_counts(a.counters, nseg, nle, 0);
}

hipError_t launch_render(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c)
{
    const int64_t n = a.st.n_slots - a.st.first_slot;
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (fp64)
        render_kernel<double><<<dim3(blocks), dim3(256), 0, st>>>(a, c);
    else
        render_kernel<float><<<dim3(blocks), dim3(256), 0, st>>>(a, c);
    return hipGetLastError();
}

// Exact pixel solid angle: F(x,y) = atan(xy / (f sqrt(x^2+y^2+f^2))) is the
// solid angle of [0,x]x[0,y] on the image plane at distance f.
__device__ __forceinline__ double pixel_solid_angle(double f, int W, int H, int row, int col)
{
    auto F = [f](double x, double y) { return atan(x * y / (f * sqrt(x * x + y * y + f * f))); };
    const double x1 = col - 0.5 * W, x2 = x1 + 1.0, y1 = row - 0.5 * H, y2 = y1 + 1.0;
    return F(x2, y2) - F(x1, y2) - F(x2, y1) + F(x1, y1);
}

// images = tallies / (N Omega_p)
__global__ void __launch_bounds__(256) render_finalize_kernel(double* __restrict__ img, DevCams c, double scale)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npix = (int64_t)c.W * c.H;
    if (i >= npix * c.n) return;
    const int d = (int)(i / npix), p = (int)(i % npix);
    img[i] *= scale / pixel_solid_angle(c.f[d], c.W, c.H, p / c.W, p % c.W);
}

hipError_t launch_render_finalize(hipStream_t st, double* img, const DevCams& c, double scale)
{
    const int64_t n = (int64_t)c.W * c.H * c.n;
    render_finalize_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(img, c, scale);
    return hipGetLastError();
}

// rho = residual / (N Omega_p)
__global__ void __launch_bounds__(256) grad_prep_kernel(const double* __restrict__ res, double* __restrict__ rho,
                                                        DevCams c, double scale)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npix = (int64_t)c.W * c.H;
    if (i >= npix * c.n) return;
    const int d = (int)(i / npix), p = (int)(i % npix);
    rho[i] = res[i] * scale / pixel_solid_angle(c.f[d], c.W, c.H, p / c.W, p % c.W);
}

hipError_t launch_grad_prep(hipStream_t st, const double* residual, double* rho, const DevCams& c, double scale)
{
    const int64_t n = (int64_t)c.W * c.H * c.n;
    grad_prep_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(residual, rho, c, scale);
    return hipGetLastError();
}

// -------------------------------------------------------------------- grad

// Per path: pass 1 recomputes every contribution c_{b,d} and its weight
// w = c rho_{d,p}; it adds the connection part of the score (-l along the
// connection, the vertex term at x_b) and keeps R_b = sum_d w_{b,d}.  Pass 2
// walks the free-flight segments backwards with the suffix sums
// A_k = sum_{b>k} R_b, adding -A_k l along segment k and A_k times the
// vertex term at x_k.  Together this is sum_{b,d} w_{b,d} S(b,d) with S the
// tomography PSF of the local-estimate sub-path.
template <typename Real>
__global__ void __launch_bounds__(256) grad_kernel(TraceArgs a, DevCams cams)
{
    const int64_t slot = a.st.first_slot + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= a.st.n_slots) return;
    const int Bn = (int)a.st.B[slot];
    if (Bn <= 0) return;
    const DevScene& s = a.s;
    const Real* __restrict__ gt = (const Real*)a.grid_tot;
    const Real* __restrict__ gd = (const Real*)a.grid_dlt;
    const float4* __restrict__ V = a.st.vtx + a.st.batch_off[slot / kWave] + (slot % kWave);
    const int nu = s.nx * s.ny * s.nz;
    const int npix = cams.W * cams.H;
    const double r2scale = 1.0 / (s.vk * s.vk);
    double* __restrict__ grad = a.grad;
    uint64_t nseg = 0, novh = 0;
    double R[kMaxOrder + 1];

    Vtx p0 = load_vtx(V, 0);
    double P = s.w0;
    double wprev[3] = {0.0, 0.0, 0.0};
    for (int b = 1; b <= Bn; ++b) {
        const Vtx p1 = load_vtx(V, b);
        double w[3];
        const double L = seg_dir(p0, p1, w);
        const Real dt = walk_sum<Real>(s, gd, p0, w, L, novh);
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
            const Real tc = walk_sum<Real>(s, gt, p1, u, dist, nseg);
            const double wgt = base * fst * exp(-(double)tc * s.vk) * (r2scale / dist2) * rho;
            Rb += wgt;
            // vertex term at x_b: w * w_c f_HG / f_s,t (written as c/f_s times w_c f_HG)
            if (fst > 0.0) vert += wgt * (s.w_c * hg / fst);
            walk_scatter<Real>(s, grad, p1, u, dist, -wgt * s.vk, novh);
        }
        if (vert != 0.0) unsafeAtomicAdd(&grad[v1], vert);
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
            walk_scatter<Real>(s, grad, pk, w, L, -A * s.vk, nseg);
            if (k >= 1) {
                const Vtx pm = load_vtx(V, k - 1);
                double wm[3];
                seg_dir(pm, pk, wm);
                const double mu = wm[0] * w[0] + wm[1] * w[1] + wm[2] * w[2];
                const int v = clamp_vox(pk.v, nu);
                const double hg = phase_hg(s, mu);
                const double fst = fs_mix(s, (double)a.bc_t[v], hg, phase_rayleigh(mu));
                if (fst > 0.0) unsafeAtomicAdd(&grad[v], A * (s.w_c * hg / fst));
            }
        }
        pk1 = pk;
    }
    flush_counts(a.counters, nseg, 0, novh);
}

hipError_t launch_grad(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c)
{
    const int64_t n = a.st.n_slots - a.st.first_slot;
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (fp64)
        grad_kernel<double><<<dim3(blocks), dim3(256), 0, st>>>(a, c);
    else
        grad_kernel<float><<<dim3(blocks), dim3(256), 0, st>>>(a, c);
    return hipGetLastError();
}

// ---------------------------------------------------------------- reweight

// log r = log mu(x|beta_t) - log mu(x|beta_ref) over the whole stored path:
// every segment's optical-depth difference (the exit segment included), the
// extinction ratio at every scatter, and the direction-pdf ratio
// f_p = f_s / beta_s at every scatter that has a successor vertex.  Per-block
// sums of r and r^2 go to partial[2*block].
template <typename Real>
__global__ void __launch_bounds__(256) reweight_kernel(TraceArgs a)
{
    __shared__ double red[2][256];
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0;
    if (slot < a.st.n_slots) {
        const int nv = (int)a.st.nv[slot];
        const int Bn = (int)a.st.B[slot];
        if (nv > 0) {
            const DevScene& s = a.s;
            const Real* __restrict__ gd = (const Real*)a.grid_dlt;
            const float4* __restrict__ V = a.st.vtx + a.st.batch_off[slot / kWave] + (slot % kWave);
            const int nu = s.nx * s.ny * s.nz;
            uint64_t cnt = 0;
            double lr = 0.0;
            Vtx p0 = load_vtx(V, 0);
            double wprev[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k + 1 < nv; ++k) {
                const Vtx p1 = load_vtx(V, k + 1);
                double w[3];
                const double L = seg_dir(p0, p1, w);
                lr -= (double)walk_sum<Real>(s, gd, p0, w, L, cnt) * s.vk;
                if (k >= 1) {
                    const int v = clamp_vox(p0.v, nu);
                    const double bct = (double)a.bc_t[v], bcr = (double)a.st.beta_ref[v];
                    const double mu = wprev[0] * w[0] + wprev[1] * w[1] + wprev[2] * w[2];
                    const double hg = phase_hg(s, mu), ra = phase_rayleigh(mu);
                    const double bst = s.w_c * bct + s.w_a * s.beta_air, bsr = s.w_c * bcr + s.w_a * s.beta_air;
                    lr += log((fs_mix(s, bct, hg, ra) * bsr) / (fs_mix(s, bcr, hg, ra) * bst));
                }
                wprev[0] = w[0]; wprev[1] = w[1]; wprev[2] = w[2];
                p0 = p1;
            }
            for (int k = 1; k <= Bn; ++k) {
                const int v = clamp_vox(vox_of(V[(int64_t)k * kWave]), nu);
                lr += log(((double)a.bc_t[v] + s.beta_air) / ((double)a.st.beta_ref[v] + s.beta_air));
            }
            r = exp(lr);
        }
    }
    red[0][threadIdx.x] = r;
    red[1][threadIdx.x] = r * r;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.partial[2 * blockIdx.x] = red[0][0];
        a.partial[2 * blockIdx.x + 1] = red[1][0];
    }
}

hipError_t launch_reweight(hipStream_t st, int fp64, const TraceArgs& a, int64_t* n_blocks)
{
    const int64_t blocks = (a.st.n_slots + 255) / 256;
    *n_blocks = blocks;
    if (fp64)
        reweight_kernel<double><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(a);
    else
        reweight_kernel<float><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace prt
