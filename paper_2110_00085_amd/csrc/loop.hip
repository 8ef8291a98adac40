// Loop glue of the optimisation (Alg. 2): appearance loss and residual
// (Eq. appearance_loss), the Adam step with projection onto beta >= 0,
// fixed-order FP64 reductions, and the space-carving initialisation of the
// reconstruction (Sec. 6.1).
#include "launch.hpp"

namespace prt {

__global__ void __launch_bounds__(256) fill_kernel(double* __restrict__ p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill(hipStream_t st, double* p, int64_t n, double v)
{
    if (n <= 0) return hipSuccess;
    fill_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(p, n, v);
    return hipGetLastError();
}

constexpr int kLossItems = 4096;  // elements per block

int64_t loss_blocks(int64_t n) { return (n + kLossItems - 1) / kLossItems; }

// residual = images - target; per-block sums of residual^2 into partial[2*b]
__global__ void __launch_bounds__(256) loss_kernel(int64_t n, const double* __restrict__ img,
                                                   const double* __restrict__ tgt, double* __restrict__ res,
                                                   double* __restrict__ partial)
{
    __shared__ double red[256];
    const int64_t base = (int64_t)blockIdx.x * kLossItems;
    double s = 0.0;
    for (int j = threadIdx.x; j < kLossItems; j += blockDim.x) {
        const int64_t i = base + j;
        if (i < n) {
            const double r = img[i] - tgt[i];
            res[i] = r;
            s += r * r;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = red[0];
        partial[2 * blockIdx.x + 1] = 0.0;
    }
}

// out2[0] = scale0 * sum of partial[2i]; out2[1] = sum of partial[2i+1]
// (only when scale0 == 1); one block, fixed order.  A separate launch rather
// than a last-workgroup sum: the device-scope fence that the latter needs
// writes back the XCD's L2 in every workgroup, which cost ~60 us in the
// reweight.
__global__ void __launch_bounds__(256) sum_pairs_kernel(const double* __restrict__ partial, int64_t nb,
                                                        double* __restrict__ out2, double scale0)
{
    __shared__ double red[2][256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[0] = red[0][0] * scale0;
        if (scale0 == 1.0) out2[1] = red[1][0];
    }
}

hipError_t launch_loss(hipStream_t st, int64_t n, const double* img, const double* tgt, double* res,
                       double* partial, double* loss)
{
    const int64_t nb = loss_blocks(n);
    loss_kernel<<<dim3((unsigned)nb), dim3(256), 0, st>>>(n, img, tgt, res, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sum_pairs_kernel<<<dim3(1), dim3(256), 0, st>>>(partial, nb, loss, 0.5);
    return hipGetLastError();
}

hipError_t launch_sum_pairs(hipStream_t st, const double* partial, int64_t n_blocks, double* out2)
{
    sum_pairs_kernel<<<dim3(1), dim3(256), 0, st>>>(partial, n_blocks, out2, 1.0);
    return hipGetLastError();
}

// stats[0] = mean r = (sum r) / n, stats[1] = ess = (sum r)^2 / sum r^2 (0
// when sum r^2 is 0) from the reweight's per-workgroup pairs, summed in the
// order of sum_pairs_kernel; one block.
__global__ void __launch_bounds__(256) reweight_stats_kernel(const double* __restrict__ partial, int64_t nb,
                                                             double n, double* __restrict__ stats)
{
    __shared__ double red[2][256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double s = red[0][0], s2 = red[1][0];
        stats[0] = s / n;
        stats[1] = s2 > 0 ? s * s / s2 : 0.0;
    }
}

hipError_t launch_reweight_stats(hipStream_t st, const double* partial, int64_t n_blocks, double n_paths,
                                 double* stats)
{
    reweight_stats_kernel<<<dim3(1), dim3(256), 0, st>>>(partial, n_blocks, n_paths, stats);
    return hipGetLastError();
}

// Adam (Kingma & Ba) with bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t,
// then projection onto beta >= 0 and the FP32 copy used by the kernels.
__global__ void __launch_bounds__(256) adam_kernel(int64_t n, double* __restrict__ beta, float* __restrict__ bf,
                                                   const double* __restrict__ g, double* __restrict__ m,
                                                   double* __restrict__ v, double lr, double b1, double b2,
                                                   double eps, double bc1, double bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const double step = lr * (mi / bc1) / (sqrt(vi / bc2) + eps);
    const double nb = fmax(beta[i] - step, 0.0);
    beta[i] = nb;
    bf[i] = (float)nb;
}

hipError_t launch_adam(hipStream_t st, int64_t n, double* beta, float* beta_f32, const double* grad, double* m,
                       double* v, double lr, double b1, double b2, double eps, double bc1, double bc2)
{
    adam_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(n, beta, beta_f32, grad, m, v, lr, b1, b2,
                                                                        eps, bc1, bc2);
    return hipGetLastError();
}

// Space carving (photo hull): one thread per voxel projects the voxel centre
// into every camera (FP64 pinhole projection) and removes the voxel when a
// camera sees it on a pixel at or below that camera's threshold.
__global__ void __launch_bounds__(256) space_carve_kernel(int nx, int ny, int nz, double vk, DevCams c,
                                                          CarveThresholds t, const double* __restrict__ img,
                                                          float fill, uint8_t* __restrict__ mask,
                                                          float* __restrict__ beta)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (int64_t)nx * ny * nz) return;
    int ix, iy, iz;
    voxel_ijk((int)v, nx, ny, ix, iy, iz);
    const int64_t npix = (int64_t)c.W * c.H;
    bool keep = true;
    for (int d = 0; d < c.n; ++d) {
        const int pix = project(c, d, ix + 0.5, iy + 0.5, iz + 0.5, vk);
        if (pix >= 0 && img[d * npix + pix] <= t.t[d]) keep = false;
    }
    mask[v] = keep ? 1 : 0;
    if (beta) beta[v] = keep ? fill : 0.f;
}

// Down-sampling of pixel-averaged images by `factor` per side: coarse pixel
// (R, C) of camera d gets sum_p Omega_p I_p / sum_p Omega_p over the fine
// pixels p = (factor R + i, factor C + j), Omega_p the fine pixels' exact
// solid angles (focal length f of the fine camera).  One thread per coarse
// pixel.
__device__ __forceinline__ double solid_angle_px(double f, int W, int H, int row, int col)
{
    auto F = [f](double x, double y) { return atan(x * y / (f * sqrt(x * x + y * y + f * f))); };
    const double x1 = col - 0.5 * W, x2 = x1 + 1.0, y1 = row - 0.5 * H, y2 = y1 + 1.0;
    return F(x2, y2) - F(x1, y2) - F(x2, y1) + F(x1, y1);
}

__global__ void __launch_bounds__(256) downsample_kernel(DevCams c, int factor, const double* __restrict__ fine,
                                                         double* __restrict__ coarse)
{
    const int Wc = c.W / factor, Hc = c.H / factor;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)c.n * Wc * Hc) return;
    const int d = (int)(i / ((int64_t)Wc * Hc));
    const int rem = (int)(i % ((int64_t)Wc * Hc));
    const int R = rem / Wc, Cc = rem % Wc;
    double num = 0.0, den = 0.0;
    for (int a = 0; a < factor; ++a)
        for (int b = 0; b < factor; ++b) {
            const int row = R * factor + a, col = Cc * factor + b;
            const double om = solid_angle_px(c.f[d], c.W, c.H, row, col);
            num += om * fine[((int64_t)d * c.H + row) * c.W + col];
            den += om;
        }
    coarse[i] = num / den;
}

hipError_t launch_downsample(hipStream_t st, const DevCams& c, int factor, const double* fine, double* coarse)
{
    const int64_t n = (int64_t)c.n * (c.W / factor) * (c.H / factor);
    if (n <= 0) return hipSuccess;
    downsample_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(c, factor, fine, coarse);
    return hipGetLastError();
}

// Sec. 6 error measures: per-block sums of |t - b|, |t| and |b| (t the true
// field, b the estimate), then one block adds them in a fixed order and
// writes epsilon = sum|t - b| / sum|t| and delta = (sum|t| - sum|b|) / sum|t|.
constexpr int kErrItems = 4096;

__global__ void __launch_bounds__(256) volume_error_sums_kernel(int64_t n, const double* __restrict__ est,
                                                                const float* __restrict__ truth,
                                                                double* __restrict__ partial)
{
    __shared__ double red[3][256];
    const int64_t base = (int64_t)blockIdx.x * kErrItems;
    double a = 0.0, t = 0.0, b = 0.0;
    for (int j = threadIdx.x; j < kErrItems; j += blockDim.x) {
        const int64_t i = base + j;
        if (i < n) {
            const double x = est[i], y = (double)truth[i];
            a += fabs(y - x);
            t += fabs(y);
            b += fabs(x);
        }
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = t;
    red[2][threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) partial[3 * blockIdx.x + k] = red[k][0];
}

__global__ void __launch_bounds__(256) volume_errors_kernel(const double* __restrict__ partial, int64_t nb,
                                                            double* __restrict__ out)
{
    __shared__ double red[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x)
        for (int k = 0; k < 3; ++k) s[k] += partial[3 * i + k];
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double a = red[0][0], t = red[1][0], b = red[2][0];
        out[0] = a / t;
        out[1] = (t - b) / t;
    }
}

int64_t volume_error_blocks(int64_t n) { return (n + kErrItems - 1) / kErrItems; }

hipError_t launch_volume_errors(hipStream_t st, int64_t n, const double* est, const float* truth, double* partial,
                                double* out)
{
    const int64_t nb = volume_error_blocks(n);
    volume_error_sums_kernel<<<dim3((unsigned)nb), dim3(256), 0, st>>>(n, est, truth, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    volume_errors_kernel<<<dim3(1), dim3(256), 0, st>>>(partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_space_carve(hipStream_t st, int nx, int ny, int nz, double vk, const DevCams& c,
                              const CarveThresholds& t, const double* img, float fill, uint8_t* mask, float* beta)
{
    const int64_t nu = (int64_t)nx * ny * nz;
    space_carve_kernel<<<dim3((unsigned)((nu + 255) / 256)), dim3(256), 0, st>>>(nx, ny, nz, vk, c, t, img, fill,
                                                                               mask, beta);
    return hipGetLastError();
}

}  // namespace prt
