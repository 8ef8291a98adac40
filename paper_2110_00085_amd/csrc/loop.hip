// Loop glue of the optimisation (Alg. 2): appearance loss and residual
// (Eq. appearance_loss), the Adam step with projection onto beta >= 0, and
// fixed-order FP64 reductions.
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
                                                   double* __restrict__ partial, double* __restrict__ loss,
                                                   unsigned int* __restrict__ done)
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
    // the last workgroup writes 0.5 * sum of squares
    finish_pairs(partial, loss, 0.5, false, done);
}

hipError_t launch_loss(hipStream_t st, int64_t n, const double* img, const double* tgt, double* res,
                       double* partial, double* loss, unsigned int* done)
{
    const int64_t nb = loss_blocks(n);
    loss_kernel<<<dim3((unsigned)nb), dim3(256), 0, st>>>(n, img, tgt, res, partial, loss, done);
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

}  // namespace prt
