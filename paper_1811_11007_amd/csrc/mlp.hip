// mlp.hip -- the warm-start network: a two-layer perceptron trained and
// evaluated by these kernels alone (no GEMM library).
//
//   h = tanh(x W1 + b1)      x: [rows][n_in], W1: [n_in][n_hidden]
//   y = h W2 + b2            W2: [n_hidden][n_out]
//
// Parameters live in one FP32 array packed as W1, b1, W2, b2 (row-major).
// Training minimises the mean over rows and outputs of (y - target)^2 with
// Adam.  Weight gradients are sums over rows; each is formed by one block in
// a fixed order (per-thread strided partial sums in FP64, then a fixed tree),
// so training is deterministic.  Matrices are small (n_in ~ 16, n_hidden
// 128, n_out 5): the work is one thread per output element with the weights
// read through the cache, and per-row activations kept for the backward pass.
#include <hip/hip_runtime.h>

#include "mlp.hpp"

namespace pt {
namespace {

__global__ void k_mlp_hidden(const float *x, const float *p, int rows, int ni, int nh, float *hact) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)rows * nh) return;
    const int r = (int)(g / nh), h = (int)(g % nh);
    const float *W1 = p, *b1 = p + (size_t)ni * nh;
    float z = b1[h];
    for (int f = 0; f < ni; ++f) z += x[(size_t)r * ni + f] * W1[(size_t)f * nh + h];
    hact[g] = tanhf(z);
}

__global__ void k_mlp_out(const float *hact, const float *p, int rows, int ni, int nh, int no, float *y) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)rows * no) return;
    const int r = (int)(g / no), o = (int)(g % no);
    const float *W2 = p + (size_t)ni * nh + nh, *b2 = W2 + (size_t)nh * no;
    float s = b2[o];
    for (int h = 0; h < nh; ++h) s += hact[(size_t)r * nh + h] * W2[(size_t)h * no + o];
    y[g] = s;
}

// dY = 2 (y - target) / (rows * no); loss partial sums per row.
__global__ void k_mlp_dy(const float *y, const float *t, int rows, int no, float *dy, double *row_loss) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double l = 0.0;
    const float scale = 2.0f / ((float)rows * (float)no);
    for (int o = 0; o < no; ++o) {
        const float d = y[(size_t)r * no + o] - t[(size_t)r * no + o];
        dy[(size_t)r * no + o] = d * scale;
        l += (double)d * d;
    }
    if (row_loss) row_loss[r] = l;
}

// dZ = (dY W2^T) * (1 - h^2): gradient at the hidden pre-activations.
__global__ void k_mlp_dz(const float *dy, const float *hact, const float *p, int rows, int ni, int nh, int no,
                         float *dz) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)rows * nh) return;
    const int r = (int)(g / nh), h = (int)(g % nh);
    const float *W2 = p + (size_t)ni * nh + nh;
    float s = 0.0f;
    for (int o = 0; o < no; ++o) s += dy[(size_t)r * no + o] * W2[(size_t)h * no + o];
    const float a = hact[g];
    dz[g] = s * (1.0f - a * a);
}

// Fixed-order block sum (256 threads) of FP64 partials.
__device__ inline double block_sum256(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// One block per parameter: the sum over rows of its gradient terms.
//   W1[f][h] += x[r][f] dz[r][h];  b1[h] += dz[r][h];
//   W2[h][o] += hact[r][h] dy[r][o];  b2[o] += dy[r][o].
__global__ void __launch_bounds__(256) k_mlp_wgrad(const float *x, const float *hact, const float *dz,
                                                    const float *dy, int rows, int ni, int nh, int no, float *grad) {
    __shared__ double sh[256];
    const int q = blockIdx.x;
    const int n_w1 = ni * nh, n_b1 = nh, n_w2 = nh * no;
    const float *A;
    const float *Bv;
    int sa, sb;  // row strides; A/B point at the element of row 0
    if (q < n_w1) {
        const int f = q / nh, h = q % nh;
        A = x + f; sa = ni;
        Bv = dz + h; sb = nh;
    } else if (q < n_w1 + n_b1) {
        const int h = q - n_w1;
        A = nullptr; sa = 0;
        Bv = dz + h; sb = nh;
    } else if (q < n_w1 + n_b1 + n_w2) {
        const int k = q - n_w1 - n_b1, h = k / no, o = k % no;
        A = hact + h; sa = nh;
        Bv = dy + o; sb = no;
    } else {
        const int o = q - n_w1 - n_b1 - n_w2;
        A = nullptr; sa = 0;
        Bv = dy + o; sb = no;
    }
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += 256)
        s += (double)(A ? A[(size_t)r * sa] : 1.0f) * (double)Bv[(size_t)r * sb];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) grad[q] = (float)s;
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_sum_rows(const double *row_loss, int rows, double *out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += 256) s += row_loss[r];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) *out = s;
}

// brlen[pos[r][o]] = clamp((max(base[r][o], 0) + shift) * exp(y[r][o]) - shift,
// t_min, t_max) for pos >= 0: the network predicts log-ratios of shifted new
// and parent lengths.
__global__ void k_warm_apply(const float *y, const int32_t *pos, const double *base, int rows, int no, double shift,
                             double t_min, double t_max, double *brlen) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)rows * no) return;
    const int32_t at = pos[g];
    if (at < 0) return;
    const double v = (fmax(base[g], 0.0) + shift) * exp((double)y[g]) - shift;
    brlen[at] = fmin(fmax(v, t_min), t_max);
}

unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t mlp_forward(const float *x, const float *p, int rows, int ni, int nh, int no, float *hact, float *y,
                       hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_hidden, dim3(blocks((int64_t)rows * nh, 256)), dim3(256), 0, s, x, p, rows, ni, nh, hact);
    hipLaunchKernelGGL(k_mlp_out, dim3(blocks((int64_t)rows * no, 256)), dim3(256), 0, s, hact, p, rows, ni, nh, no, y);
    return hipGetLastError();
}

hipError_t mlp_backward(const float *x, const float *p, const float *hact, const float *dy, int rows, int ni, int nh,
                        int no, float *dz, float *grad, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_dz, dim3(blocks((int64_t)rows * nh, 256)), dim3(256), 0, s, dy, hact, p, rows, ni, nh,
                       no, dz);
    const int np = ni * nh + nh + nh * no + no;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(np), dim3(256), 0, s, x, hact, dz, dy, rows, ni, nh, no, grad);
    return hipGetLastError();
}

hipError_t mlp_loss_grad(const float *y, const float *t, int rows, int no, float *dy, double *row_loss,
                         double *loss, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_dy, dim3(blocks(rows, 256)), dim3(256), 0, s, y, t, rows, no, dy, row_loss);
    if (loss) hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, row_loss, rows, loss);
    return hipGetLastError();
}

hipError_t mlp_warm_apply(const float *y, const int32_t *pos, const double *base, int rows, int no, double shift,
                          double t_min, double t_max, double *brlen, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_warm_apply, dim3(blocks((int64_t)rows * no, 256)), dim3(256), 0, s, y, pos, base, rows, no,
                       shift, t_min, t_max, brlen);
    return hipGetLastError();
}

hipError_t mlp_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(blocks(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace pt
