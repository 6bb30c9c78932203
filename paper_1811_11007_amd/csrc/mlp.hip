// mlp.hip -- the warm-start network: a two-layer perceptron trained and
// evaluated by these kernels alone (no GEMM library).
//
//   h = tanh(x W1 + b1)      x: [rows][n_in], W1: [n_in][n_hidden]
//   y = h W2 + b2            W2: [n_hidden][n_out]
//
// Parameters live in one FP32 array packed as W1, b1, W2, b2 (row-major).
// Training minimises the mean over rows and outputs of (y - target)^2 with
// Adam.  Weight gradients are sums over rows, formed in a fixed order, so
// training is deterministic: blocks of 32 rows staged in LDS, each block's
// sums in FP64 and the blocks added in order (a network whose
// staging exceeds 48 KiB of LDS: one block per parameter, per-thread strided
// partial sums in FP64, then a fixed tree).  Matrices are small (n_in ~ 16,
// n_hidden 128, n_out 5): the hidden layer is one thread per element with
// the weights read through the cache; the output layer stages 64 rows of
// activations and the weights in LDS; per-row activations are kept for the
// backward pass.
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

// The output layer by row tiles: a block stages 64 rows of h and all of W2
// and b2 in LDS (coalesced), then each thread forms outputs from LDS; the
// same sums in the same order as k_mlp_out.
constexpr int kOutRows = 64;

__global__ void __launch_bounds__(256) k_mlp_out_tiles(const float *hact, const float *p, int rows, int ni, int nh,
                                                        int no, float *y) {
    extern __shared__ float tile[];
    // rows padded by one word, so the lanes of a wave (several rows) read
    // different LDS banks
    const int ld = nh + 1;
    float *th = tile, *tw = th + kOutRows * ld, *tb = tw + (size_t)nh * no;
    const float *W2 = p + (size_t)ni * nh + nh, *b2 = W2 + (size_t)nh * no;
    const int r0 = blockIdx.x * kOutRows;
    const int nr = min(kOutRows, rows - r0);
    for (int i = threadIdx.x; i < nr * nh; i += 256) th[(i / nh) * ld + i % nh] = hact[(size_t)r0 * nh + i];
    for (int i = threadIdx.x; i < nh * no; i += 256) tw[i] = W2[i];
    for (int i = threadIdx.x; i < no; i += 256) tb[i] = b2[i];
    __syncthreads();
    for (int g = threadIdx.x; g < nr * no; g += 256) {
        const int r = g / no, o = g % no;
        float s = tb[o];
        for (int h = 0; h < nh; ++h) s += th[r * ld + h] * tw[h * no + o];
        y[(size_t)r0 * no + g] = s;
    }
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

// Weight gradients by row tiles: block b sums the terms of its 32 rows for
// every parameter, from their rows of x, h, dz and dy staged in LDS
// (instead of one block per parameter re-reading every row), and
// writes them to part[b][np] in FP64; k_mlp_wgrad_sum then adds the blocks
// in order.  Each sum runs over the rows in order; a thread accumulates its
// parameters across the stagings in its own entries of part.
constexpr int kWgradRows = 32;  // rows staged in LDS at a time
constexpr int kWgradSub = 1;    // stagings per block

__global__ void __launch_bounds__(256) k_mlp_wgrad_tiles(const float *x, const float *hact, const float *dz,
                                                          const float *dy, int rows, int ni, int nh, int no,
                                                          double *part) {
    extern __shared__ float tile[];
    float *tx = tile, *th = tx + kWgradRows * ni, *tz = th + kWgradRows * nh, *ty = tz + kWgradRows * nh;
    const int n_w1 = ni * nh, n_b1 = nh, n_w2 = nh * no;
    const int np = n_w1 + n_b1 + n_w2 + no;
    for (int sub = 0; sub < kWgradSub; ++sub) {
        const int r0 = (blockIdx.x * kWgradSub + sub) * kWgradRows;
        if (r0 >= rows) break;  // uniform
        const int nr = min(kWgradRows, rows - r0);
        if (sub > 0) __syncthreads();  // the previous staging is read
        for (int i = threadIdx.x; i < nr * ni; i += 256) tx[i] = x[(size_t)r0 * ni + i];
        for (int i = threadIdx.x; i < nr * nh; i += 256) {
            th[i] = hact[(size_t)r0 * nh + i];
            tz[i] = dz[(size_t)r0 * nh + i];
        }
        for (int i = threadIdx.x; i < nr * no; i += 256) ty[i] = dy[(size_t)r0 * no + i];
        __syncthreads();
        for (int q = threadIdx.x; q < np; q += 256) {
            double s = 0.0;
            if (q < n_w1) {
                const int f = q / nh, h = q % nh;
                for (int r = 0; r < nr; ++r) s += (double)tx[r * ni + f] * (double)tz[r * nh + h];
            } else if (q < n_w1 + n_b1) {
                const int h = q - n_w1;
                for (int r = 0; r < nr; ++r) s += (double)tz[r * nh + h];
            } else if (q < n_w1 + n_b1 + n_w2) {
                const int k = q - n_w1 - n_b1, h = k / no, o = k % no;
                for (int r = 0; r < nr; ++r) s += (double)th[r * nh + h] * (double)ty[r * no + o];
            } else {
                const int o = q - n_w1 - n_b1 - n_w2;
                for (int r = 0; r < nr; ++r) s += (double)ty[r * no + o];
            }
            // the block's sum over its stagings, in order
            double *out = part + (size_t)blockIdx.x * np + q;
            *out = sub == 0 ? s : *out + s;
        }
    }
}

__global__ void k_mlp_wgrad_sum(const double *part, int tiles, int np, float *grad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    double s = 0.0;
    int b = 0;
    for (; b + 8 <= tiles; b += 8) {  // eight loads in flight, added in order
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(b + u) * np + q];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; b < tiles; ++b) s += part[(size_t)b * np + q];
    grad[q] = (float)s;
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
    const size_t lds = sizeof(float) * ((size_t)kOutRows * (nh + 1) + (size_t)nh * no + no);
    if (lds <= kMlpTileLdsMax)
        hipLaunchKernelGGL(k_mlp_out_tiles, dim3(blocks(rows, kOutRows)), dim3(256), lds, s, hact, p, rows, ni, nh, no,
                           y);
    else
        hipLaunchKernelGGL(k_mlp_out, dim3(blocks((int64_t)rows * no, 256)), dim3(256), 0, s, hact, p, rows, ni, nh, no,
                           y);
    return hipGetLastError();
}

size_t mlp_wgrad_tile_lds(int ni, int nh, int no) {
    return sizeof(float) * kWgradRows * ((size_t)ni + 2 * (size_t)nh + (size_t)no);
}

size_t mlp_wgrad_part_doubles(int rows, int ni, int nh, int no) {
    if (mlp_wgrad_tile_lds(ni, nh, no) > kMlpTileLdsMax) return 0;
    const int tiles = (rows + kWgradRows * kWgradSub - 1) / (kWgradRows * kWgradSub);
    return (size_t)tiles * ((size_t)ni * nh + nh + (size_t)nh * no + no);
}

hipError_t mlp_backward(const float *x, const float *p, const float *hact, const float *dy, int rows, int ni, int nh,
                        int no, float *dz, float *grad, double *part, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_dz, dim3(blocks((int64_t)rows * nh, 256)), dim3(256), 0, s, dy, hact, p, rows, ni, nh,
                       no, dz);
    const int np = ni * nh + nh + nh * no + no;
    const size_t lds = mlp_wgrad_tile_lds(ni, nh, no);
    if (part && lds <= kMlpTileLdsMax) {
        const int tiles = (rows + kWgradRows * kWgradSub - 1) / (kWgradRows * kWgradSub);
        hipLaunchKernelGGL(k_mlp_wgrad_tiles, dim3(tiles), dim3(256), lds, s, x, hact, dz, dy, rows, ni, nh, no, part);
        hipLaunchKernelGGL(k_mlp_wgrad_sum, dim3(blocks(np, 64)), dim3(64), 0, s, part, tiles, np, grad);
    } else {
        hipLaunchKernelGGL(k_mlp_wgrad, dim3(np), dim3(256), 0, s, x, hact, dz, dy, rows, ni, nh, no, grad);
    }
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
