// mlp.hpp -- launch wrappers of the warm-start network kernels (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pt {

// hact[rows][nh] = tanh(x W1 + b1); y[rows][no] = hact W2 + b2.
hipError_t mlp_forward(const float *x, const float *p, int rows, int ni, int nh, int no, float *hact, float *y,
                       hipStream_t s);
// dy = d(mean squared error)/dy; row_loss[r] = sum_o (y - t)^2; *loss = sum.
hipError_t mlp_loss_grad(const float *y, const float *t, int rows, int no, float *dy, double *row_loss,
                         double *loss, hipStream_t s);
// grad (packed like the parameters) from dy, the inputs and the activations.
// part: FP64 workspace of mlp_wgrad_part_doubles(rows, ...) doubles for the
// row-tiled weight gradient (0 when the network's row tile does not fit the
// LDS limit; part may then be NULL).
constexpr size_t kMlpTileLdsMax = 48 * 1024;
size_t mlp_wgrad_part_doubles(int rows, int ni, int nh, int no);
hipError_t mlp_backward(const float *x, const float *p, const float *hact, const float *dy, int rows, int ni, int nh,
                        int no, float *dz, float *grad, double *part, hipStream_t s);
// brlen[pos] = clamp((max(base, 0) + shift) * exp(y) - shift, t_min, t_max) where pos >= 0.
hipError_t mlp_warm_apply(const float *y, const int32_t *pos, const double *base, int rows, int no, double shift,
                          double t_min, double t_max, double *brlen, hipStream_t s);
// Adam step with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t.
hipError_t mlp_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s);

}  // namespace pt
