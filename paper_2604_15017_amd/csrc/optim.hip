// Inverse loop on the device: the clip-and-scale parameterisation (Eq. clip01,
// Eq. scale_phys) and one Adam step (Eq. adam) with the clip derivative
// (Eq. clip_grad) and global-norm gradient clipping. One block does the whole
// vector so that the norm and the update need no second launch.
#include "kernels.h"

namespace usrt {

namespace {

__global__ __launch_bounds__(256) void k_param_map(const double* __restrict__ u, const double* __restrict__ lo,
                                                   const double* __restrict__ hi, int n,
                                                   double* __restrict__ theta) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double un = fmin(fmax(u[j], 0.0), 1.0);
  theta[j] = lo[j] == hi[j] ? lo[j] : lo[j] + un * (hi[j] - lo[j]);
}

__device__ __forceinline__ double unconstrained_grad(double g, double u, double lo, double hi) {
  return (u > 0.0 && u < 1.0 && lo < hi) ? g * (hi - lo) : 0.0;
}

__global__ __launch_bounds__(1024) void k_adam(double* __restrict__ u, double* __restrict__ m,
                                               double* __restrict__ v, const double* __restrict__ g,
                                               const double* __restrict__ lo, const double* __restrict__ hi,
                                               const double* __restrict__ lr, int n, int step, double b1,
                                               double b2, double eps, double max_norm) {
  __shared__ double red[1024];
  double ss = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double gu = unconstrained_grad(g[j], u[j], lo[j], hi[j]);
    ss += gu * gu;
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double norm = sqrt(red[0]);
  const double scale = (max_norm > 0.0 && norm > max_norm) ? max_norm / norm : 1.0;
  const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double gu = unconstrained_grad(g[j], u[j], lo[j], hi[j]) * scale;
    const double mj = b1 * m[j] + (1.0 - b1) * gu;
    const double vj = b2 * v[j] + (1.0 - b2) * gu * gu;
    m[j] = mj;
    v[j] = vj;
    u[j] -= lr[j] * (mj / c1) / (sqrt(vj / c2) + eps);
  }
}

}  // namespace

void launch_param_map(const double* u, const double* lo, const double* hi, int n, double* theta,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_param_map, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, u, lo, hi, n, theta);
}

void launch_adam(double* u, double* m, double* v, const double* g, const double* lo, const double* hi,
                 const double* lr, int n, int step, double b1, double b2, double eps, double max_norm,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(1), dim3(1024), 0, s, u, m, v, g, lo, hi, lr, n, step, b1, b2, eps, max_norm);
}

}  // namespace usrt
