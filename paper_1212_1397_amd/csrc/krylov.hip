// Vector kernels of the Krylov loops (GMRES Arnoldi with modified
// Gram-Schmidt, cycle updates, SKS updates), complex128.
//
// Reductions are deterministic: a fixed grid of kRedBlocks blocks writes one
// partial per block (grid-stride order fixed), and a single-block kernel sums
// the partials in a fixed tree order.  The inner products stay on the device;
// only Hessenberg columns and residual norms are copied to the host.
#include "h6_internal.h"

namespace h6 {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block-level sum of (a, b) into partials[2*blockIdx.x + {0,1}].
__device__ __forceinline__ void block_store2(double a, double b, double* partials) {
  __shared__ double sa[kThreads / 64], sb[kThreads / 64];
  a = warp_sum(a);
  b = warp_sum(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sa[w] = a; sb[w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) { ta += sa[i]; tb += sb[i]; }
    partials[2 * blockIdx.x] = ta;
    partials[2 * blockIdx.x + 1] = tb;
  }
}

// partial sum of conj(a) * b
__global__ __launch_bounds__(kThreads) void dot_kernel(const double2* __restrict__ a,
                                                       const double2* __restrict__ b, size_t n,
                                                       double* __restrict__ partials) {
  double re = 0.0, im = 0.0;
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    const double2 u = a[i], v = b[i];
    re = fma(u.x, v.x, fma(u.y, v.y, re));
    im = fma(u.x, v.y, fma(-u.y, v.x, im));
  }
  block_store2(re, im, partials);
}

// w -= h * vprev (if vprev), then partial conj(vcur) * w (if vcur) or |w|^2.
__global__ __launch_bounds__(kThreads) void mgs_kernel(double2* __restrict__ w,
                                                       const double2* __restrict__ vprev,
                                                       const double2* __restrict__ hprev,
                                                       const double2* __restrict__ vcur, size_t n,
                                                       double* __restrict__ partials) {
  double2 h = make_double2(0.0, 0.0);
  if (vprev) h = *hprev;
  double re = 0.0, im = 0.0;
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    double2 x = w[i];
    if (vprev) {
      const double2 v = vprev[i];
      x.x -= h.x * v.x - h.y * v.y;
      x.y -= h.x * v.y + h.y * v.x;
      w[i] = x;
    }
    if (vcur) {
      const double2 u = vcur[i];
      re = fma(u.x, x.x, fma(u.y, x.y, re));
      im = fma(u.x, x.y, fma(-u.y, x.x, im));
    } else {
      re = fma(x.x, x.x, fma(x.y, x.y, re));
    }
  }
  block_store2(re, im, partials);
}

__global__ __launch_bounds__(kThreads) void reduce_kernel(const double* __restrict__ partials,
                                                          int nparts, int ncomp,
                                                          double2* __restrict__ out) {
  __shared__ double sa[kThreads], sb[kThreads];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) {
    a += partials[ncomp * i];
    if (ncomp == 2) b += partials[2 * i + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = make_double2(sa[0], sb[0]);
}

__global__ __launch_bounds__(kThreads) void scale_kernel(double2* v, const double2* src,
                                                         const double2* __restrict__ nrm, size_t n) {
  const double s = 1.0 / sqrt(nrm->x);
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    const double2 x = src[i];
    v[i] = make_double2(x.x * s, x.y * s);
  }
}

// out (+)= sum_i y_i V_i, V_i = V + i * n
__global__ __launch_bounds__(kThreads) void multi_axpy_kernel(double2* __restrict__ out,
                                                              const double2* __restrict__ V,
                                                              const double2* __restrict__ y, int m,
                                                              size_t n, int accumulate) {
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    double2 acc = accumulate ? out[i] : make_double2(0.0, 0.0);
    for (int j = 0; j < m; ++j) {
      const double2 c = y[j], v = V[size_t(j) * n + i];
      acc.x += c.x * v.x - c.y * v.y;
      acc.y += c.x * v.y + c.y * v.x;
    }
    out[i] = acc;
  }
}

__global__ __launch_bounds__(kThreads) void add_kernel(double2* __restrict__ U,
                                                       const double2* __restrict__ z, size_t n) {
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    const double2 a = U[i], b = z[i];
    U[i] = make_double2(a.x + b.x, a.y + b.y);
  }
}

int grid_for(size_t n) {
  const size_t b = (n + kThreads - 1) / kThreads;
  return int(b < size_t(kRedBlocks) ? (b > 0 ? b : 1) : kRedBlocks);
}

}  // namespace

hipError_t launch_dot_partials(const double2* a, const double2* b, size_t n, double* partials,
                               hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(kRedBlocks), dim3(kThreads), 0, s, a, b, n, partials);
  return hipGetLastError();
}

hipError_t launch_mgs_step(double2* w, const double2* vprev, const double2* hprev,
                           const double2* vcur, size_t n, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(mgs_kernel, dim3(kRedBlocks), dim3(kThreads), 0, s, w, vprev, hprev, vcur, n,
                     partials);
  return hipGetLastError();
}

hipError_t launch_norm2_partials(const double2* a, size_t n, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(mgs_kernel, dim3(kRedBlocks), dim3(kThreads), 0, s, const_cast<double2*>(a),
                     nullptr, nullptr, nullptr, n, partials);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nparts, int ncomp, double2* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, partials, nparts, ncomp, out);
  return hipGetLastError();
}

hipError_t launch_axpy_norm(double2* w, const double2* v, const double2* h, size_t n,
                            double* partials, hipStream_t s) {
  hipLaunchKernelGGL(mgs_kernel, dim3(kRedBlocks), dim3(kThreads), 0, s, w, v, h, nullptr, n,
                     partials);
  return hipGetLastError();
}

hipError_t launch_scale_inv_norm(double2* v, const double2* src, const double2* nrm, size_t n,
                                 hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, v, src, nrm, n);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(double2* out, const double2* V, const double2* y, int m, size_t n,
                             int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, out, V, y, m, n,
                     accumulate);
  return hipGetLastError();
}

hipError_t launch_add(double2* U, const double2* z, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(add_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, U, z, n);
  return hipGetLastError();
}

}  // namespace h6
