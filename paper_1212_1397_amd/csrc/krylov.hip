// Vector kernels of the Krylov loops, complex128.
//
// GMRES orthogonalisation is modified Gram-Schmidt written in its inverse
// compact WY form: for a new vector w and an (unnormalised) basis Q, one pass
// forms all inner products <q_i, w>; the host turns them into the MGS
// coefficients with the Gram matrix of the basis (a small triangular solve);
// one more pass applies w -= sum_i c_i q_i and, while the basis streams by,
// forms |w|^2 and the Gram row <q_i, w> of the new basis vector.  This moves
// (2j + 4) vectors per Arnoldi step instead of (4j + 5) for the
// one-projection-per-pass form, with the same coefficients in exact
// arithmetic.
//
// Reductions are deterministic: a fixed grid (one full wave of resident
// blocks) writes one partial per block and component in grid-stride order,
// and a second kernel sums each component's partials in a fixed tree order.
#include "h6_internal.h"

namespace h6 {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block sum of NV per-thread values; partials laid out [component][block].
template <int NV>
__device__ __forceinline__ void block_store(double (&v)[NV], double* partials, int comp0,
                                            int nblocks) {
  __shared__ double s[kThreads / 64][NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) v[c] = warp_sum(v[c]);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) s[w][c] = v[c];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < NV; c += kThreads) {
    double t = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) t += s[i][c];
    partials[size_t(comp0 + c) * nblocks + blockIdx.x] = t;
  }
}

// |a|^2 partials (component 0)
__global__ __launch_bounds__(kThreads) void norm2_kernel(const double2* __restrict__ a, size_t n,
                                                         double* __restrict__ partials) {
  double v[1] = {0.0};
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    const double2 x = a[i];
    v[0] = fma(x.x, x.x, fma(x.y, x.y, v[0]));
  }
  block_store<1>(v, partials, 0, gridDim.x);
}

// For basis vectors q_{i0 .. i0+cnt-1} (stride n from Q): partials of
// <q_i, w> (components 2 i, 2 i + 1 = re, im).
template <int CH>
__global__ __launch_bounds__(kThreads) void block_dots_kernel(const double2* __restrict__ Q, int i0,
                                                              int cnt, const double2* __restrict__ w,
                                                              size_t n, double* __restrict__ partials) {
  double acc[2 * CH];
#pragma unroll
  for (int c = 0; c < 2 * CH; ++c) acc[c] = 0.0;
  for (size_t k = blockIdx.x * size_t(kThreads) + threadIdx.x; k < n; k += size_t(gridDim.x) * kThreads) {
    const double2 x = w[k];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      if (i < cnt) {
        const double2 q = Q[size_t(i0 + i) * n + k];
        acc[2 * i] = fma(q.x, x.x, fma(q.y, x.y, acc[2 * i]));
        acc[2 * i + 1] = fma(q.x, x.y, fma(-q.y, x.x, acc[2 * i + 1]));
      }
    }
  }
  block_store<2 * CH>(acc, partials, 2 * i0, gridDim.x);
}

// w -= sum_{i < m} c_i q_i, then partials of |w|^2 (component 0) and of
// <q_i, w> for i < min(m, CH) (components 1 + 2 i, 2 + 2 i): the Gram row of
// the new basis vector w, formed while the basis is streamed for the update.
template <int CH>
__global__ __launch_bounds__(kThreads) void update_gram_kernel(double2* __restrict__ w,
                                                               const double2* __restrict__ Q,
                                                               const double2* __restrict__ c, int m,
                                                               size_t n, double* __restrict__ partials) {
  double acc[1 + 2 * CH];
#pragma unroll
  for (int i = 0; i < 1 + 2 * CH; ++i) acc[i] = 0.0;
  const int mg = m < CH ? m : CH;
  for (size_t k = blockIdx.x * size_t(kThreads) + threadIdx.x; k < n; k += size_t(gridDim.x) * kThreads) {
    double2 x = w[k];
    double2 q[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      if (i < mg) {
        q[i] = Q[size_t(i) * n + k];
        const double2 a = c[i];
        x.x -= a.x * q[i].x - a.y * q[i].y;
        x.y -= a.x * q[i].y + a.y * q[i].x;
      }
    }
    for (int i = CH; i < m; ++i) {
      const double2 a = c[i], qq = Q[size_t(i) * n + k];
      x.x -= a.x * qq.x - a.y * qq.y;
      x.y -= a.x * qq.y + a.y * qq.x;
    }
    w[k] = x;
    acc[0] = fma(x.x, x.x, fma(x.y, x.y, acc[0]));
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      if (i < mg) {
        acc[1 + 2 * i] = fma(q[i].x, x.x, fma(q[i].y, x.y, acc[1 + 2 * i]));
        acc[2 + 2 * i] = fma(q[i].x, x.y, fma(-q[i].y, x.x, acc[2 + 2 * i]));
      }
    }
  }
  block_store<1 + 2 * CH>(acc, partials, 0, gridDim.x);
}

// out[c] = sum_b partials[c * nblocks + b], one block per component
__global__ __launch_bounds__(kThreads) void reduce_cols_kernel(const double* __restrict__ partials,
                                                               int nblocks, double* __restrict__ out) {
  __shared__ double s[kThreads];
  double a = 0.0;
  const double* p = partials + size_t(blockIdx.x) * nblocks;
  for (int i = threadIdx.x; i < nblocks; i += kThreads) a += p[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

// out (+)= sum_i y_i V_i, V_i = V + i * n (FP64 arithmetic)
template <typename TV>
__global__ __launch_bounds__(kThreads) void multi_axpy_kernel(double2* __restrict__ out,
                                                              const TV* __restrict__ V,
                                                              const double2* __restrict__ y, int m,
                                                              size_t n, int accumulate) {
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    double2 acc = accumulate ? out[i] : make_double2(0.0, 0.0);
    for (int j = 0; j < m; ++j) {
      const double2 c = y[j];
      const TV vv = V[size_t(j) * n + i];
      const double2 v = make_double2(double(vv.x), double(vv.y));
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

constexpr int kDotChunk = 16;
constexpr int kGramChunk = kGramMax;

}  // namespace

hipError_t launch_norm2(const double2* a, size_t n, double* partials, double* out, hipStream_t s) {
  hipLaunchKernelGGL(norm2_kernel, dim3(kRedBlocks), dim3(kThreads), 0, s, a, n, partials);
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(1), dim3(kThreads), 0, s, partials, kRedBlocks, out);
  return hipGetLastError();
}

hipError_t launch_reduce_sum(const double* partials, int nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(1), dim3(kThreads), 0, s, partials, nparts, out);
  return hipGetLastError();
}

int reduction_blocks() {
  static int blocks = 0;
  if (!blocks) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, block_dots_kernel<kDotChunk>, kThreads, 0) !=
            hipSuccess || cus <= 0 || per <= 0)
      blocks = kRedBlocks;
    else
      blocks = cus * per;      // one full wave of resident blocks, no tail
    if (blocks > kRedBlocks * 2) blocks = kRedBlocks * 2;   // partials capacity: 514 x 2048
  }
  return blocks;
}

hipError_t launch_block_dots(const double2* Q, int m, const double2* w, size_t n, double* partials,
                             double* out, hipStream_t s) {
  const int nb = reduction_blocks();
  for (int i0 = 0; i0 < m; i0 += kDotChunk) {
    const int cnt = m - i0 < kDotChunk ? m - i0 : kDotChunk;
    hipLaunchKernelGGL(block_dots_kernel<kDotChunk>, dim3(nb), dim3(kThreads), 0, s, Q, i0, cnt, w, n,
                       partials);
  }
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(2 * m), dim3(kThreads), 0, s, partials, nb, out);
  return hipGetLastError();
}

hipError_t launch_update_gram(double2* w, const double2* Q, const double2* c, int m, size_t n,
                              double* partials, double* out, hipStream_t s) {
  const int nb = reduction_blocks();
  hipLaunchKernelGGL(update_gram_kernel<kGramChunk>, dim3(nb), dim3(kThreads), 0, s, w, Q, c, m, n,
                     partials);
  const int mg = m < kGramChunk ? m : kGramChunk;
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(1 + 2 * mg), dim3(kThreads), 0, s, partials, nb, out);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(double2* out, const double2* V, const double2* y, int m, size_t n,
                             int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(multi_axpy_kernel<double2>, dim3(grid_for(n)), dim3(kThreads), 0, s, out, V, y, m,
                     n, accumulate);
  return hipGetLastError();
}

hipError_t launch_multi_axpy_f32(double2* out, const float2* V, const double2* y, int m, size_t n,
                                 int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(multi_axpy_kernel<float2>, dim3(grid_for(n)), dim3(kThreads), 0, s, out, V, y, m,
                     n, accumulate);
  return hipGetLastError();
}

hipError_t launch_add(double2* U, const double2* z, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(add_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, U, z, n);
  return hipGetLastError();
}

}  // namespace h6
