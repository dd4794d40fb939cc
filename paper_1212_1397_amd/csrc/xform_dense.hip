// Sine / cosine transforms of Section 3.3 as dense products on the matrix
// cores, for the axes whose period parameter M has no fast path here (every
// M but 257).  Along an axis with L unknowns the transform of each line is
// out_m = sum_q W[m][q] in_q with the L x L basis matrix W of the plan (scale
// factors folded in: see build_dense_matrices), so a whole pass is one GEMM
// per z-plane (y) or per block of lines (x):
//   y: C[m][c] = sum_q W[m][q] X[q][c],   X = the plane as L x 2n'x reals
//      (row q = y index; real and imaginary parts of each x are columns);
//   x: C[r][m] = sum_q X[r][q] W[m][q],   rows r = (line, real or imaginary part).
// Complex data times a real matrix needs no extra flops.  One MFMA tile is
// 16 x 16 with K = 4 (v_mfma_f32_16x16x4f32 in complex64 plans,
// v_mfma_f64_16x16x4f64 in complex128 ones); a workgroup of 4 waves owns a
// 64 x 64 output tile and stages 16-wide K chunks of both operands in LDS.
// W is stored zero-padded to [Lm][Lq] (Lm a multiple of 64, Lq of 16), so
// operand reads of W need no bounds checks.
#include "h6_internal.h"

namespace h6 {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// MFMA 16x16x4: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and
// receives D[row(l, e)][l % 16], e = 0..3 (layouts checked on gfx950).
template <typename R> struct Mma;
template <> struct Mma<float> {
  using V = f32x4;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int e) { return 4 * (l >> 4) + e; }
  // x pass: row of (line li of the 16-row tile, part c) so that each lane's
  // four outputs are two whole complex values (lines 2g, 2g + 1)
  static __device__ __forceinline__ int xrow(int li, int c) { return 2 * li + c; }
};
template <> struct Mma<double> {
  using V = f64x4;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int e) { return 4 * e + (l >> 4); }
  // lines g and g + 4 (re in rows 0..7, im in rows 8..15)
  static __device__ __forceinline__ int xrow(int li, int c) { return li + 8 * c; }
};

constexpr int kT = 64;       // output tile edge
constexpr int kKC = 16;      // K chunk staged per step
constexpr int kPad = kKC + 1;

template <typename R, typename Tin, typename Tout>
__global__ __launch_bounds__(256) void dense_x_kernel(const Tin* __restrict__ in, Tout* __restrict__ out,
                                                      const R* __restrict__ W, int Lq, int L, int nlines,
                                                      int acc, const int* __restrict__ skip) {
  if (skip && *skip) return;
  using M = Mma<R>;
  __shared__ R As[kT][kPad];   // rows (line, part) of 32 lines, K chunk
  __shared__ R Ws[kT][kPad];   // rows m, K chunk
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.x * kT, line0 = blockIdx.y * (kT / 2);
  typename M::V acc4[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc4[t] = typename M::V{0, 0, 0, 0};
  // staging of one K chunk in registers: 32 lines x 16 q of the data
  // (contiguous along q) and 64 m x 16 q of W (padded: always in bounds);
  // the next chunk's loads are issued before the current chunk's MFMAs
  R xre[2], xim[2], wv4[4];
  auto load = [&](int q0) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int i = tid + 256 * j;
      const int ll = i / kKC, qq = i % kKC;
      const int line = line0 + ll, q = q0 + qq;
      xre[j] = 0;
      xim[j] = 0;
      if (line < nlines && q < L) {
        const Tin v = in[size_t(line) * L + q];
        xre[j] = R(v.x);
        xim[j] = R(v.y);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = tid + 256 * j;
      wv4[j] = W[size_t(m0 + i / kKC) * Lq + q0 + i % kKC];
    }
  };
  load(0);
  for (int q0 = 0; q0 < L; q0 += kKC) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int i = tid + 256 * j;
      const int ll = i / kKC, qq = i % kKC;
      const int wv = ll >> 3, li = ll & 7;
      As[16 * wv + M::xrow(li, 0)][qq] = xre[j];
      As[16 * wv + M::xrow(li, 1)][qq] = xim[j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = tid + 256 * j;
      Ws[i / kKC][i % kKC] = wv4[j];
    }
    __syncthreads();
    if (q0 + kKC < L) load(q0 + kKC);
#pragma unroll
    for (int kk = 0; kk < kKC / 4; ++kk) {
      const R a = As[16 * w + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc4[t] = M::mma(a, Ws[16 * t + (lane & 15)][4 * kk + (lane >> 4)], acc4[t]);
    }
    __syncthreads();
  }
  // lane holds lines (la, lb) of its wave's 8, both parts, for column m
  const int g = lane >> 4;
  const int la = sizeof(R) == 4 ? 2 * g : g, lb = sizeof(R) == 4 ? 2 * g + 1 : g + 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int m = m0 + 16 * t + (lane & 15);
    if (m >= L) continue;
    const typename M::V v = acc4[t];
    const R ra = v[0], ia = sizeof(R) == 4 ? v[1] : v[2];
    const R rb = sizeof(R) == 4 ? v[2] : v[1], ib = v[3];
    const int lines[2] = {line0 + 8 * w + la, line0 + 8 * w + lb};
    const R res[2][2] = {{ra, ia}, {rb, ib}};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (lines[h] >= nlines) continue;
      const size_t o = size_t(lines[h]) * L + m;
      Tout u;
      if (acc) {
        u = out[o];
        u.x += res[h][0];
        u.y += res[h][1];
      } else {
        u.x = res[h][0];
        u.y = res[h][1];
      }
      out[o] = u;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void dense_y_kernel(const R* __restrict__ in, R* __restrict__ out,
                                                      const R* __restrict__ W, int Lq, int L, int ncols,
                                                      const int* __restrict__ skip) {
  if (skip && *skip) return;
  using M = Mma<R>;
  __shared__ R Ws[kT][kPad];          // rows m, K chunk
  __shared__ R Xs[kKC][kT + 1];       // K chunk, columns
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c0 = blockIdx.x * kT, m0 = blockIdx.y * kT;
  const size_t plane = size_t(L) * ncols;
  const R* __restrict__ X = in + blockIdx.z * plane;
  typename M::V acc4[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc4[t] = typename M::V{0, 0, 0, 0};
  // one K chunk in registers (64 m x 16 q of W, 16 rows x 64 columns of the
  // plane, contiguous along columns); the next chunk is loaded during the MFMAs
  R wv4[4], xv4[4];
  auto load = [&](int q0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = tid + 256 * j;
      wv4[j] = W[size_t(m0 + i / kKC) * Lq + q0 + i % kKC];
      const int q = q0 + i / kT, c = c0 + i % kT;
      xv4[j] = (q < L && c < ncols) ? X[size_t(q) * ncols + c] : R(0);
    }
  };
  load(0);
  for (int q0 = 0; q0 < L; q0 += kKC) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = tid + 256 * j;
      Ws[i / kKC][i % kKC] = wv4[j];
      Xs[i / kT][i % kT] = xv4[j];
    }
    __syncthreads();
    if (q0 + kKC < L) load(q0 + kKC);
#pragma unroll
    for (int kk = 0; kk < kKC / 4; ++kk) {
      const R a = Ws[16 * w + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc4[t] = M::mma(a, Xs[4 * kk + (lane >> 4)][16 * t + (lane & 15)], acc4[t]);
    }
    __syncthreads();
  }
  R* __restrict__ Y = out + blockIdx.z * plane;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = c0 + 16 * t + (lane & 15);
    if (c >= ncols) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = m0 + 16 * w + M::row(lane, e);
      if (m < L) Y[size_t(m) * ncols + c] = acc4[t][e];
    }
  }
}

}  // namespace

template <typename R, typename Tin, typename Tout>
hipError_t launch_dense_x(const AxisXform& X, bool inverse, const Tin* in, Tout* out, int nlines, int acc,
                          hipStream_t s, const int* skip) {
  const R* W = static_cast<const R*>(X.wmat) + (inverse ? size_t(X.Lm) * X.Lq : 0);
  const dim3 grid((X.L + kT - 1) / kT, (nlines + kT / 2 - 1) / (kT / 2));
  hipLaunchKernelGGL((dense_x_kernel<R, Tin, Tout>), grid, dim3(256), 0, s, in, out, W, X.Lq, X.L, nlines, acc, skip);
  return hipGetLastError();
}

template <typename R, typename T2>
hipError_t launch_dense_y(const AxisXform& Y, bool inverse, const T2* in, T2* out, int nx, int nz,
                          hipStream_t s, const int* skip) {
  const R* W = static_cast<const R*>(Y.wmat) + (inverse ? size_t(Y.Lm) * Y.Lq : 0);
  const int ncols = 2 * nx;
  const dim3 grid((ncols + kT - 1) / kT, (Y.L + kT - 1) / kT, nz);
  hipLaunchKernelGGL((dense_y_kernel<R>), grid, dim3(256), 0, s, reinterpret_cast<const R*>(in),
                     reinterpret_cast<R*>(out), W, Y.Lq, Y.L, ncols, skip);
  return hipGetLastError();
}

template hipError_t launch_dense_x<double, double2, double2>(const AxisXform&, bool, const double2*, double2*,
                                                             int, int, hipStream_t, const int*);
template hipError_t launch_dense_x<float, double2, float2>(const AxisXform&, bool, const double2*, float2*,
                                                           int, int, hipStream_t, const int*);
template hipError_t launch_dense_x<float, float2, double2>(const AxisXform&, bool, const float2*, double2*,
                                                           int, int, hipStream_t, const int*);
template hipError_t launch_dense_x<float, float2, float2>(const AxisXform&, bool, const float2*, float2*,
                                                          int, int, hipStream_t, const int*);
template hipError_t launch_dense_y<double, double2>(const AxisXform&, bool, const double2*, double2*, int, int,
                                                    hipStream_t, const int*);
template hipError_t launch_dense_y<float, float2>(const AxisXform&, bool, const float2*, float2*, int, int,
                                                  hipStream_t, const int*);

}  // namespace h6
