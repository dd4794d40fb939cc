// Sine / cosine transforms of Section 3.3 as dense products on the matrix
// cores, for the axes the FFT paths do not take.  Along an axis with L
// unknowns the transform of each line is out_m = sum_q W[m][q] in_q with the
// L x L basis matrix W of the plan (scale factors folded in).
//
// Every such W (inverse and forward, sine and cosine basis) is even or odd
// under the reflection of the nodes q -> M - q, i.e. of the array index
// q -> L - 1 - q: W[m][L-1-q] = (-1)^m W[m][q].  So with H = ceil(L / 2),
// h = floor(L / 2), u_p = x_p + x_{L-1-p}, v_p = x_p - x_{L-1-p} (p < h) and
// u_h = x_h for odd L (the middle node),
//   out_{2j}   = sum_{p < H} We[j][p] u_p,   We[j][p] = W[2j][p],
//   out_{2j+1} = sum_{p < h} Wo[j][p] v_p,   Wo[j][p] = W[2j+1][p]:
// two half-size products, half the matrix-core work of the L x L one.  A pass
// is one GEMM pair per z-plane (y) or per block of lines (x):
//   y: C[m][c] = sum_q W[m][q] X[q][c],   X = the plane as L x 2n'x reals
//      (row q = y index; real and imaginary parts of each x are columns);
//   x: C[r][m] = sum_q X[r][q] W[m][q],   rows r = (line, real or imaginary part).
// Complex data times a real matrix needs no extra flops.  One MFMA tile is
// 16 x 16 with K = 4 (v_mfma_f32_16x16x4f32 in complex64 plans,
// v_mfma_f64_16x16x4f64 in complex128 ones).  A workgroup of 4 waves owns the
// 64 consecutive outputs m = 64 b .. 64 b + 63 (32 even and 32 odd ones, j =
// 32 b .. 32 b + 31) of 32 lines (x) or 64 columns (y), folding the line
// halves into u and v as it stages K chunks in LDS.  We and Wo are stored
// zero-padded to [Hm][Hk] (Hm a multiple of 32, Hk of the K chunk), so
// operand reads of them need no bounds checks.
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
constexpr int kKC = kDenseKChunk;                  // K chunk staged per step
constexpr int kXL = (kT / 2) * kKC / 256;          // (line, p) values of a chunk per thread (x)
constexpr int kWL = kT * kKC / 256;                // W values of a chunk per thread
constexpr int kYL = kKC * kT / 256;                // (p, column) values of a chunk per thread (y)
static_assert(kWL == kYL, "the y kernel stages W and data in one loop");
constexpr int kPad = kKC + 1;

template <typename R, typename Tin, typename Tout>
__global__ __launch_bounds__(256) void dense_x_kernel(const Tin* __restrict__ in, Tout* __restrict__ out,
                                                      const R* __restrict__ W, int Hm, int Hk, int L, int nlines,
                                                      int acc, const int* __restrict__ skip) {
  if (skip && *skip) return;
  using M = Mma<R>;
  __shared__ R Au[kT][kPad];   // rows (line, part) of 32 lines, K chunk of u
  __shared__ R Av[kT][kPad];   // the same rows, K chunk of v
  __shared__ R Ws[kT][kPad];   // rows j of We (0..31), then of Wo (32..63), K chunk
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int j0 = blockIdx.x * (kT / 2), line0 = blockIdx.y * (kT / 2);
  const int h = L >> 1, H = L - h;
  typename M::V acc4[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc4[t] = typename M::V{0, 0, 0, 0};
  // accumulator tile t: even outputs (t < 2) or odd ones, j = j0 + 16 (t & 1) ..;
  // tiles 1 and 3 idle when j0 + 16 is past the last j
  const bool upper = j0 + 16 < H;
  // staging of one K chunk in registers: 32 lines x 16 p of u and v (two
  // coalesced reads per value, one ascending and one descending along the
  // line) and 64 rows x 16 p of We / Wo (padded: always in bounds); the next
  // chunk's loads are issued before the current chunk's MFMAs
  R ure[kXL], uim[kXL], vre[kXL], vim[kXL], wv4[kWL];
  auto load = [&](int p0) {
#pragma unroll
    for (int j = 0; j < kXL; ++j) {
      const int i = tid + 256 * j;
      const int ll = i / kKC, pp = i % kKC;
      const int line = line0 + ll, p = p0 + pp;
      ure[j] = 0;
      uim[j] = 0;
      vre[j] = 0;
      vim[j] = 0;
      if (line < nlines && p < H) {
        const Tin a = in[size_t(line) * L + p];
        if (p < h) {
          const Tin b = in[size_t(line) * L + (L - 1 - p)];
          ure[j] = R(a.x) + R(b.x);
          uim[j] = R(a.y) + R(b.y);
          vre[j] = R(a.x) - R(b.x);
          vim[j] = R(a.y) - R(b.y);
        } else {
          ure[j] = R(a.x);
          uim[j] = R(a.y);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kWL; ++j) {
      const int i = tid + 256 * j;
      const int r = i / kKC;
      wv4[j] = W[(size_t(r >> 5) * Hm + j0 + (r & 31)) * Hk + p0 + i % kKC];
    }
  };
  load(0);
  for (int p0 = 0; p0 < H; p0 += kKC) {
#pragma unroll
    for (int j = 0; j < kXL; ++j) {
      const int i = tid + 256 * j;
      const int ll = i / kKC, pp = i % kKC;
      const int wv = ll >> 3, li = ll & 7;
      Au[16 * wv + M::xrow(li, 0)][pp] = ure[j];
      Au[16 * wv + M::xrow(li, 1)][pp] = uim[j];
      Av[16 * wv + M::xrow(li, 0)][pp] = vre[j];
      Av[16 * wv + M::xrow(li, 1)][pp] = vim[j];
    }
#pragma unroll
    for (int j = 0; j < kWL; ++j) {
      const int i = tid + 256 * j;
      Ws[i / kKC][i % kKC] = wv4[j];
    }
    __syncthreads();
    if (p0 + kKC < H) load(p0 + kKC);
    if (upper) {
#pragma unroll
      for (int kk = 0; kk < kKC / 4; ++kk) {
        const R au = Au[16 * w + (lane & 15)][4 * kk + (lane >> 4)];
        const R av = Av[16 * w + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc4[t] = M::mma(t < 2 ? au : av, Ws[16 * t + (lane & 15)][4 * kk + (lane >> 4)], acc4[t]);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < kKC / 4; ++kk) {
        const R au = Au[16 * w + (lane & 15)][4 * kk + (lane >> 4)];
        const R av = Av[16 * w + (lane & 15)][4 * kk + (lane >> 4)];
        acc4[0] = M::mma(au, Ws[(lane & 15)][4 * kk + (lane >> 4)], acc4[0]);
        acc4[2] = M::mma(av, Ws[32 + (lane & 15)][4 * kk + (lane >> 4)], acc4[2]);
      }
    }
    __syncthreads();
  }
  // lane holds lines (la, lb) of its wave's 8, both parts, for output m
  const int g = lane >> 4;
  const int la = sizeof(R) == 4 ? 2 * g : g, lb = sizeof(R) == 4 ? 2 * g + 1 : g + 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int m = 2 * (j0 + 16 * (t & 1) + (lane & 15)) + (t >> 1);
    if (m >= L) continue;
    const typename M::V v = acc4[t];
    const R ra = v[0], ia = sizeof(R) == 4 ? v[1] : v[2];
    const R rb = sizeof(R) == 4 ? v[2] : v[1], ib = v[3];
    const int lines[2] = {line0 + 8 * w + la, line0 + 8 * w + lb};
    const R res[2][2] = {{ra, ia}, {rb, ib}};
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      if (lines[hh] >= nlines) continue;
      const size_t o = size_t(lines[hh]) * L + m;
      Tout u;
      if (acc) {
        u = out[o];
        u.x += res[hh][0];
        u.y += res[hh][1];
      } else {
        u.x = res[hh][0];
        u.y = res[hh][1];
      }
      out[o] = u;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void dense_y_kernel(const R* __restrict__ in, R* __restrict__ out,
                                                      const R* __restrict__ W, int Hm, int Hk, int L, int ncols,
                                                      const int* __restrict__ skip) {
  if (skip && *skip) return;
  using M = Mma<R>;
  __shared__ R Ws[kT][kPad];          // rows j of We (0..31), then of Wo (32..63), K chunk
  __shared__ R Us[kKC][kT + 1];       // K chunk of u, columns
  __shared__ R Vs[kKC][kT + 1];       // K chunk of v, columns
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c0 = blockIdx.x * kT, j0 = blockIdx.y * (kT / 2);
  const int h = L >> 1, H = L - h;
  const size_t plane = size_t(L) * ncols;
  const R* __restrict__ X = in + blockIdx.z * plane;
  typename M::V acc4[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc4[t] = typename M::V{0, 0, 0, 0};
  // waves 0, 1: even outputs j0 + 16 w ..; waves 2, 3: odd outputs j0 + 16 (w - 2) ..
  const bool odd = w >= 2;
  const bool busy = j0 + 16 * (w & 1) < (odd ? h : H);
  // one K chunk in registers (64 rows x 16 p of We / Wo, 16 rows x 64 columns
  // of u and v from two coalesced plane rows each); the next chunk is loaded
  // during the MFMAs
  R wv4[kWL], uv4[kYL], vv4[kYL];
  auto load = [&](int p0) {
#pragma unroll
    for (int j = 0; j < kWL; ++j) {
      const int i = tid + 256 * j;
      const int r = i / kKC;
      wv4[j] = W[(size_t(r >> 5) * Hm + j0 + (r & 31)) * Hk + p0 + i % kKC];
      const int p = p0 + i / kT, c = c0 + i % kT;
      uv4[j] = 0;
      vv4[j] = 0;
      if (p < H && c < ncols) {
        const R a = X[size_t(p) * ncols + c];
        if (p < h) {
          const R b = X[size_t(L - 1 - p) * ncols + c];
          uv4[j] = a + b;
          vv4[j] = a - b;
        } else {
          uv4[j] = a;
        }
      }
    }
  };
  load(0);
  for (int p0 = 0; p0 < H; p0 += kKC) {
#pragma unroll
    for (int j = 0; j < kWL; ++j) {
      const int i = tid + 256 * j;
      Ws[i / kKC][i % kKC] = wv4[j];
      Us[i / kT][i % kT] = uv4[j];
      Vs[i / kT][i % kT] = vv4[j];
    }
    __syncthreads();
    if (p0 + kKC < H) load(p0 + kKC);
    if (busy) {
      const R(*B)[kT + 1] = odd ? Vs : Us;
#pragma unroll
      for (int kk = 0; kk < kKC / 4; ++kk) {
        const R a = Ws[16 * w + (lane & 15)][4 * kk + (lane >> 4)];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc4[t] = M::mma(a, B[4 * kk + (lane >> 4)][16 * t + (lane & 15)], acc4[t]);
      }
    }
    __syncthreads();
  }
  if (!busy) return;
  R* __restrict__ Y = out + blockIdx.z * plane;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = c0 + 16 * t + (lane & 15);
    if (c >= ncols) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = 2 * (j0 + 16 * (w & 1) + M::row(lane, e)) + (odd ? 1 : 0);
      if (m < L) Y[size_t(m) * ncols + c] = acc4[t][e];
    }
  }
}

}  // namespace

// Matrices of one direction: We then Wo, [Hm][Hk] each; the inverse follows the forward.
template <typename R, typename Tin, typename Tout>
hipError_t launch_dense_x(const AxisXform& X, bool inverse, const Tin* in, Tout* out, int nlines, int acc,
                          hipStream_t s, const int* skip) {
  const R* W = static_cast<const R*>(X.wmat) + (inverse ? 2 * size_t(X.Hm) * X.Hk : 0);
  const int H = X.L - X.L / 2;
  const dim3 grid((H + kT / 2 - 1) / (kT / 2), (nlines + kT / 2 - 1) / (kT / 2));
  hipLaunchKernelGGL((dense_x_kernel<R, Tin, Tout>), grid, dim3(256), 0, s, in, out, W, X.Hm, X.Hk, X.L, nlines,
                     acc, skip);
  return hipGetLastError();
}

template <typename R, typename T2>
hipError_t launch_dense_y(const AxisXform& Y, bool inverse, const T2* in, T2* out, int nx, int nz,
                          hipStream_t s, const int* skip) {
  const R* W = static_cast<const R*>(Y.wmat) + (inverse ? 2 * size_t(Y.Hm) * Y.Hk : 0);
  const int ncols = 2 * nx, H = Y.L - Y.L / 2;
  const dim3 grid((ncols + kT - 1) / kT, (H + kT / 2 - 1) / (kT / 2), nz);
  hipLaunchKernelGGL((dense_y_kernel<R>), grid, dim3(256), 0, s, reinterpret_cast<const R*>(in),
                     reinterpret_cast<R*>(out), W, Y.Hm, Y.Hk, Y.L, ncols, skip);
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
