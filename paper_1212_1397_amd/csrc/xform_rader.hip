// Fast sine / cosine transforms of Section 3.3 for a prime period parameter
// M with M - 1 = 256 (the 256^3 grids: n = 256, M = n + 1 = 257).
//
// Reduction to one complex DFT of length M per line.  For a line x of complex
// values, with s_q = x_q + x_{M-q}, d_q = x_q - x_{M-q}, q = 1..M-1:
//
//  sine sum    S_m = sum_{q=1}^{M-1} x_q sin(pi q m / M), m = 1..M-1:
//     y_q = s_q sin(pi q/M) + d_q,  Y = DFT_M(y),
//     S_{2j}   = (i/4)(Y_j - Y_{M-j}),
//     S_{2j+1} = Y_0/2 + sum_{i=1..j} (Y_i + Y_{M-i})/2;
//  cosine sum  C_m = sum_{q=0}^{M} x_q cos(pi q m / M), m = 0..M:
//     y_q = s_q + d_q sin(pi q/M),  Y = DFT_M(y),
//     C_{2j}   = x_0 + x_M + (Y_j + Y_{M-j})/4,
//     C_{2j+1} = x_0 - x_M + C'_1 - i sum_{i=1..j} (Y_i - Y_{M-i})/2,
//     C'_1     = (1/2) sum_q d_q cos(pi q/M).
// (Both follow from splitting y into its symmetric and antisymmetric parts,
// whose DFTs are the cosine and (-i times) the sine sums, and from the
// identities sin(a+b) - sin(a-b) = 2 cos a sin b, cos(a+b) - cos(a-b) =
// -2 sin a sin b for the odd outputs.)
//
// DFT_M for prime M by Rader's algorithm: with a primitive root g of M,
// Y_{g^b} = y_0 + sum_a y_{g^{-a}} w^{g^{b-a}} (w = e^{-2 pi i / M}), a cyclic
// convolution of length M - 1 = 256, done as FFT_256 -> pointwise product
// with the precomputed FFT of the kernel -> inverse FFT_256.  FFT_256 is the
// four-step 16 x 16 algorithm: 16 threads per line, each holding 16 values in
// registers; a radix-4 x 4 FFT16 per thread, twiddles, one LDS transpose.
// Forward output order is kept for the pointwise product and undone by the
// inverse, so the convolution costs two LDS transposes.
//
// Forward transforms apply W^{-1} ((2/M) sine sum, or (2/M) C W^T C for the
// cosine basis, C = diag(1/2, 1, .., 1, 1/2)); inverse transforms apply W
// (plain sums).  Lines are staged through LDS with coalesced loads/stores;
// along x a workgroup owns KL whole lines, along y a tile of KL consecutive x
// columns at one z (KL = 4, 8 or 16, chosen per axis: more columns make
// longer contiguous row segments along y, fewer lines more workgroups along x).
#include "fft16.h"
#include "h6_internal.h"
#include "xform_rader.h"

namespace h6 {
namespace {

using namespace fftdev;

#define T2 typename V2<R>::T

constexpr int kStride = 273;       // LDS row stride (complex) per line, >= 258 and >= 16*17
constexpr int kHalf = 128;         // (M - 1) / 2

// LDS use per line: the input is stored in Rader order (slot a holds node
// q = g^{-a}; slot a + 128 then holds node M - q because g^{128} = -1 mod M;
// the cosine basis keeps its end nodes q = 0, M in slots 256, 257), so the
// gather of (x_q, x_{M-q}) pairs reads consecutive slots; the 16 x 16
// transposes use a row stride of 17; Y is scattered to natural order and the
// outputs are written back in natural order for a coalesced store.
// table entries in the compute precision
template <typename R>
__device__ __forceinline__ typename V2<R>::T tab_tw(const RaderTables& tab, int i) {
  if constexpr (sizeof(R) == 4) return tab.tw_f[i];
  else return tab.tw256[i];
}
template <typename R>
__device__ __forceinline__ typename V2<R>::T tab_kf(const RaderTables& tab, int i) {
  if constexpr (sizeof(R) == 4) return tab.kf_f[i];
  else return tab.kf[i];
}
template <typename R>
__device__ __forceinline__ R tab_sin(const RaderTables& tab, int i) {
  if constexpr (sizeof(R) == 4) return tab.sin_f[i];
  else return tab.sin_a[i];
}
template <typename R>
__device__ __forceinline__ R tab_cos(const RaderTables& tab, int i) {
  if constexpr (sizeof(R) == 4) return tab.cos_f[i];
  else return tab.cos_a[i];
}

template <typename R, int AXIS, bool NEU, bool INV, int KL, typename Tin, typename Tout>
__global__ __launch_bounds__(KL * 16) void rader257_kernel(const Tin* __restrict__ in,
                                                               Tout* __restrict__ out, int nlines,
                                                               int nx, int L, RaderTables tab,
                                                               int acc, const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ T2 buf[KL][kStride];
  constexpr int kPx = (258 + KL * 16 - 1) / (KL * 16);   // loads per x line (L <= 258)
  constexpr int M = 257;
  const int tid = threadIdx.x;
  const int g = tid >> 4, t = tid & 15;
  const int* __restrict__ slot = NEU ? tab.slot_n : tab.slot_d;
  // ---- load KL lines into LDS in Rader order: all global reads of a
  // thread are issued before any LDS write (coalesced, many loads in flight) ----
  int nl;
  size_t gbase;
  // along y, a workgroup's columns share 128-byte lines with its neighbours':
  // neighbouring column groups are kept on one XCD
  int bx = blockIdx.x, by = blockIdx.y;
  if (AXIS == 1) {
    const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    bx = lid % gridDim.x;
    by = lid / gridDim.x;
  }
  const int line0 = bx * KL;
  if (AXIS == 0) {
    nl = min(KL, nlines - line0);
    gbase = size_t(line0) * L;
    // LDS slots first, unconditionally (clamped), so that no slot lookup is
    // waited on between the data loads and their LDS writes
    int sl[kPx];
#pragma unroll
    for (int k = 0; k < kPx; ++k) sl[k] = slot[min(tid + k * KL * 16, L - 1)];
    T2 r[KL][kPx];
#pragma unroll
    for (int b = 0; b < KL; ++b)
#pragma unroll
      for (int k = 0; k < kPx; ++k) {
        const int p = tid + k * KL * 16;
        if (b < nl && p < L) r[b][k] = cv<T2>(in[gbase + size_t(b) * L + p]);
      }
#pragma unroll
    for (int b = 0; b < KL; ++b)
#pragma unroll
      for (int k = 0; k < kPx; ++k) {
        const int p = tid + k * KL * 16;
        if (b < nl && p < L) buf[b][sl[k]] = r[b][k];
      }
  } else {
    nl = min(KL, nx - line0);                   // x columns i0 .. i0 + nl - 1
    gbase = size_t(by) * nx * L + line0;
    constexpr int kPer = (KL * 258 + KL * 16 - 1) / (KL * 16);
    int sl[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) sl[k] = slot[min((tid + k * KL * 16) / KL, L - 1)];
    T2 r[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * KL * 16;
      const int q = e / KL, b = e - q * KL;
      if (q < L && b < nl) r[k] = cv<T2>(in[gbase + size_t(q) * nx + b]);
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * KL * 16;
      const int q = e / KL, b = e - q * KL;
      if (q < L && b < nl) buf[b][sl[k]] = r[k];
    }
  }
  __syncthreads();

  // ---- gather y_{g^{-a}} (a = t + 16 n2) with the pre-processing ----
  T2 v[16];
  T2 y0sum = mk2<R>(0, 0), c1sum = mk2<R>(0, 0);
  T2 xa = mk2<R>(0, 0), xb = mk2<R>(0, 0);  // x_0 and x_M (cosine sums)
  if (NEU) {
    xa = buf[g][256];
    xb = buf[g][257];
    if (!INV) {
      xa = scl<R>(xa, R(0.5));
      xb = scl<R>(xb, R(0.5));
    }
  }
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) {
    const int a = t + 16 * n2;
    const T2 xq = buf[g][a], xr = buf[g][(a + 128) & 255];
    const T2 s = add<R>(xq, xr), d = sub<R>(xq, xr);
    const R sn = tab_sin<R>(tab, a);
    T2 y;
    if (NEU) {
      y = add<R>(s, scl<R>(d, sn));
      c1sum = add<R>(c1sum, scl<R>(d, R(0.5) * tab_cos<R>(tab, a)));
    } else {
      y = add<R>(scl<R>(s, sn), d);
    }
    y0sum = add<R>(y0sum, y);
    v[n2] = y;
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
    y0sum.x += __shfl_xor(y0sum.x, o, 16);
    y0sum.y += __shfl_xor(y0sum.y, o, 16);
    if (NEU) {
      c1sum.x += __shfl_xor(c1sum.x, o, 16);
      c1sum.y += __shfl_xor(c1sum.y, o, 16);
    }
  }
  __syncthreads();

  // ---- forward FFT_256: thread t = n1 holds element n1 + 16 n2 in v[n2] ----
  fft16<R, false>(v);                      // over n2 -> v[k2]
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) {
    const T2 w = tab_tw<R>(tab, (t * k2) & 255);
    buf[g][17 * t + k2] = mul<R>(v[k2], w);
  }
  __syncthreads();
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) v[n1] = buf[g][17 * n1 + t];   // thread t = k2
  fft16<R, false>(v);                      // over n1 -> X[16 k1 + k2] in v[k1]
  // pointwise product with the kernel spectrum (1/256 folded in), then
  // inverse FFT_256 back to the natural index
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) v[k1] = mul<R>(v[k1], tab_kf<R>(tab, 16 * k1 + t));
  fft16<R, true>(v);                       // over k1 -> Z[n1][k2] in v[n1]
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const T2 w = tab_tw<R>(tab, (n1 * t) & 255);
    buf[g][17 * n1 + t] = mul<R>(v[n1], mk2<R>(w.x, -w.y));
  }
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) v[k2] = buf[g][17 * t + k2];   // thread t = n1
  fft16<R, true>(v);                       // -> conv[n1 + 16 n2] in v[n2]
  __syncthreads();
  // Y_{g^b} = conv[b]; Y_0 = sum y
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) buf[g][tab.perm_out[t + 16 * n2]] = v[n2];
  if (t == 0) buf[g][0] = y0sum;
  __syncthreads();

  // ---- post-processing: thread t takes j = 9t .. 9t+8 (j <= 128).  The odd
  // outputs need running sums of the increments over j: a serial prefix over
  // the thread's own nine values plus one 16-lane scan of the thread totals ----
  T2 ev[9], od[9];
  T2 loc = mk2<R>(0, 0);
#pragma unroll
  for (int u = 0; u < 9; ++u) {
    const int j = 9 * t + u;
    const bool ok = j <= kHalf;
    const int jj = ok ? j : 0;
    const T2 Yj = buf[g][jj], Ym = buf[g][jj == 0 ? 0 : M - jj];
    T2 inc = mk2<R>(0, 0);
    if (ok && j >= 1) inc = NEU ? scl<R>(sub<R>(Yj, Ym), R(0.5)) : scl<R>(add<R>(Yj, Ym), R(0.5));
    loc = add<R>(loc, inc);
    od[u] = loc;                          // running sum within the thread (inclusive)
    if (NEU) {
      const T2 A = (j == 0) ? Yj : scl<R>(add<R>(Yj, Ym), R(0.5));
      ev[u] = add<R>(add<R>(xa, xb), scl<R>(A, R(0.5)));                      // C_{2j}
    } else {
      const T2 D = sub<R>(Yj, Ym);
      ev[u] = mk2<R>(-R(0.25) * D.y, R(0.25) * D.x);                          // S_{2j}
    }
  }
  T2 sc = loc;
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    const R px = __shfl_up(sc.x, o, 16), py = __shfl_up(sc.y, o, 16);
    if (t >= o) { sc.x += px; sc.y += py; }
  }
  const T2 off = sub<R>(sc, loc);        // sum over the lanes before t
#pragma unroll
  for (int u = 0; u < 9; ++u) {
    const T2 run = add<R>(off, od[u]);   // sum over 1 <= i <= j
    if (NEU)
      od[u] = add<R>(sub<R>(xa, xb), add<R>(c1sum, mk2<R>(run.y, -run.x)));  // C_{2j+1}
    else
      od[u] = add<R>(scl<R>(y0sum, R(0.5)), run);                             // S_{2j+1}
  }
  __syncthreads();
  // scaled outputs into LDS in natural order
  const R fs = INV ? R(1) : R(2) / R(M);
#pragma unroll
  for (int u = 0; u < 9; ++u) {
    const int j = 9 * t + u;
    if (j > kHalf) continue;
    if (NEU) {
      const int me = 2 * j, mo = 2 * j + 1;              // m = 0..M
      R se = fs, so = fs;
      if (!INV && me == 0) se *= R(0.5);
      if (!INV && mo == M) so *= R(0.5);
      buf[g][me] = scl<R>(ev[u], se);
      if (mo <= M) buf[g][mo] = scl<R>(od[u], so);
    } else {
      if (j >= 1) buf[g][2 * j - 1] = scl<R>(ev[u], fs);           // m = 2j -> index 2j - 1
      if (2 * j + 1 <= M - 2) buf[g][2 * j] = scl<R>(od[u], fs);   // m = 2j + 1
    }
  }
  __syncthreads();
  // ---- store (coalesced); with acc, out += result (all reads issued first) ----
  if (AXIS == 0) {
    if (acc) {
      Tout o[KL][kPx];
#pragma unroll
      for (int b = 0; b < KL; ++b)
#pragma unroll
        for (int k = 0; k < kPx; ++k) {
          const int p = tid + k * KL * 16;
          if (b < nl && p < L) o[b][k] = out[gbase + size_t(b) * L + p];
        }
#pragma unroll
      for (int b = 0; b < KL; ++b)
#pragma unroll
        for (int k = 0; k < kPx; ++k) {
          const int p = tid + k * KL * 16;
          if (b < nl && p < L) {
            const Tout v = cv<Tout>(buf[b][p]);
            Tout u;
            u.x = o[b][k].x + v.x;
            u.y = o[b][k].y + v.y;
            out[gbase + size_t(b) * L + p] = u;
          }
        }
    } else {
#pragma unroll
      for (int b = 0; b < KL; ++b)
#pragma unroll
        for (int k = 0; k < kPx; ++k) {
          const int p = tid + k * KL * 16;
          if (b < nl && p < L) out[gbase + size_t(b) * L + p] = cv<Tout>(buf[b][p]);
        }
    }
  } else {
    constexpr int kPer = (KL * 258 + KL * 16 - 1) / (KL * 16);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * KL * 16;
      const int q = e / KL, b = e - q * KL;
      if (q < L && b < nl) out[gbase + size_t(q) * nx + b] = cv<Tout>(buf[b][q]);
    }
  }
}

#undef T2

template <typename R, int AXIS, bool NEU, int KL, typename Tin, typename Tout>
void launch_one(bool inv, const Tin* in, Tout* out, int nlines, int nx, int L, int nz,
                const RaderTables& tab, hipStream_t s, int acc, const int* skip) {
  const dim3 grid = AXIS == 0 ? dim3((nlines + KL - 1) / KL) : dim3((nx + KL - 1) / KL, nz);
  if (inv)
    hipLaunchKernelGGL((rader257_kernel<R, AXIS, NEU, true, KL, Tin, Tout>), grid, dim3(KL * 16), 0,
                       s, in, out, nlines, nx, L, tab, acc, skip);
  else
    hipLaunchKernelGGL((rader257_kernel<R, AXIS, NEU, false, KL, Tin, Tout>), grid, dim3(KL * 16), 0,
                       s, in, out, nlines, nx, L, tab, 0, skip);
}

template <typename R, int AXIS, int KL, typename Tin, typename Tout>
void launch_bc(bool neumann, bool inv, const Tin* in, Tout* out, int nlines, int nx, int L, int nz,
               const RaderTables& tab, hipStream_t s, int acc, const int* skip) {
  if (neumann)
    launch_one<R, AXIS, true, KL>(inv, in, out, nlines, nx, L, nz, tab, s, acc, skip);
  else
    launch_one<R, AXIS, false, KL>(inv, in, out, nlines, nx, L, nz, tab, s, acc, skip);
}

}  // namespace

bool rader_lines_ok(int axis, int lines) {
  return axis == 0 ? (lines == 4 || lines == 8) : (lines == 8 || lines == 16);
}

template <typename R, typename Tin, typename Tout>
hipError_t launch_rader_x(bool neumann, bool inverse, const Tin* in, Tout* out, int nlines, int L,
                          const RaderTables& tab, hipStream_t s, int accumulate, int lines, const int* skip) {
  if (lines == 4)
    launch_bc<R, 0, 4>(neumann, inverse, in, out, nlines, 0, L, 0, tab, s, accumulate, skip);
  else if (lines == 8)
    launch_bc<R, 0, 8>(neumann, inverse, in, out, nlines, 0, L, 0, tab, s, accumulate, skip);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename R, typename T>
hipError_t launch_rader_y(bool neumann, bool inverse, const T* in, T* out, int nx, int L, int nz,
                          const RaderTables& tab, hipStream_t s, int lines, const int* skip) {
  if (lines == 8)
    launch_bc<R, 1, 8>(neumann, inverse, in, out, 0, nx, L, nz, tab, s, 0, skip);
  else if (lines == 16)
    launch_bc<R, 1, 16>(neumann, inverse, in, out, 0, nx, L, nz, tab, s, 0, skip);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template hipError_t launch_rader_x<double, double2, double2>(bool, bool, const double2*, double2*,
                                                             int, int, const RaderTables&, hipStream_t, int, int, const int*);
template hipError_t launch_rader_x<float, double2, float2>(bool, bool, const double2*, float2*, int,
                                                           int, const RaderTables&, hipStream_t, int, int, const int*);
template hipError_t launch_rader_x<float, float2, double2>(bool, bool, const float2*, double2*, int,
                                                           int, const RaderTables&, hipStream_t, int, int, const int*);
template hipError_t launch_rader_x<float, float2, float2>(bool, bool, const float2*, float2*, int,
                                                          int, const RaderTables&, hipStream_t, int, int, const int*);
template hipError_t launch_rader_y<double, double2>(bool, bool, const double2*, double2*, int, int,
                                                    int, const RaderTables&, hipStream_t, int, const int*);
template hipError_t launch_rader_y<float, float2>(bool, bool, const float2*, float2*, int, int, int,
                                                  const RaderTables&, hipStream_t, int, const int*);

}  // namespace h6
