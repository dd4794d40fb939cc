// Fast sine / cosine transforms of Section 3.3 for odd period parameters
// M = n + 1 <= 255 (the grids other than 256^3: 32^3, 48^3, 64^3, 96^3,
// 128^3, 160^3, ...).
//
// The reduction to one complex DFT of length M per line is the one of
// xform_rader.hip: from the line x, with s_q = x_q + x_{M-q} and
// d_q = x_q - x_{M-q}, y_q = s_q sin(pi q / M) + d_q (sine basis) or
// y_q = s_q + d_q sin(pi q / M) (cosine basis) for q = 1..M-1, y_0 = 0,
// Y = DFT_M(y), and the even / odd outputs from Y_j +- Y_{M-j} with a prefix
// sum for the odd ones.
//
// DFT_M by Bluestein's algorithm: with c_j = exp(-i pi j^2 / M) and
// qk = (q^2 + k^2 - (k - q)^2) / 2,
//   Y_k = sum_q y_q exp(-2 pi i q k / M) = c_k sum_q (y_q c_q) conj(c_{k - q}),
// a convolution of a_q = y_q c_q with b_j = conj(c_j).  As y_0 = 0 the lags
// j = k - q run over 1 - M .. M - 2, 2M - 2 values, so a cyclic convolution of
// length P >= 2M - 2 is exact (P = 256 for M <= 129, else 512): FFT_P, product
// with FFT_P(b) / P (a table), inverse FFT_P.
//
// FFT_P is four-step with P = 16 Q: 16 threads per line, thread n1 holding
// elements n1 + 16 n2 (n2 < Q) in registers.  Forward: FFT_Q over n2 in
// registers (Q = 32: two FFT_16 and a radix-2 step), twiddles
// exp(-2 pi i n1 k2 / P), one LDS transpose (rows of Q + 1), then FFT_16 over
// n1 for each of the thread's Q / 16 columns k2: X[k2 + Q k1].  The inverse
// runs the same steps backwards, ending with conv[n1 + 16 n2] in the same
// registers the forward FFT started from.
#include "fft16.h"
#include "h6_internal.h"
#include "xform_bluestein.h"

namespace h6 {
namespace {

using namespace fftdev;

#define T2 typename V2<R>::T

template <typename R> __device__ __forceinline__ T2 tb_chirp(const BluesteinTables& t, int i) {
  if constexpr (sizeof(R) == 4) return t.chirp_f[i]; else return t.chirp[i];
}
template <typename R> __device__ __forceinline__ T2 tb_bhat(const BluesteinTables& t, int i) {
  if constexpr (sizeof(R) == 4) return t.bhat_f[i]; else return t.bhat[i];
}
template <typename R> __device__ __forceinline__ T2 tb_tw(const BluesteinTables& t, int i) {
  if constexpr (sizeof(R) == 4) return t.tw_f[i]; else return t.tw[i];
}
template <typename R> __device__ __forceinline__ R tb_sin(const BluesteinTables& t, int i) {
  if constexpr (sizeof(R) == 4) return t.sin_f[i]; else return t.sin_q[i];
}
template <typename R> __device__ __forceinline__ R tb_cos(const BluesteinTables& t, int i) {
  if constexpr (sizeof(R) == 4) return t.cos_f[i]; else return t.cos_q[i];
}

// FFT of length Q = 16 or 32 in registers (natural order in and out)
template <typename R, int Q, bool INV>
__device__ __forceinline__ void fftq(T2 (&v)[Q]) {
  if constexpr (Q == 16) {
    fft16<R, INV>(v);
  } else {
    static_assert(Q == 32, "FFT length");
    T2 a[16], b[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      a[i] = v[2 * i];
      b[i] = v[2 * i + 1];
    }
    fft16<R, INV>(a);
    fft16<R, INV>(b);
    // X[k] = A[k] + w^k B[k], X[k + 16] = A[k] - w^k B[k], w^k = cos(2 pi k / 32) -+ i sin(2 pi k / 32)
    constexpr double c32[16] = {1.0, 0.98078528040323044913, 0.92387953251128675613, 0.83146961230254523708,
                                0.70710678118654752440, 0.55557023301960222474, 0.38268343236508977173,
                                0.19509032201612826785, 0.0, -0.19509032201612826785, -0.38268343236508977173,
                                -0.55557023301960222474, -0.70710678118654752440, -0.83146961230254523708,
                                -0.92387953251128675613, -0.98078528040323044913};
    constexpr double s32[16] = {0.0, 0.19509032201612826785, 0.38268343236508977173, 0.55557023301960222474,
                                0.70710678118654752440, 0.83146961230254523708, 0.92387953251128675613,
                                0.98078528040323044913, 1.0, 0.98078528040323044913, 0.92387953251128675613,
                                0.83146961230254523708, 0.70710678118654752440, 0.55557023301960222474,
                                0.38268343236508977173, 0.19509032201612826785};
    const R sg = INV ? R(1) : R(-1);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const T2 w = mk2<R>(R(c32[k]), sg * R(s32[k]));
      const T2 t = mul<R>(b[k], w);
      v[k] = add<R>(a[k], t);
      v[k + 16] = sub<R>(a[k], t);
    }
  }
}

template <int P> struct BShape {
  static constexpr int Q = P / 16;                          // registers per thread
  static constexpr int kRow = Q + 1;                        // LDS row of the transpose
  static constexpr int kStride = 16 * kRow + 1;             // LDS per line (>= 256 line values)
  static constexpr int kOut = (P == 256 ? 5 : 8);           // post-processed outputs per thread, 16 kOut > (M-1)/2
};

template <typename R, int AXIS, bool NEU, bool INV, int P, int KL, typename Tin, typename Tout>
__global__ __launch_bounds__(KL * 16) void bluestein_kernel(const Tin* __restrict__ in, Tout* __restrict__ out,
                                                            int nlines, int nx, int L, BluesteinTables tab, int acc,
                                                            const int* __restrict__ skip) {
  if (skip && *skip) return;
  using S = BShape<P>;
  constexpr int Q = S::Q, kRow = S::kRow;
  __shared__ T2 buf[KL][S::kStride];
  const int M = tab.M;
  const int tid = threadIdx.x;
  const int g = tid >> 4, t = tid & 15;
  constexpr int kPx = (256 + KL * 16 - 1) / (KL * 16);      // loads per x line (L <= 256)
  int nl;
  size_t gbase;
  const int line0 = blockIdx.x * KL;
  // ---- load KL lines into LDS in natural order (all reads issued first) ----
  if (AXIS == 0) {
    nl = min(KL, nlines - line0);
    gbase = size_t(line0) * L;
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
        if (b < nl && p < L) buf[b][p] = r[b][k];
      }
  } else {
    nl = min(KL, nx - line0);
    gbase = size_t(blockIdx.y) * nx * L + line0;
    constexpr int kPer = (KL * 256 + KL * 16 - 1) / (KL * 16);
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
      if (q < L && b < nl) buf[b][q] = r[k];
    }
  }
  __syncthreads();

  // ---- a_q = y_q c_q for q = t + 16 n2 (zero for q = 0 and q >= M) ----
  const int off = NEU ? 0 : -1;                             // array index of node q: q (cosine), q - 1 (sine)
  T2 v[Q];
  T2 c1sum = mk2<R>(0, 0), xa = mk2<R>(0, 0), xb = mk2<R>(0, 0);
  if (NEU) {
    xa = buf[g][0];
    xb = buf[g][M];
    if (!INV) {
      xa = scl<R>(xa, R(0.5));
      xb = scl<R>(xb, R(0.5));
    }
  }
#pragma unroll
  for (int n2 = 0; n2 < Q; ++n2) {
    const int q = t + 16 * n2;
    T2 a = mk2<R>(0, 0);
    if (q >= 1 && q < M) {
      const T2 xq = buf[g][q + off], xr = buf[g][M - q + off];
      const T2 s = add<R>(xq, xr), d = sub<R>(xq, xr);
      const R sn = tb_sin<R>(tab, q);
      T2 y;
      if (NEU) {
        y = add<R>(s, scl<R>(d, sn));
        c1sum = add<R>(c1sum, scl<R>(d, R(0.5) * tb_cos<R>(tab, q)));
      } else {
        y = add<R>(scl<R>(s, sn), d);
      }
      a = mul<R>(y, tb_chirp<R>(tab, q));
    }
    v[n2] = a;
  }
  if (NEU) {
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      c1sum.x += __shfl_xor(c1sum.x, o, 16);
      c1sum.y += __shfl_xor(c1sum.y, o, 16);
    }
  }
  __syncthreads();

  // ---- forward FFT_P ----
  fftq<R, Q, false>(v);                                     // over n2 -> k2
#pragma unroll
  for (int k2 = 0; k2 < Q; ++k2) buf[g][kRow * t + k2] = mul<R>(v[k2], tb_tw<R>(tab, t * k2));
  __syncthreads();
  constexpr int C = Q / 16;                                 // columns k2 = t + 16 c of this thread
  T2 u[C][16];
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) u[c][n1] = buf[g][kRow * n1 + t + 16 * c];
    fft16<R, false>(u[c]);                                  // X[k2 + Q k1] in u[c][k1]
    // product with the kernel spectrum (1/P folded in), inverse FFT_16 over k1
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) u[c][k1] = mul<R>(u[c][k1], tb_bhat<R>(tab, t + 16 * c + Q * k1));
    fft16<R, true>(u[c]);                                   // Z[n1] for column k2
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) {
      const T2 w = tb_tw<R>(tab, n1 * (t + 16 * c));
      buf[g][kRow * n1 + t + 16 * c] = mul<R>(u[c][n1], mk2<R>(w.x, -w.y));
    }
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < Q; ++k2) v[k2] = buf[g][kRow * t + k2];
  fftq<R, Q, true>(v);                                      // conv[t + 16 n2] in v[n2]
  __syncthreads();
  // Y_k = c_k conv_k, natural order
#pragma unroll
  for (int n2 = 0; n2 < Q; ++n2) {
    const int k = t + 16 * n2;
    if (k < M) buf[g][k] = mul<R>(v[n2], tb_chirp<R>(tab, k));
  }
  __syncthreads();

  // ---- post-processing: thread t takes j = J t .. J t + J - 1 (j <= (M - 1) / 2 <= 16 J - 1) ----
  constexpr int J = S::kOut;
  const int kHalfM = (M - 1) / 2;
  const T2 Y0 = buf[g][0];
  T2 ev[J], od[J];
  T2 loc = mk2<R>(0, 0);
#pragma unroll
  for (int uu = 0; uu < J; ++uu) {
    const int j = J * t + uu;
    const bool ok = j <= kHalfM;
    const int jj = ok ? j : 0;
    const T2 Yj = buf[g][jj], Ym = buf[g][jj == 0 ? 0 : M - jj];
    T2 inc = mk2<R>(0, 0);
    if (ok && j >= 1) inc = NEU ? scl<R>(sub<R>(Yj, Ym), R(0.5)) : scl<R>(add<R>(Yj, Ym), R(0.5));
    loc = add<R>(loc, inc);
    od[uu] = loc;
    if (NEU) {
      const T2 A = (j == 0) ? Yj : scl<R>(add<R>(Yj, Ym), R(0.5));
      ev[uu] = add<R>(add<R>(xa, xb), scl<R>(A, R(0.5)));   // C_{2j}
    } else {
      const T2 D = sub<R>(Yj, Ym);
      ev[uu] = mk2<R>(-R(0.25) * D.y, R(0.25) * D.x);       // S_{2j}
    }
  }
  T2 sc = loc;
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    const R px = __shfl_up(sc.x, o, 16), py = __shfl_up(sc.y, o, 16);
    if (t >= o) {
      sc.x += px;
      sc.y += py;
    }
  }
  const T2 before = sub<R>(sc, loc);                        // sum over the lanes before t
#pragma unroll
  for (int uu = 0; uu < J; ++uu) {
    const T2 run = add<R>(before, od[uu]);                  // sum over 1 <= i <= j
    if (NEU)
      od[uu] = add<R>(sub<R>(xa, xb), add<R>(c1sum, mk2<R>(run.y, -run.x)));   // C_{2j+1}
    else
      od[uu] = add<R>(scl<R>(Y0, R(0.5)), run);                                // S_{2j+1}
  }
  __syncthreads();
  const R fs = INV ? R(1) : R(2) / R(M);
#pragma unroll
  for (int uu = 0; uu < J; ++uu) {
    const int j = J * t + uu;
    if (j > kHalfM) continue;
    if (NEU) {
      const int me = 2 * j, mo = 2 * j + 1;                 // m = 0..M
      R se = fs, so = fs;
      if (!INV && me == 0) se *= R(0.5);
      if (!INV && mo == M) so *= R(0.5);
      buf[g][me] = scl<R>(ev[uu], se);
      if (mo <= M) buf[g][mo] = scl<R>(od[uu], so);
    } else {
      if (j >= 1) buf[g][2 * j - 1] = scl<R>(ev[uu], fs);   // m = 2j -> index 2j - 1
      if (2 * j + 1 <= M - 2) buf[g][2 * j] = scl<R>(od[uu], fs);   // m = 2j + 1
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
            const Tout w = cv<Tout>(buf[b][p]);
            Tout r2;
            r2.x = o[b][k].x + w.x;
            r2.y = o[b][k].y + w.y;
            out[gbase + size_t(b) * L + p] = r2;
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
    constexpr int kPer = (KL * 256 + KL * 16 - 1) / (KL * 16);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * KL * 16;
      const int q = e / KL, b = e - q * KL;
      if (q < L && b < nl) out[gbase + size_t(q) * nx + b] = cv<Tout>(buf[b][q]);
    }
  }
}

#undef T2

template <typename R, int AXIS, int P, int KL, typename Tin, typename Tout>
void launch_b(bool neumann, bool inv, const Tin* in, Tout* out, int nlines, int nx, int L, int nz,
              const BluesteinTables& tab, hipStream_t s, int acc, const int* skip) {
  const dim3 grid = AXIS == 0 ? dim3((nlines + KL - 1) / KL) : dim3((nx + KL - 1) / KL, nz);
#define H6_BL(N, I)                                                                                       \
  if (neumann == N && inv == I) {                                                                        \
    hipLaunchKernelGGL((bluestein_kernel<R, AXIS, N, I, P, KL, Tin, Tout>), grid, dim3(KL * 16), 0, s, in, \
                       out, nlines, nx, L, tab, acc, skip);                                              \
    return;                                                                                              \
  }
  H6_BL(true, true) H6_BL(true, false) H6_BL(false, true) H6_BL(false, false)
#undef H6_BL
}

}  // namespace

// lines per workgroup: 4 along x; along y 16 (complex64, P = 256), 8 (complex64 with P = 512 or
// complex128 with P = 256), 4 (complex128, P = 512): LDS per workgroup 17-35 KB
template <typename R, typename Tin, typename Tout>
hipError_t launch_bluestein_x(bool neumann, bool inverse, const Tin* in, Tout* out, int nlines, int L,
                              const BluesteinTables& tab, hipStream_t s, int accumulate, const int* skip) {
  if (!bluestein_ok(tab.M) || L > 256 || tab.P != bluestein_length(tab.M)) return hipErrorInvalidValue;
  if (tab.P == 256)
    launch_b<R, 0, 256, 4>(neumann, inverse, in, out, nlines, 0, L, 0, tab, s, accumulate, skip);
  else
    launch_b<R, 0, 512, 4>(neumann, inverse, in, out, nlines, 0, L, 0, tab, s, accumulate, skip);
  return hipGetLastError();
}

template <typename R, typename T>
hipError_t launch_bluestein_y(bool neumann, bool inverse, const T* in, T* out, int nx, int L, int nz,
                              const BluesteinTables& tab, hipStream_t s, const int* skip) {
  if (!bluestein_ok(tab.M) || L > 256 || tab.P != bluestein_length(tab.M)) return hipErrorInvalidValue;
  constexpr bool f32 = sizeof(R) == 4;
  if (tab.P == 256)
    launch_b<R, 1, 256, f32 ? 16 : 8>(neumann, inverse, in, out, 0, nx, L, nz, tab, s, 0, skip);
  else
    launch_b<R, 1, 512, f32 ? 8 : 4>(neumann, inverse, in, out, 0, nx, L, nz, tab, s, 0, skip);
  return hipGetLastError();
}

template hipError_t launch_bluestein_x<double, double2, double2>(bool, bool, const double2*, double2*, int, int,
                                                                 const BluesteinTables&, hipStream_t, int,
                                                                 const int*);
template hipError_t launch_bluestein_x<float, double2, float2>(bool, bool, const double2*, float2*, int, int,
                                                               const BluesteinTables&, hipStream_t, int,
                                                               const int*);
template hipError_t launch_bluestein_x<float, float2, double2>(bool, bool, const float2*, double2*, int, int,
                                                               const BluesteinTables&, hipStream_t, int,
                                                               const int*);
template hipError_t launch_bluestein_x<float, float2, float2>(bool, bool, const float2*, float2*, int, int,
                                                              const BluesteinTables&, hipStream_t, int,
                                                              const int*);
template hipError_t launch_bluestein_y<double, double2>(bool, bool, const double2*, double2*, int, int, int,
                                                        const BluesteinTables&, hipStream_t, const int*);
template hipError_t launch_bluestein_y<float, float2>(bool, bool, const float2*, float2*, int, int, int,
                                                      const BluesteinTables&, hipStream_t, const int*);

}  // namespace h6
