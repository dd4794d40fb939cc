// z = A_p^{-1} r for the 7-point preconditioner of eq. (3DAP) (Section 3.3):
//   1. forward transform along x (sine basis for a Dirichlet pair, cosine basis
//      for a Neumann pair),
//   2. forward transform along y,
//   3. per transverse mode (m_x, m_y), one tridiagonal solve along z with
//      T_z + (kappa + lambda_x(m_x) + lambda_y(m_y)) I,
//   4. inverse transform along y, 5. inverse transform along x.
// With M = n + 1 the bases are W_qm = sin(pi q m / M) (q, m = 1..n) and
// W_qm = cos(pi q m / M) (q, m = 0..M); W^{-1} = (2/M) W^T and
// (2/M) C W^T C (C = diag(1/2, 1, .., 1, 1/2)) respectively.
//
// Compute type R is double (FP64 plans) or float (mixed plans, complex64
// intermediates); the input r and output z are complex128 in both.
#include <type_traits>

#include "h6_internal.h"

namespace h6 {
namespace {

template <typename R> struct C2;
template <> struct C2<double> { using T = double2; };
template <> struct C2<float> { using T = float2; };

template <typename R>
__device__ __forceinline__ typename C2<R>::T mk(R a, R b) {
  typename C2<R>::T v;
  v.x = a;
  v.y = b;
  return v;
}

template <typename Tdst, typename Tsrc>
__device__ __forceinline__ Tdst cvt(Tsrc v) {
  Tdst d;
  d.x = v.x;
  d.y = v.y;
  return d;
}

// out_m = scale_m * sum_q coef(q, m) * w_q * buf[q * es]: the dense sum of
// one output of a DST-I / DCT-I pair (see the file header).
template <typename R>
__device__ __forceinline__ typename C2<R>::T dense_out(const typename C2<R>::T* buf, int es, int L,
                                                       int M, int neumann, int inverse, int m,
                                                       const R* sinT, const R* cosT) {
  const int twoM = 2 * M;
  R sx = 0, sy = 0;
  if (!neumann) {
    const int step = m + 1;
    int t = step;
    for (int q = 0; q < L; ++q) {
      const R c = sinT[t];
      const typename C2<R>::T v = buf[q * es];
      sx += c * v.x;
      sy += c * v.y;
      t += step;
      if (t >= twoM) t -= twoM;
    }
    if (!inverse) {
      const R s = R(2) / R(M);
      sx *= s;
      sy *= s;
    }
  } else {
    int t = 0;
    for (int q = 0; q < L; ++q) {
      R c = cosT[t];
      if (!inverse && (q == 0 || q == L - 1)) c *= R(0.5);
      const typename C2<R>::T v = buf[q * es];
      sx += c * v.x;
      sy += c * v.y;
      t += m;
      if (t >= twoM) t -= twoM;
    }
    if (!inverse) {
      R s = R(2) / R(M);
      if (m == 0 || m == L - 1) s *= R(0.5);
      sx *= s;
      sy *= s;
    }
  }
  return mk<R>(sx, sy);
}

constexpr int kXLines = 4;      // x lines per workgroup
constexpr int kYCols = 8;       // x columns per y-transform workgroup

template <typename Tin, typename Tout, typename R>
__global__ __launch_bounds__(256) void xform_x_kernel(const Tin* __restrict__ in,
                                                      Tout* __restrict__ out, int nlines, int L,
                                                      int M, int neumann, int inverse,
                                                      const double* __restrict__ trig) {
  using T2 = typename C2<R>::T;
  extern __shared__ unsigned char smem_raw[];
  R* sinT = reinterpret_cast<R*>(smem_raw);
  R* cosT = sinT + 2 * M;
  T2* buf = reinterpret_cast<T2*>(cosT + 2 * M + ((4 * M) & 1));
  for (int t = threadIdx.x; t < 2 * M; t += blockDim.x) {
    sinT[t] = R(trig[t]);
    cosT[t] = R(trig[2 * M + t]);
  }
  const int line0 = blockIdx.x * kXLines;
  const int nl = min(kXLines, nlines - line0);
  const size_t base = size_t(line0) * L;
  for (int e = threadIdx.x; e < nl * L; e += blockDim.x) buf[e] = cvt<T2>(in[base + e]);
  __syncthreads();
  for (int e = threadIdx.x; e < nl * L; e += blockDim.x) {
    const int b = e / L, m = e - b * L;
    out[base + e] = cvt<Tout>(dense_out<R>(buf + b * L, 1, L, M, neumann, inverse, m, sinT, cosT));
  }
}

template <typename T2in, typename R>
__global__ __launch_bounds__(256) void xform_y_kernel(const T2in* __restrict__ in,
                                                      T2in* __restrict__ out, int nx, int L,
                                                      int M, int neumann, int inverse,
                                                      const double* __restrict__ trig) {
  using T2 = typename C2<R>::T;
  extern __shared__ unsigned char smem_raw[];
  R* sinT = reinterpret_cast<R*>(smem_raw);
  R* cosT = sinT + 2 * M;
  T2* buf = reinterpret_cast<T2*>(cosT + 2 * M + ((4 * M) & 1));
  for (int t = threadIdx.x; t < 2 * M; t += blockDim.x) {
    sinT[t] = R(trig[t]);
    cosT[t] = R(trig[2 * M + t]);
  }
  const int i0 = blockIdx.x * kYCols;
  const int nc = min(kYCols, nx - i0);
  const size_t zoff = size_t(blockIdx.y) * nx * L;
  for (int e = threadIdx.x; e < L * kYCols; e += blockDim.x) {
    const int q = e / kYCols, c = e - q * kYCols;
    if (c < nc) buf[c * L + q] = cvt<T2>(in[zoff + size_t(q) * nx + i0 + c]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < L * kYCols; e += blockDim.x) {
    const int m = e / kYCols, c = e - m * kYCols;
    if (c < nc)
      out[zoff + size_t(m) * nx + i0 + c] =
          cvt<T2in>(dense_out<R>(buf + c * L, 1, L, M, neumann, inverse, m, sinT, cosT));
  }
}

template <typename R>
__device__ __forceinline__ typename C2<R>::T cdiv(typename C2<R>::T a, typename C2<R>::T b) {
  const R d = b.x * b.x + b.y * b.y;
  return mk<R>((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

template <typename R>
__device__ __forceinline__ typename C2<R>::T cmulr(typename C2<R>::T a, typename C2<R>::T b) {
  return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One thread per transverse mode: Gaussian elimination without pivoting
// (Thomas) on T_z + shift I; c' goes to scratch, d' to the output, then back
// substitution in place.
template <typename R>
__global__ __launch_bounds__(256) void tridiag_z_kernel(const typename C2<R>::T* __restrict__ in,
                                                        typename C2<R>::T* __restrict__ out,
                                                        typename C2<R>::T* __restrict__ cp,
                                                        const double2* __restrict__ tri,
                                                        const double* __restrict__ lx,
                                                        const double* __restrict__ ly, double kap_re,
                                                        double kap_im, int nx, int ny, int nz) {
  using T2 = typename C2<R>::T;
  const int mode = blockIdx.x * blockDim.x + threadIdx.x;
  if (mode >= nx * ny) return;
  const int i = mode % nx, j = mode / nx;
  const size_t stride = size_t(nx) * ny;
  const T2 shift = mk<R>(R(kap_re + lx[i] + ly[j]), R(kap_im));
  T2 cprev = mk<R>(0, 0), dprev = mk<R>(0, 0);
  for (int l = 0; l < nz; ++l) {
    const T2 sub = cvt<T2>(tri[l]), dia = cvt<T2>(tri[nz + l]), sup = cvt<T2>(tri[2 * nz + l]);
    const T2 sc = cmulr<R>(sub, cprev);
    const T2 piv = mk<R>(dia.x + shift.x - sc.x, dia.y + shift.y - sc.y);
    const T2 rhs = in[mode + l * stride];
    const T2 sd = cmulr<R>(sub, dprev);
    cprev = cdiv<R>(sup, piv);
    dprev = cdiv<R>(mk<R>(rhs.x - sd.x, rhs.y - sd.y), piv);
    cp[mode + l * stride] = cprev;
    out[mode + l * stride] = dprev;
  }
  T2 xn = dprev;
  for (int l = nz - 2; l >= 0; --l) {
    const T2 c = cp[mode + l * stride];
    const T2 d = out[mode + l * stride];
    const T2 t = cmulr<R>(c, xn);
    xn = mk<R>(d.x - t.x, d.y - t.y);
    out[mode + l * stride] = xn;
  }
}

template <typename R>
hipError_t pinv_impl(h6_plan P, const double2* r, double2* z, hipStream_t s) {
  using T2 = typename C2<R>::T;
  const int nx = P->dims[0], ny = P->dims[1], nz = P->dims[2];
  T2* w0 = static_cast<T2*>(P->w_pc[0]);
  T2* w1 = static_cast<T2*>(P->w_pc[1]);
  T2* w2 = static_cast<T2*>(P->w_pc[2]);
  const AxisXform& X = P->ax[0];
  const AxisXform& Y = P->ax[1];
  const int nlines_x = ny * nz;
  const size_t shx = 4 * X.M * sizeof(R) + sizeof(R) + kXLines * X.L * sizeof(T2) + 16;
  const size_t shy = 4 * Y.M * sizeof(R) + sizeof(R) + kYCols * Y.L * sizeof(T2) + 16;
  const dim3 gx((nlines_x + kXLines - 1) / kXLines), gy((nx + kYCols - 1) / kYCols, nz);
  hipEvent_t ev;

  auto xform_x = [&](bool inv, auto* src, auto* dst) {
    timing_begin(P, KC_XFORM_X, s, &ev);
    if (X.fast)
      (void)launch_rader_x<R>(X.neumann, inv, src, dst, nlines_x, X.L, X.rader, s);
    else
      hipLaunchKernelGGL((xform_x_kernel<std::remove_cv_t<std::remove_pointer_t<decltype(src)>>,
                                         std::remove_pointer_t<decltype(dst)>, R>),
                         gx, dim3(256), shx, s, src, dst, nlines_x, X.L, X.M, X.neumann, inv ? 1 : 0,
                         P->d_trig_x);
    timing_end(P, KC_XFORM_X, s, ev);
  };
  auto xform_y = [&](bool inv, const T2* src, T2* dst) {
    timing_begin(P, KC_XFORM_Y, s, &ev);
    if (Y.fast)
      (void)launch_rader_y<R>(Y.neumann, inv, src, dst, nx, Y.L, nz, Y.rader, s);
    else
      hipLaunchKernelGGL((xform_y_kernel<T2, R>), gy, dim3(256), shy, s, src, dst, nx, Y.L, Y.M,
                         Y.neumann, inv ? 1 : 0, P->d_trig_y);
    timing_end(P, KC_XFORM_Y, s, ev);
  };
  xform_x(false, r, w0);
  xform_y(false, w0, w1);
  timing_begin(P, KC_TRIDIAG, s, &ev);
  hipLaunchKernelGGL((tridiag_z_kernel<R>), dim3((nx * ny + 255) / 256), dim3(256), 0, s, w1, w0,
                     w2, P->d_tri, P->d_lambda_x, P->d_lambda_y, P->kappa.real(),
                     P->kappa.imag(), nx, ny, nz);
  timing_end(P, KC_TRIDIAG, s, ev);
  xform_y(true, w0, w1);
  xform_x(true, static_cast<const T2*>(w1), z);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pinv(h6_plan P, const double2* r, double2* z, hipStream_t s) {
  if (P->p.precision == H6_MIXED) return pinv_impl<float>(P, r, z, s);
  return pinv_impl<double>(P, r, z, s);
}

}  // namespace h6
