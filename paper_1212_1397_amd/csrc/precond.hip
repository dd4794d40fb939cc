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
// Steps 1, 2, 4, 5 use the Rader FFT path for M = 257 (xform_rader.hip) and
// the dense basis-matrix products on the matrix cores otherwise
// (xform_dense.hip).  Compute type R is double (FP64 plans) or float (mixed
// plans, complex64 intermediates); the input r and output z are complex128 in
// both.
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

template <typename R>
__device__ __forceinline__ typename C2<R>::T cdiv(typename C2<R>::T a, typename C2<R>::T b) {
  const R d = b.x * b.x + b.y * b.y;
  return mk<R>((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

template <typename R>
__device__ __forceinline__ typename C2<R>::T cmulr(typename C2<R>::T a, typename C2<R>::T b) {
  return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Partitioned Gaussian elimination without pivoting (the Thomas algorithm
// with its recurrences re-associated) on T_z + shift I, one transverse mode per
// line.  A workgroup owns kLanes consecutive modes (lanes) and splits every
// z line into kSegs segments of S <= kSmax rows, one thread each, rows held in
// registers.  Thomas' recurrences are
//   c'_i = c_i / m_i,  m_i = b_i - a_i c'_{i-1}        (data independent),
//   d'_i = (d_i - a_i d'_{i-1}) / m_i                   (affine in d'_{i-1}),
//   x_i  = d'_i - c'_i x_{i+1}                           (affine in x_{i+1}).
// The c' value entering each segment depends only on the matrix, so the plan
// stores it (cstart[seg][mode], computed in FP64 at setup with the pivot
// check).  Each thread replays c' over its rows, composes the two affine maps
// over its segment, and the segment maps are chained in order through LDS.
// HBM traffic: one read and one write of the vector plus the small cstart table.
// launch shapes: kLanes modes x kSegs segments = 512 threads; 32 x 16 up to
// n'z = 272 (256-byte row segments), 16 x 32 above (n'z <= 544)

template <typename R>
__device__ __forceinline__ typename C2<R>::T csub(typename C2<R>::T a, typename C2<R>::T b) {
  return mk<R>(a.x - b.x, a.y - b.y);
}
template <typename R>
__device__ __forceinline__ typename C2<R>::T cadd(typename C2<R>::T a, typename C2<R>::T b) {
  return mk<R>(a.x + b.x, a.y + b.y);
}

// 1/x for x > 0: hardware reciprocal refined by Newton steps (FP64: two steps)
__device__ __forceinline__ double rcp_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_pos(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename R>
__device__ __forceinline__ typename C2<R>::T crecip(typename C2<R>::T b) {
  const R d = rcp_pos(b.x * b.x + b.y * b.y);
  return mk<R>(b.x * d, -b.y * d);
}

template <typename R, int kLanes, int kSegs, int kSmax>
__global__ __launch_bounds__(kLanes * kSegs) void tridiag_z_kernel(
    const typename C2<R>::T* __restrict__ in, typename C2<R>::T* __restrict__ out,
    const double2* __restrict__ tri, const typename C2<R>::T* __restrict__ cstart,
    const double* __restrict__ lx, const double* __restrict__ ly, double kap_re, double kap_im,
    int nx, int ny, int nz, const int* __restrict__ skip) {
  if (skip && *skip) return;
  using T2 = typename C2<R>::T;
  constexpr int kThr = kLanes * kSegs;
  constexpr int kTabPer = (3 * kMaxZ + kThr - 1) / kThr;
  __shared__ T2 sh[2][kSegs][kLanes];
  __shared__ T2 tz[kTabPer * kThr];  // sub-, main and super-diagonal of T_z (main without the shift)
  const int tid = threadIdx.x;
  const int lane = tid % kLanes;
  const int seg = tid / kLanes;
  const int nmodes = nx * ny;
  const int mode = blockIdx.x * kLanes + lane;
  const bool active = mode < nmodes;
  const int mc = active ? mode : nmodes - 1;
  const int i = mc % nx, j = mc / nx;
  const size_t stride = size_t(nx) * ny;
  const int S = (nz + kSegs - 1) / kSegs;
  const int r0 = min(seg * S, nz), cnt = min(S, nz - r0);
  const T2 one = mk<R>(1, 0), zero = mk<R>(0, 0);

  // All global reads are issued up front and unconditionally (clamped
  // indices): first the matrix (it is written to LDS first, so waiting for it
  // leaves the vector loads in flight), then the start value of c', the
  // transverse eigenvalues and this thread's rows of the vector.
  double2 tv[kTabPer];
#pragma unroll
  for (int k = 0; k < kTabPer; ++k) tv[k] = tri[min(tid + k * kThr, 3 * nz - 1)];
  const T2 cst = cstart[size_t(seg) * nmodes + mc];
  const double lxi = lx[i], lyj = ly[j];
  T2 d[kSmax], ip[kSmax];     // right-hand side, then d'; inverse pivots 1/m_i
#pragma unroll
  for (int u = 0; u < kSmax; ++u) d[u] = in[mc + size_t(min(r0 + u, nz - 1)) * stride];
#pragma unroll
  for (int k = 0; k < kTabPer; ++k) tz[tid + k * kThr] = cvt<T2>(tv[k]);   // entries past 3 n'z unused
  __syncthreads();
  const T2 shift = mk<R>(R(kap_re + lxi + lyj), R(kap_im));

  // The off-diagonals of T_z are real (1 inside, 0 or 2 on the end rows):
  // a and c scale complex values by real factors.
  auto scl = [](T2 v, R f) { return mk<R>(v.x * f, v.y * f); };
  // local pass: c' from the stored start value, inverse pivots, and the
  // affine map d'_{last} = A d'_{r0-1} + B
  T2 cprev = cst, A = one, B = zero;
#pragma unroll
  for (int u = 0; u < kSmax; ++u) {
    if (u < cnt) {
      const int r = r0 + u;
      const R a = tz[r].x, c = tz[2 * nz + r].x;
      const T2 b = cadd<R>(tz[nz + r], shift);
      ip[u] = crecip<R>(csub<R>(b, scl(cprev, a)));
      const T2 al = scl(ip[u], -a);
      A = cmulr<R>(al, A);
      B = cadd<R>(cmulr<R>(al, B), cmulr<R>(d[u], ip[u]));
      cprev = scl(ip[u], c);
    } else {
      ip[u] = zero;
    }
  }
  sh[0][seg][lane] = A;
  sh[1][seg][lane] = B;
  __syncthreads();
  T2 dprev = zero;
  for (int s2 = 0; s2 < seg; ++s2) dprev = cadd<R>(cmulr<R>(sh[0][s2][lane], dprev), sh[1][s2][lane]);
  // replay d', then compose the back substitution x_{r0} = C x_{r0+cnt} + D
#pragma unroll
  for (int u = 0; u < kSmax; ++u) {
    if (u < cnt) {
      const R a = tz[r0 + u].x;
      d[u] = cmulr<R>(csub<R>(d[u], scl(dprev, a)), ip[u]);
      dprev = d[u];
    }
  }
  T2 C = one, D = zero;
#pragma unroll
  for (int u = kSmax - 1; u >= 0; --u) {
    if (u < cnt) {
      const T2 ncp = scl(ip[u], -tz[2 * nz + r0 + u].x);     // -c'_u
      D = cadd<R>(d[u], cmulr<R>(ncp, D));
      C = cmulr<R>(ncp, C);
    }
  }
  __syncthreads();
  sh[0][seg][lane] = C;
  sh[1][seg][lane] = D;
  __syncthreads();
  T2 x = zero;
  for (int s2 = kSegs - 1; s2 > seg; --s2) x = cadd<R>(cmulr<R>(sh[0][s2][lane], x), sh[1][s2][lane]);
#pragma unroll
  for (int u = kSmax - 1; u >= 0; --u) {
    if (u < cnt) {
      x = csub<R>(d[u], cmulr<R>(scl(ip[u], tz[2 * nz + r0 + u].x), x));
      if (active) out[mode + size_t(r0 + u) * stride] = x;
    }
  }
}

// z = A_p^{-1} r, or z += A_p^{-1} r with acc != 0 (folded into the last pass)
template <typename R, typename Tin, typename Tout>
hipError_t pinv_impl(h6_plan P, const Tin* r, Tout* z, hipStream_t s, int part, int acc = 0) {
  using T2 = typename C2<R>::T;
  const int nx = P->dims[0], ny = P->dims[1], nz = P->dims[2];
  T2* w0 = static_cast<T2*>(P->w_pc[0]);
  T2* w1 = static_cast<T2*>(P->w_pc[1]);
  const AxisXform& X = P->ax[0];
  const AxisXform& Y = P->ax[1];
  const int nlines_x = ny * nz;
  hipEvent_t ev;

  const double Nd = double(P->N);
  auto xform_x = [&](bool inv, auto* src, auto* dst, int accumulate) {
    timing_begin(P, KC_XFORM_X, s, &ev);
    if (X.fast)
      (void)launch_rader_x<R>(X.neumann, inv, src, dst, nlines_x, X.L, X.rader, s, accumulate, X.lines,
                              P->skip);
    else
      (void)launch_dense_x<R>(X, inv, src, dst, nlines_x, accumulate, s, P->skip);
    timing_end(P, KC_XFORM_X, s, ev, Nd * (sizeof(*src) + sizeof(*dst) * (accumulate ? 2 : 1)));
  };
  auto xform_y = [&](bool inv, const T2* src, T2* dst) {
    timing_begin(P, KC_XFORM_Y, s, &ev);
    if (Y.fast)
      (void)launch_rader_y<R>(Y.neumann, inv, src, dst, nx, Y.L, nz, Y.rader, s, Y.lines, P->skip);
    else
      (void)launch_dense_y<R>(Y, inv, src, dst, nx, nz, s, P->skip);
    timing_end(P, KC_XFORM_Y, s, ev, Nd * 2 * sizeof(T2));
  };
  if (part & PINV_FIRST) xform_x(false, r, w0, 0);
  if (!(part & PINV_REST)) return hipGetLastError();
  xform_y(false, w0, w1);
  timing_begin(P, KC_TRIDIAG, s, &ev);
  {
    const double kr = P->kappa.real(), ki = P->kappa.imag();
    const T2* cst = static_cast<const T2*>(P->d_cstart);
    auto go = [&](auto kern, int lanes) {
      hipLaunchKernelGGL(kern, dim3((nx * ny + lanes - 1) / lanes), dim3(512), 0, s, w1, w0, P->d_tri, cst,
                         P->d_lambda_x, P->d_lambda_y, kr, ki, nx, ny, nz, P->skip);
    };
    if (z_segments(nz, sizeof(R) == 4) == 16) {
      if (nz <= 16 * 5) go(tridiag_z_kernel<R, 32, 16, 5>, 32);
      else if (nz <= 16 * 9) go(tridiag_z_kernel<R, 32, 16, 9>, 32);
      else go(tridiag_z_kernel<R, 32, 16, 17>, 32);
    } else {
      if (nz <= 32 * 9) go(tridiag_z_kernel<R, 16, 32, 9>, 16);
      else go(tridiag_z_kernel<R, 16, 32, 17>, 16);
    }
  }
  timing_end(P, KC_TRIDIAG, s, ev, Nd * 2 * sizeof(T2));
  xform_y(true, w0, w1);
  xform_x(true, static_cast<const T2*>(w1), z, acc);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pinv(h6_plan P, const double2* r, double2* z, hipStream_t s, int part) {
  if (P->p.precision == H6_MIXED) return pinv_impl<float, double2, double2>(P, r, z, s, part);
  return pinv_impl<double, double2, double2>(P, r, z, s, part);
}

hipError_t launch_pinv_acc(h6_plan P, const double2* r, double2* U, hipStream_t s, int part) {
  if (P->p.precision == H6_MIXED) return pinv_impl<float, double2, double2>(P, r, U, s, part, 1);
  return pinv_impl<double, double2, double2>(P, r, U, s, part, 1);
}

hipError_t launch_pinv_acc_f32in(h6_plan P, const float2* r, double2* U, hipStream_t s, int part) {
  if (P->p.precision != H6_MIXED) return hipErrorInvalidValue;
  return pinv_impl<float, float2, double2>(P, r, U, s, part, 1);
}

hipError_t launch_pinv_f32out(h6_plan P, const double2* r, float2* z, hipStream_t s, int part) {
  if (P->p.precision != H6_MIXED) return hipErrorInvalidValue;
  return pinv_impl<float, double2, float2>(P, r, z, s, part);
}

}  // namespace h6
