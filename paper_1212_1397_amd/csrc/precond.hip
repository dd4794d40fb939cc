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
#include <mutex>
#include <type_traits>
#include <vector>

#include "h6_internal.h"

namespace h6 {

// Fixed device work space of helmholtz6_apply_Pinv_noalloc: the two
// intermediate vectors of the five passes, for callers that cannot allocate.
// Every GPU the library runs on holds one copy until the process ends.  In
// host code the name is only a host-side handle: kernels receive the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticWorkBytes];

namespace {
std::mutex g_scratch_mutex;
std::vector<void*> g_scratch_addr;   // per device ordinal, resolved once
}  // namespace

hipError_t static_work_address(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> g(g_scratch_mutex);
  if (size_t(dev) >= g_scratch_addr.size()) g_scratch_addr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

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

template <typename R>
__device__ __forceinline__ typename C2<R>::T cmulr(typename C2<R>::T a, typename C2<R>::T b) {
  return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

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

// Partitioned Gaussian elimination without pivoting (the Thomas algorithm
// with its recurrences re-associated) on T_z + shift I, one transverse mode per
// line.  With the end rows scaled as described at ZEnds, every off-diagonal is
// 1 and the main diagonal is b = shift - 2 except on rows 0 and n'z - 1, so
// Thomas' recurrences read
//   p_i = 1 / (b_i - c'_{i-1}),  c'_i = p_i                 (data independent),
//   d'_i = p_i (d_i - d'_{i-1})                            (affine in d'_{i-1}),
//   x_i  = d'_i - p_i x_{i+1}                               (affine in x_{i+1}).
// A workgroup owns kLanes consecutive modes (lanes) and splits every z line
// into kSegs segments of S <= kSmax rows, one thread each, rows held in
// registers.  The c' value entering each segment depends only on the matrix,
// so the plan stores it (cstart[seg][mode], computed in FP64 at setup with the
// pivot check).  Each thread replays c' over its rows and composes both affine
// maps over its segment: their linear parts are the same product of -p_i, so
// one product serves the forward and the backward chain.  The segment maps are
// chained in order through LDS.  Row 0 of the system never sees the value
// entering from above (it is zero) and row n'z - 1 never sees the one from
// below, so their missing off-diagonal needs no special case.
// HBM traffic: one read and one write of the vector plus the small cstart table.
// launch shapes: kLanes modes x kSegs segments = 512 threads; 32 x 16 up to
// n'z = 272 (256-byte row segments), 16 x 32 above (n'z <= 544)

template <typename R, int kLanes, int kSegs, int kSmax>
__global__ __launch_bounds__(kLanes * kSegs) void tridiag_z_kernel(
    const typename C2<R>::T* __restrict__ in, typename C2<R>::T* __restrict__ out,
    const typename C2<R>::T* __restrict__ cstart, const double* __restrict__ lx,
    const double* __restrict__ ly, const double* __restrict__ zp, int nx, int ny, int nz,
    const int* __restrict__ skip) {
  if (skip && *skip) return;
  // kappa and the scaled end rows (ZEnds), from device memory (kZParams doubles)
  const double kap_re = zp[0], kap_im = zp[1];
  const ZEnds ends{zp[2], zp[3], zp[4], zp[5], zp[6], zp[7]};
  using T2 = typename C2<R>::T;
  __shared__ T2 sh[2][kSegs][kLanes];
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
  // the last row sits in segment segL at offset uL (the same for every thread)
  const int segL = (nz - 1) / S, uL = nz - 1 - segL * S;
  const bool first = seg == 0, last = seg == segL;
  const T2 one = mk<R>(1, 0), zero = mk<R>(0, 0);

  // global reads up front, with clamped indices
  const T2 cst = cstart[size_t(seg) * nmodes + mc];
  const double lxi = lx[i], lyj = ly[j];
  T2 d[kSmax], p[kSmax];     // right-hand side, then d'; inverse pivots p_i
#pragma unroll
  for (int u = 0; u < kSmax; ++u) d[u] = in[mc + size_t(min(r0 + u, nz - 1)) * stride];

  auto scl = [](T2 v, R f) { return mk<R>(v.x * f, v.y * f); };
  const T2 shift = mk<R>(R(kap_re + lxi + lyj), R(kap_im));
  const T2 bM = cadd<R>(mk<R>(-2, 0), shift);
  const T2 bF = scl(cadd<R>(mk<R>(R(ends.b0_re), R(ends.b0_im)), shift), R(ends.s0));
  const T2 bL = scl(cadd<R>(mk<R>(R(ends.bl_re), R(ends.bl_im)), shift), R(ends.sl));
  if (first) d[0] = scl(d[0], R(ends.s0));
#pragma unroll
  for (int u = 0; u < kSmax; ++u)
    if (u == uL && last) d[u] = scl(d[u], R(ends.sl));

  // local pass: inverse pivots from the stored c', and the affine map
  // d'_{last} = Q d'_{r0-1} + B
  T2 cprev = cst, Q = one, B = zero;
#pragma unroll
  for (int u = 0; u < kSmax; ++u) {
    if (u < cnt) {
      T2 b = bM;
      if (u == 0 && first) b = bF;
      if (u == uL && last) b = bL;
      p[u] = crecip<R>(csub<R>(b, cprev));
      Q = cmulr<R>(mk<R>(-p[u].x, -p[u].y), Q);
      B = cmulr<R>(p[u], csub<R>(d[u], B));
      cprev = p[u];
    } else {
      p[u] = zero;
    }
  }
  sh[0][seg][lane] = Q;
  sh[1][seg][lane] = B;
  __syncthreads();
  T2 dprev = zero;
  for (int s2 = 0; s2 < seg; ++s2) dprev = cadd<R>(cmulr<R>(sh[0][s2][lane], dprev), sh[1][s2][lane]);
  // replay d', then compose the back substitution x_{r0} = Q x_{r0+cnt} + D
#pragma unroll
  for (int u = 0; u < kSmax; ++u) {
    if (u < cnt) {
      d[u] = cmulr<R>(p[u], csub<R>(d[u], dprev));
      dprev = d[u];
    }
  }
  T2 D = zero;
#pragma unroll
  for (int u = kSmax - 1; u >= 0; --u)
    if (u < cnt) D = csub<R>(d[u], cmulr<R>(p[u], D));
  __syncthreads();
  sh[1][seg][lane] = D;
  __syncthreads();
  T2 x = zero;
  for (int s2 = kSegs - 1; s2 > seg; --s2) x = cadd<R>(cmulr<R>(sh[0][s2][lane], x), sh[1][s2][lane]);
#pragma unroll
  for (int u = kSmax - 1; u >= 0; --u) {
    if (u < cnt) {
      x = csub<R>(d[u], cmulr<R>(p[u], x));
      if (active) out[mode + size_t(r0 + u) * stride] = x;
    }
  }
}

// z = A_p^{-1} r, or z += A_p^{-1} r with acc != 0 (folded into the last pass)
// (ws: the two work vectors; NULL: the plan's own)
template <typename R, typename Tin, typename Tout>
hipError_t pinv_impl(h6_plan P, const Tin* r, Tout* z, hipStream_t s, int part, int acc = 0,
                     void* const* ws = nullptr) {
  using T2 = typename C2<R>::T;
  const int nx = P->dims[0], ny = P->dims[1], nz = P->dims[2];
  T2* w0 = static_cast<T2*>(ws ? ws[0] : P->w_pc[0]);
  T2* w1 = static_cast<T2*>(ws ? ws[1] : P->w_pc[1]);
  const AxisXform& X = P->ax[0];
  const AxisXform& Y = P->ax[1];
  const int nlines_x = ny * nz;
  hipEvent_t ev;

  const double Nd = double(P->N);
  // the first error a transform launcher reports without launching (a shape
  // its kernels do not take); launch failures proper show in hipGetLastError
  hipError_t refused = hipSuccess;
  auto note = [&](hipError_t e) {
    if (refused == hipSuccess && e != hipSuccess) refused = e;
  };
  auto xform_x = [&](bool inv, auto* src, auto* dst, int accumulate) {
    timing_begin(P, KC_XFORM_X, s, &ev);
    if (X.fast == 1)
      note(launch_rader_x<R>(X.neumann, inv, src, dst, nlines_x, X.L, X.rader, s, accumulate, X.lines,
                             P->skip));
    else if (X.fast == 2)
      note(launch_bluestein_x<R>(X.neumann, inv, src, dst, nlines_x, X.L, X.blue, s, accumulate, P->skip));
    else
      note(launch_dense_x<R>(X, inv, src, dst, nlines_x, accumulate, s, P->skip));
    timing_end(P, KC_XFORM_X, s, ev, Nd * (sizeof(*src) + sizeof(*dst) * (accumulate ? 2 : 1)));
  };
  auto xform_y = [&](bool inv, const T2* src, T2* dst) {
    timing_begin(P, KC_XFORM_Y, s, &ev);
    if (Y.fast == 1)
      note(launch_rader_y<R>(Y.neumann, inv, src, dst, nx, Y.L, nz, Y.rader, s, Y.lines, P->skip));
    else if (Y.fast == 2)
      note(launch_bluestein_y<R>(Y.neumann, inv, src, dst, nx, Y.L, nz, Y.blue, s, P->skip));
    else
      note(launch_dense_y<R>(Y, inv, src, dst, nx, nz, s, P->skip));
    timing_end(P, KC_XFORM_Y, s, ev, Nd * 2 * sizeof(T2));
  };
  if (part & PINV_FIRST) xform_x(false, r, w0, 0);
  if (!(part & PINV_REST)) return refused != hipSuccess ? refused : hipGetLastError();
  xform_y(false, w0, w1);
  timing_begin(P, KC_TRIDIAG, s, &ev);
  {
    const T2* cst = static_cast<const T2*>(P->d_cstart);
    auto go = [&](auto kern, int lanes) {
      hipLaunchKernelGGL(kern, dim3((nx * ny + lanes - 1) / lanes), dim3(512), 0, s, w1, w0, cst,
                         P->d_lambda_x, P->d_lambda_y, P->d_zparams, nx, ny, nz, P->skip);
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
  return refused != hipSuccess ? refused : hipGetLastError();
}

}  // namespace

hipError_t launch_pinv(h6_plan P, const double2* r, double2* z, hipStream_t s, int part) {
  if (P->p.precision == H6_MIXED) return pinv_impl<float, double2, double2>(P, r, z, s, part);
  return pinv_impl<double, double2, double2>(P, r, z, s, part);
}

hipError_t launch_pinv_ws(h6_plan P, const double2* r, double2* z, void* const ws[2], hipStream_t s) {
  if (P->p.precision == H6_MIXED) return pinv_impl<float, double2, double2>(P, r, z, s, PINV_ALL, 0, ws);
  return pinv_impl<double, double2, double2>(P, r, z, s, PINV_ALL, 0, ws);
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
