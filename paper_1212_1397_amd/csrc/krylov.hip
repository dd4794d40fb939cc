// Vector kernels of the Krylov loops, complex128.
//
// GMRES orthogonalisation is modified Gram-Schmidt written in its inverse
// compact WY form: for a new vector w and an (unnormalised) basis Q, one pass
// forms all inner products <q_i, w>; a one-wave kernel turns them into the MGS
// coefficients with the Gram matrix of the basis (a small triangular solve);
// one more pass applies w -= sum_i c_i q_i and, while the basis streams by,
// forms |w|^2 and the Gram row <q_i, w> of the new basis vector.  This moves
// (2j + 4) vectors per Arnoldi step instead of (4j + 5) for the
// one-projection-per-pass form, with the same coefficients in exact
// arithmetic.
//
// Reductions are deterministic: a fixed grid (one full wave of resident
// blocks) writes one partial per block and component in
// grid-stride order, and a second kernel sums each component's partials in a
// fixed tree order.  Load loops use compile-time vector counts, so every load
// of an element is issued before the first one is waited on.
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

// |a - b|^2 partials (component 0)
__global__ __launch_bounds__(kThreads) void diff_norm2_kernel(const double2* __restrict__ a,
                                                              const double2* __restrict__ b, size_t n,
                                                              double* __restrict__ partials) {
  double v[1] = {0.0};
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    const double2 x = a[i], y = b[i];
    const double dx = x.x - y.x, dy = x.y - y.y;
    v[0] = fma(dx, dx, fma(dy, dy, v[0]));
  }
  block_store<1>(v, partials, 0, gridDim.x);
}

// For basis vectors q_{i0 .. i0+CNT-1} (stride n from Q): partials of
// <q_i, w> (components 2 i, 2 i + 1 = re, im).  CNT is a compile-time count so
// that all CNT + 1 loads of an element are issued back to back, unconditionally.
template <int CNT>
__global__ __launch_bounds__(kThreads) void block_dots_kernel(const double2* __restrict__ Q, int i0,
                                                              const double2* __restrict__ w,
                                                              size_t n, double* __restrict__ partials,
                                                              const int* __restrict__ skip) {
  if (skip && *skip) return;
  double acc[2 * CNT];
#pragma unroll
  for (int c = 0; c < 2 * CNT; ++c) acc[c] = 0.0;
  const double2* __restrict__ Qb = Q + size_t(i0) * n;
  for (size_t k = blockIdx.x * size_t(kThreads) + threadIdx.x; k < n; k += size_t(gridDim.x) * kThreads) {
    const double2 x = w[k];
    double2 q[CNT];
#pragma unroll
    for (int i = 0; i < CNT; ++i) q[i] = Qb[size_t(i) * n + k];
#pragma unroll
    for (int i = 0; i < CNT; ++i) {
      acc[2 * i] = fma(q[i].x, x.x, fma(q[i].y, x.y, acc[2 * i]));
      acc[2 * i + 1] = fma(q[i].x, x.y, fma(-q[i].y, x.x, acc[2 * i + 1]));
    }
  }
  block_store<2 * CNT>(acc, partials, 2 * i0, gridDim.x);
}

// w -= sum_{i < m} c_i q_i, then partials of |w|^2 (component 0) and of
// <q_i, w> for i < MG = min(m, kGramMax) (components 1 + 2 i, 2 + 2 i): the
// Gram row of the new basis vector w, formed while the basis is streamed for
// the update.  Vectors beyond MG (m > kGramMax) are applied four at a time
// (loads past m re-read q_{m-1} with a zero coefficient).
template <int MG>
__global__ __launch_bounds__(kThreads) void update_gram_kernel(double2* __restrict__ w,
                                                               const double2* __restrict__ Q,
                                                               const double2* __restrict__ c, int m,
                                                               size_t n, double* __restrict__ partials,
                                                               const int* __restrict__ skip) {
  if (skip && *skip) return;
  double acc[1 + 2 * MG];
#pragma unroll
  for (int i = 0; i < 1 + 2 * MG; ++i) acc[i] = 0.0;
  double2 cf[MG];
#pragma unroll
  for (int i = 0; i < MG; ++i) cf[i] = c[i];
  for (size_t k = blockIdx.x * size_t(kThreads) + threadIdx.x; k < n; k += size_t(gridDim.x) * kThreads) {
    double2 x = w[k];
    double2 q[MG];
#pragma unroll
    for (int i = 0; i < MG; ++i) q[i] = Q[size_t(i) * n + k];
#pragma unroll
    for (int i = 0; i < MG; ++i) {
      x.x -= cf[i].x * q[i].x - cf[i].y * q[i].y;
      x.y -= cf[i].x * q[i].y + cf[i].y * q[i].x;
    }
    for (int i = MG; i < m; i += 4) {
      double2 qq[4], a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ii = i + u < m ? i + u : m - 1;
        qq[u] = Q[size_t(ii) * n + k];
        a[u] = i + u < m ? c[i + u] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x.x -= a[u].x * qq[u].x - a[u].y * qq[u].y;
        x.y -= a[u].x * qq[u].y + a[u].y * qq[u].x;
      }
    }
    w[k] = x;
    acc[0] = fma(x.x, x.x, fma(x.y, x.y, acc[0]));
#pragma unroll
    for (int i = 0; i < MG; ++i) {
      acc[1 + 2 * i] = fma(q[i].x, x.x, fma(q[i].y, x.y, acc[1 + 2 * i]));
      acc[2 + 2 * i] = fma(q[i].x, x.y, fma(-q[i].y, x.x, acc[2 + 2 * i]));
    }
  }
  block_store<1 + 2 * MG>(acc, partials, 0, gridDim.x);
}

// MGS coefficients of Arnoldi step j (one wave):
//   nu_j = |q~_j|,  G_{j,i} = conj(<q~_i, q~_j>) / (nu_i nu_j)  (i < j),
//   h_i = <q~_i, w~> / (nu_i nu_j) - sum_{l<i} G_{i,l} h_l,  c_i = nu_j h_i / nu_i.
// For j < 64 the Gram rows are staged in LDS (packed lower triangle, loads
// batched) and the recurrence runs column by column: lane i holds h_i, and
// at step l the final h_l is broadcast by a lane shuffle and subtracted from
// the lanes below.  Larger j: the recurrence runs over i, each inner sum split
// over the lanes and reduced in a fixed order.
constexpr int kCoefMax = 257;
constexpr int kCoefFast = 64;
__global__ __launch_bounds__(64) void mgs_coef_kernel(int j, const double* __restrict__ dots,
                                                      const double* __restrict__ nrow,
                                                      const double* __restrict__ gram2,
                                                      double* __restrict__ nu, double2* __restrict__ G,
                                                      int gdim, double2* __restrict__ hcol,
                                                      double2* __restrict__ coef,
                                                      const int* __restrict__ skip,
                                                      double2* __restrict__ hmirror) {
  if (skip && *skip) return;
  __shared__ double2 h[kCoefMax];
  __shared__ double2 Gt[kCoefFast * (kCoefFast - 1) / 2];   // rows 1..63, entry (r, c) at r(r-1)/2 + c
  const int t = threadIdx.x;
  const double nuj = sqrt(fmax(nrow[0], 0.0));
  if (t == 0) nu[j] = nuj;
  const bool fast = j < kCoefFast;
  for (int i = t; i < j; i += 64) {
    double lx, ly;
    if (i < kGramMax) {
      lx = nrow[1 + 2 * i];
      ly = nrow[2 + 2 * i];
    } else {
      lx = gram2[2 * (i - kGramMax)];
      ly = gram2[2 * (i - kGramMax) + 1];
    }
    const double d = nu[i] * nuj;
    const double2 gv = make_double2(lx / d, -ly / d);
    G[size_t(j) * gdim + i] = gv;
    if (fast) Gt[j * (j - 1) / 2 + i] = gv;
  }
  if (fast) {
    const int cnt = j * (j - 1) / 2;          // entries of rows 1 .. j-1
    for (int e0 = 0; e0 < cnt; e0 += 4 * 64) {
      double2 v[4];
      int at[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {           // four loads in flight per lane
        const int e = e0 + u * 64 + t;
        at[u] = -1;
        if (e < cnt) {
          int r = int((1.0 + sqrt(1.0 + 8.0 * double(e))) * 0.5);
          while (r * (r - 1) / 2 > e) --r;
          while ((r + 1) * r / 2 <= e) ++r;
          v[u] = G[size_t(r) * gdim + (e - r * (r - 1) / 2)];
          at[u] = e;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (at[u] >= 0) Gt[at[u]] = v[u];
    }
    __syncthreads();
    double2 acc = make_double2(0.0, 0.0);
    double nui = 1.0;
    if (t <= j) {
      nui = t == j ? nuj : nu[t];
      const double d = nui * nuj;
      acc = make_double2(dots[2 * t] / d, dots[2 * t + 1] / d);
    }
    for (int l = 0; l < j; ++l) {
      const double hx = __shfl(acc.x, l, 64), hy = __shfl(acc.y, l, 64);   // h_l, final
      if (t > l && t <= j) {
        const double2 g = Gt[t * (t - 1) / 2 + l];
        acc.x -= g.x * hx - g.y * hy;
        acc.y -= g.x * hy + g.y * hx;
      }
    }
    if (t <= j) {
      hcol[t] = acc;
      if (hmirror) hmirror[t] = acc;
      const double f = nuj / nui;
      coef[t] = make_double2(f * acc.x, f * acc.y);
    }
    return;
  }
  __syncthreads();
  for (int i = 0; i <= j; ++i) {
    double ax = 0.0, ay = 0.0;
    for (int l = t; l < i; l += 64) {
      const double2 g = G[size_t(i) * gdim + l], hl = h[l];
      ax += g.x * hl.x - g.y * hl.y;
      ay += g.x * hl.y + g.y * hl.x;
    }
    for (int o = 32; o > 0; o >>= 1) {
      ax += __shfl_xor(ax, o, 64);
      ay += __shfl_xor(ay, o, 64);
    }
    if (t == 0) {
      const double nui = i == j ? nuj : nu[i];
      const double d = nui * nuj;
      const double2 hv = make_double2(dots[2 * i] / d - ax, dots[2 * i + 1] / d - ay);
      h[i] = hv;
      hcol[i] = hv;
      if (hmirror) hmirror[i] = hv;
      const double f = nuj / nui;
      coef[i] = make_double2(f * hv.x, f * hv.y);
    }
    __syncthreads();
  }
}

// out[c] = sum_b partials[c * nblocks + b], one block per component
__global__ __launch_bounds__(kThreads) void reduce_cols_kernel(const double* __restrict__ partials,
                                                               int nblocks, double* __restrict__ out,
                                                               const int* __restrict__ skip,
                                                               double* __restrict__ hout0) {
  if (skip && *skip) return;
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
  if (threadIdx.x == 0) {
    out[blockIdx.x] = s[0];
    if (hout0 && blockIdx.x == 0) hout0[0] = s[0];
  }
}

// out (+)= sum_i y_i V_i, V_i = V + i * n (FP64 arithmetic).  Vectors are
// taken eight at a time with all eight loads issued together (loads past m
// re-read V_{m-1} with a zero coefficient).
template <typename TV>
__global__ __launch_bounds__(kThreads) void multi_axpy_kernel(double2* __restrict__ out,
                                                              const TV* __restrict__ V,
                                                              const double2* __restrict__ y, int m,
                                                              size_t n, int accumulate,
                                                              const int* __restrict__ mdev) {
  constexpr int kU = 8;
  if (mdev) m = min(m, *mdev);
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    double2 acc = accumulate ? out[i] : make_double2(0.0, 0.0);
    for (int j = 0; j < m; j += kU) {
      TV vv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) vv[u] = V[size_t(j + u < m ? j + u : m - 1) * n + i];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const double2 c = j + u < m ? y[j + u] : make_double2(0.0, 0.0);
        const double2 v = make_double2(double(vv[u].x), double(vv[u].y));
        acc.x += c.x * v.x - c.y * v.y;
        acc.y += c.x * v.y + c.y * v.x;
      }
    }
    out[i] = acc;
  }
}

// Chebyshev step: e = c1 e + c2 t; U += e
__global__ __launch_bounds__(kThreads) void cheb_update_kernel(double2* __restrict__ e,
                                                               const double2* __restrict__ t,
                                                               double2* __restrict__ U, double c1,
                                                               double c2, size_t n) {
  for (size_t i = blockIdx.x * size_t(kThreads) + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
    const double2 a = e[i], b = t[i], u = U[i];
    const double2 v = make_double2(c1 * a.x + c2 * b.x, c1 * a.y + c2 * b.y);
    e[i] = v;
    U[i] = make_double2(u.x + v.x, u.y + v.y);
  }
}

// Complex Givens rotation (c real, s complex) with [c s; -conj(s) c] [a; b] = [r; 0], b real >= 0.
__device__ void givens_rot(double2 a, double b, double& c, double2& s, double2& r) {
  const double aa = hypot(a.x, a.y);
  if (b == 0.0) { c = 1.0; s = make_double2(0.0, 0.0); r = a; return; }
  if (aa == 0.0) { c = 0.0; s = make_double2(1.0, 0.0); r = make_double2(b, 0.0); return; }
  const double t = hypot(aa, b);
  const double2 ph = make_double2(a.x / aa, a.y / aa);
  c = aa / t;
  s = make_double2(ph.x * b / t, ph.y * b / t);
  r = make_double2(ph.x * t, ph.y * t);
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }

// One step of the least-squares update of a whole-cycle graph (one thread;
// the same arithmetic as the host path of the per-step solver).
__global__ __launch_bounds__(64) void givens_step_kernel(int j, int m, const double* __restrict__ nrow,
                                                         const double* __restrict__ nu,
                                                         const double2* __restrict__ hcol, GivensState st,
                                                         const double* __restrict__ prm) {
  if (*st.stop) return;
  if (threadIdx.x != 0) return;
  double2* Rj = st.R + size_t(j) * m;
  for (int i = 0; i <= j; ++i) Rj[i] = hcol[i];
  const double nuj = nu[j];
  const double hn = sqrt(fmax(nrow[0], 0.0)) / nuj;
  if (j == 0) st.g[0] = make_double2(nuj, 0.0);
  for (int i = 0; i < j; ++i) {
    const double c = st.cs[i];
    const double2 sn = st.sn[i], a = Rj[i], b = Rj[i + 1];
    const double2 t = make_double2(c * a.x + zmul(sn, b).x, c * a.y + zmul(sn, b).y);
    const double2 u = zmul(zconj(sn), a);
    Rj[i + 1] = make_double2(-u.x + c * b.x, -u.y + c * b.y);
    Rj[i] = t;
  }
  double c;
  double2 sr, rr;
  givens_rot(Rj[j], hn, c, sr, rr);
  st.cs[j] = c;
  st.sn[j] = sr;
  Rj[j] = rr;
  const double2 gj = st.g[j];
  const double2 gn = zmul(zconj(sr), gj);
  st.g[j + 1] = make_double2(-gn.x, -gn.y);
  st.g[j] = make_double2(c * gj.x, c * gj.y);
  const double est = hypot(gn.x, gn.y) / prm[1];
  st.est[j] = est;
  *st.jdone = j + 1;
  const bool breakdown = !(hn > 1e-300);
  if (est <= prm[2] || double(j + 1) >= prm[0] || breakdown || !isfinite(est)) *st.stop = 1;
}

// y = R^{-1} g over the steps done; y_i / nu_i for the unnormalised basis;
// zero beyond (one thread)
__global__ __launch_bounds__(64) void lsq_solve_kernel(int m, GivensState st, const double* __restrict__ nu,
                                                       double2* __restrict__ y) {
  if (threadIdx.x != 0) return;
  const int jd = min(max(*st.jdone, 0), m);
  for (int i = m - 1; i >= jd; --i) y[i] = make_double2(0.0, 0.0);
  for (int i = jd - 1; i >= 0; --i) {
    double2 acc = st.g[i];
    for (int k = i + 1; k < jd; ++k) {
      const double2 p = zmul(st.R[size_t(k) * m + i], y[k]);
      acc.x -= p.x;
      acc.y -= p.y;
    }
    const double2 d = st.R[size_t(i) * m + i];
    const double dd = d.x * d.x + d.y * d.y;
    y[i] = make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd);
  }
  // the basis is stored unnormalised: coefficients of q~_i are y_i / nu_i
  for (int i = 0; i < jd; ++i) y[i] = make_double2(y[i].x / nu[i], y[i].y / nu[i]);
}

__global__ void clear_int_kernel(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

int grid_for(size_t n) {
  const size_t b = (n + kThreads - 1) / kThreads;
  return int(b < size_t(kRedBlocks) ? (b > 0 ? b : 1) : kRedBlocks);
}

constexpr int kDotChunk = 16;
constexpr int kGramChunk = kGramMax;

}  // namespace

hipError_t launch_mgs_coef(int j, const double* dots, const double* nrow, const double* gram2,
                           double* nu, double2* G, int gdim, double2* hcol, double2* coef,
                           hipStream_t s, const int* skip, double2* hmirror) {
  if (j < 0 || j >= kCoefMax || j >= gdim) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mgs_coef_kernel, dim3(1), dim3(64), 0, s, j, dots, nrow, gram2, nu, G, gdim,
                     hcol, coef, skip, hmirror);
  return hipGetLastError();
}

hipError_t launch_norm2(const double2* a, size_t n, double* partials, double* out, hipStream_t s) {
  hipLaunchKernelGGL(norm2_kernel, dim3(kRedBlocks), dim3(kThreads), 0, s, a, n, partials);
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(1), dim3(kThreads), 0, s, partials, kRedBlocks, out,
                     static_cast<const int*>(nullptr), static_cast<double*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_reduce_sum_skip(const double* partials, int nparts, double* out, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(1), dim3(kThreads), 0, s, partials, nparts, out, skip,
                     static_cast<double*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_diff_norm2(const double2* a, const double2* b, size_t n, double* partials, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(diff_norm2_kernel, dim3(kRedBlocks), dim3(kThreads), 0, s, a, b, n, partials);
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(1), dim3(kThreads), 0, s, partials, kRedBlocks, out,
                     static_cast<const int*>(nullptr), static_cast<double*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_reduce_sum(const double* partials, int nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(1), dim3(kThreads), 0, s, partials, nparts, out,
                     static_cast<const int*>(nullptr), static_cast<double*>(nullptr));
  return hipGetLastError();
}

// Grid of the reductions: one full wave of resident blocks of the widest
// block_dots instance (no tail), at most 2048 (the partials capacity: 514
// components x 2048 blocks).  The same grid serves every instance: more
// blocks did not help the narrow ones.
int reduction_blocks() {
  static const int blocks = [] {     // initialised once, thread-safe
    int dev = 0, cus = 0, per = 0, b = kRedBlocks;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, block_dots_kernel<kDotChunk>, kThreads, 0) ==
            hipSuccess &&
        cus > 0 && per > 0)
      b = cus * per;
    return b > kRedBlocks * 2 ? kRedBlocks * 2 : b;
  }();
  return blocks;
}

// the grid for vectors of n elements: at least 2048 elements per block (short
// vectors get fewer blocks and fewer partial sums to reduce), at most the
// resident wave above
int reduction_blocks(size_t n) {
  const size_t want = (n + 2047) / 2048;
  const int full = reduction_blocks();
  return want < size_t(full) ? int(want > 0 ? want : 1) : full;
}

// compile-time chunk counts 1..16
#define H6_COUNTS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_block_dots(const double2* Q, int m, const double2* w, size_t n, double* partials,
                             double* out, hipStream_t s, const int* skip) {
  // one grid size for all chunks (the partials of all 2m components are
  // reduced together)
  const int nb = reduction_blocks(n);
  for (int i0 = 0; i0 < m; i0 += kDotChunk) {
    const int cnt = m - i0 < kDotChunk ? m - i0 : kDotChunk;
    switch (cnt) {
#define H6_DOTS(C)                                                                                \
  case C:                                                                                         \
    hipLaunchKernelGGL(block_dots_kernel<C>, dim3(nb), dim3(kThreads), 0, s, Q, i0, w, n, partials, skip); \
    break;
      H6_COUNTS(H6_DOTS)
#undef H6_DOTS
      default: return hipErrorInvalidValue;
    }
  }
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(2 * m), dim3(kThreads), 0, s, partials, nb, out, skip,
                     static_cast<double*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_update_gram(double2* w, const double2* Q, const double2* c, int m, size_t n,
                              double* partials, double* out, hipStream_t s, const int* skip,
                              double* hnorm) {
  const int nb = reduction_blocks(n);
  const int mg = m < kGramChunk ? m : kGramChunk;
  if (mg < 1) return hipErrorInvalidValue;
  switch (mg) {
#define H6_UPD(C)                                                                                  \
  case C:                                                                                          \
    hipLaunchKernelGGL(update_gram_kernel<C>, dim3(nb), dim3(kThreads), 0, s, w, Q, c, m, n, partials, skip); \
    break;
    H6_COUNTS(H6_UPD)
#undef H6_UPD
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(1 + 2 * mg), dim3(kThreads), 0, s, partials, nb, out, skip,
                     hnorm);
  return hipGetLastError();
}

hipError_t launch_cheb_update(double2* e, const double2* t, double2* U, double c1, double c2, size_t n,
                              hipStream_t s) {
  hipLaunchKernelGGL(cheb_update_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, e, t, U, c1, c2, n);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(double2* out, const double2* V, const double2* y, int m, size_t n,
                             int accumulate, hipStream_t s, const int* mdev) {
  hipLaunchKernelGGL(multi_axpy_kernel<double2>, dim3(grid_for(n)), dim3(kThreads), 0, s, out, V, y, m,
                     n, accumulate, mdev);
  return hipGetLastError();
}

hipError_t launch_multi_axpy_f32(double2* out, const float2* V, const double2* y, int m, size_t n,
                                 int accumulate, hipStream_t s, const int* mdev) {
  hipLaunchKernelGGL(multi_axpy_kernel<float2>, dim3(grid_for(n)), dim3(kThreads), 0, s, out, V, y, m,
                     n, accumulate, mdev);
  return hipGetLastError();
}

size_t givens_bytes(int m) {
  // g (m + 1), sn (m), R (m * m) complex; cs, est (m) doubles; two ints
  return sizeof(double2) * (size_t(m + 1) + m + size_t(m) * m) + sizeof(double) * 2 * m + 2 * sizeof(int) + 64;
}

GivensState givens_state(h6_plan P, int m) {
  char* b = reinterpret_cast<char*>(P->d_givens);
  GivensState st;
  st.g = reinterpret_cast<double2*>(b);
  st.sn = st.g + (m + 1);
  st.R = st.sn + m;
  st.cs = reinterpret_cast<double*>(st.R + size_t(m) * m);
  st.est = st.cs + m;
  st.stop = reinterpret_cast<int*>(st.est + m);
  st.jdone = st.stop + 1;
  return st;
}

hipError_t launch_givens_step(int j, const double* nrow, const double* nu, const double2* hcol, GivensState st,
                              int m, const double* prm, hipStream_t s) {
  if (j < 0 || j >= m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(givens_step_kernel, dim3(1), dim3(64), 0, s, j, m, nrow, nu, hcol, st, prm);
  return hipGetLastError();
}

hipError_t launch_lsq_solve(int m, GivensState st, const double* nu, double2* y, hipStream_t s) {
  hipLaunchKernelGGL(lsq_solve_kernel, dim3(1), dim3(64), 0, s, m, st, nu, y);
  return hipGetLastError();
}

hipError_t launch_clear_int(int* p, hipStream_t s) {
  hipLaunchKernelGGL(clear_int_kernel, dim3(1), dim3(64), 0, s, p);
  return hipGetLastError();
}

}  // namespace h6
