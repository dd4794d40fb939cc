// y = A x (or r = F - A x with partial |r|^2): the h^2-scaled sixth-order
// compact 27-point operator of eq. (scheme) with the Neumann (3DN) and
// Sommerfeld (3DDISCS) closure rows, complex128.
//
// Each row is sum_{d=-1,0,1} W[rowtype][d] . S_{l+d}, where S_p holds, for
// plane p, the centre value, the sum of the four edge neighbours and the sum
// of the four corner neighbours of a point (the in-plane parts of D_x + D_y
// and D_x D_y).  Neumann x/y faces enter through mirror ghosts, Dirichlet
// faces through zeros.
//
// Launch shape (2.5D march): a workgroup of 256 threads owns a 64 x 8 x-y tile
// and a chunk of up to kTZ z-planes (8, 16 or 32: the plan's autotuned depth).  It streams the planes of its chunk plus
// one halo plane on each side through a double-buffered LDS tile of 66 x 10
// complex values, computes S_p once per plane, and scatters it into the two
// running row accumulators.  Each plane is read from HBM once per tile
// (halo columns and the two halo planes are the only re-reads).  Workgroup
// ids are remapped so that consecutive tiles land on the same XCD (shared L2
// for halos).
#include "h6_internal.h"

namespace h6 {
namespace {

constexpr int kTX = 64, kTY = 8;      // x-y tile; the z chunk (8, 16 or 32 planes) is a template parameter
constexpr int kLX = kTX + 2, kLY = kTY + 2;
constexpr int kThreads = 256;
constexpr int kLoads = (kLX * kLY + kThreads - 1) / kThreads;   // 3

struct S3 {
  double2 c, e, k;
};

__device__ __forceinline__ void cmac(double2& acc, double2 w, double2 s) {
  acc.x = fma(w.x, s.x, acc.x);
  acc.x = fma(-w.y, s.y, acc.x);
  acc.y = fma(w.x, s.y, acc.y);
  acc.y = fma(w.y, s.x, acc.y);
}

__device__ __forceinline__ void apply_w(double2& acc, const W9& w, const S3& s) {
  cmac(acc, w.c, s.c);
  cmac(acc, w.e, s.e);
  cmac(acc, w.k, s.k);
}

__device__ __forceinline__ double2 add2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

template <bool RESID, typename Tin, typename Tout, int kTZ>
__global__ __launch_bounds__(kThreads) void stencil_kernel(
    const Tin* __restrict__ x, Tout* __restrict__ y, const double2* __restrict__ F,
    double* __restrict__ partials, double* __restrict__ fpartials, const StencilTable* __restrict__ W,
    int nx, int ny, int nz,
    int xmir, int ymir, int zlo_cl, int zhi_cl, int ntx, int nty, int nwg, const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double2 tile[2][kLY][kLX];
  __shared__ double red[kThreads / 64];

  const int L = xcd_remap(blockIdx.x, nwg);
  const int tx_i = L % ntx;
  const int ty_i = (L / ntx) % nty;
  const int tz_i = L / (ntx * nty);
  const int x0 = tx_i * kTX, y0 = ty_i * kTY, z0 = tz_i * kTZ;
  const int z1 = min(z0 + kTZ, nz);
  const int tid = threadIdx.x;
  const int tx = tid & 63, ty = tid >> 6;
  const size_t plane = size_t(nx) * ny;

  // element e of the (kLY x kLX) tile -> global (gx, gy) with ghost rules;
  // returns -1 for a zero value
  int src_off[kLoads];
#pragma unroll
  for (int i = 0; i < kLoads; ++i) {
    const int e = tid + i * kThreads;
    int off = -1;
    if (e < kLX * kLY) {
      const int r = e / kLX, c = e - r * kLX;
      int gx = x0 - 1 + c, gy = y0 - 1 + r;
      bool ok = true;
      if (gx < 0) { if (xmir) gx = 1; else ok = false; }
      else if (gx == nx) { if (xmir) gx = nx - 2; else ok = false; }
      else if (gx > nx) ok = false;
      if (gy < 0) { if (ymir) gy = 1; else ok = false; }
      else if (gy == ny) { if (ymir) gy = ny - 2; else ok = false; }
      else if (gy > ny) ok = false;
      if (ok) off = gx + nx * gy;
    }
    src_off[i] = off;
  }

  // A plane in flight: raw input values (converted to complex128 only when
  // written to LDS) and a mask of the valid ones.  The loads are unconditional
  // (invalid ones read element 0 of the plane and are masked at the LDS
  // write), so the code is straight-line and waiting for one plane's loads
  // does not wait for the loads issued after them.
  struct Plane {
    Tin v[kLoads];
    unsigned ok;
  };
  // planes outside [z0 - 1, z1] or outside the grid are masked; their loads
  // re-read the last plane of the chunk (already in cache)
  const int zlast = min(z1, nz - 1);
  auto load_plane = [&](int p, Plane& pl) {
    const bool okp = p >= 0 && p < nz && p <= z1;
    const Tin* xp = x + size_t(okp ? p : zlast) * plane;
    pl.ok = 0;
#pragma unroll
    for (int i = 0; i < kLoads; ++i) {
      pl.v[i] = xp[src_off[i] >= 0 ? src_off[i] : 0];
      if (okp && src_off[i] >= 0) pl.ok |= 1u << i;
    }
  };
  auto store_plane = [&](int b, const Plane& pl) {
#pragma unroll
    for (int i = 0; i < kLoads; ++i) {
      const int e = tid + i * kThreads;
      const bool ok = (pl.ok >> i) & 1u;
      if (e < kLX * kLY)
        (&tile[b][0][0])[e] = make_double2(ok ? double(pl.v[i].x) : 0.0, ok ? double(pl.v[i].y) : 0.0);
    }
  };

  auto row_type = [&](int l) { return (l == 0 && zlo_cl) ? 1 : ((l == nz - 1 && zhi_cl) ? 2 : 0); };

  double2 acc_a[2], acc_b[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) acc_a[s] = acc_b[s] = make_double2(0.0, 0.0);
  double nrm = 0.0, fnrm = 0.0;   // |r|^2 and (fpartials != nullptr) |F|^2 of this workgroup's rows

  // planes stream through two register sets (loads issued two planes ahead)
  // into the double-buffered LDS tile
  Plane va, vb;
  const int nplanes = z1 - z0 + 2;
  load_plane(z0 - 1, va);
  store_plane(0, va);
  load_plane(z0, vb);                     // plane of iteration 1 (nplanes >= 3)
  __syncthreads();

  auto step = [&](int it, Plane& cur, Plane& nxt) {
    // LDS buffer (it & 1) holds plane p; nxt holds plane p + 1; cur is free
    const int p = z0 - 1 + it;
    load_plane(p + 2, cur);   // unconditional (masked past the chunk): straight-line waits
    const int b = it & 1;
    // row types of the three rows this plane feeds (uniform across the block)
    const W9 w_prev = W->w[row_type(p - 1)][2];
    const W9 w_cur = W->w[row_type(p)][1];
    const W9 w_next = W->w[row_type(p + 1)][0];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int r = ty + 4 * s + 1, c = tx + 1;
      S3 S;
      S.c = tile[b][r][c];
      S.e = add2(add2(tile[b][r][c - 1], tile[b][r][c + 1]), add2(tile[b][r - 1][c], tile[b][r + 1][c]));
      S.k = add2(add2(tile[b][r - 1][c - 1], tile[b][r - 1][c + 1]),
                 add2(tile[b][r + 1][c - 1], tile[b][r + 1][c + 1]));
      // row p-1 receives its +1 plane and is complete
      if (p - 1 >= z0) {
        apply_w(acc_a[s], w_prev, S);
        const int gx = x0 + tx, gy = y0 + ty + 4 * s;
        if (gx < nx && gy < ny) {
          const size_t o = size_t(p - 1) * plane + gx + size_t(nx) * gy;
          double2 out = acc_a[s];
          if (RESID) {
            const double2 f = F[o];
            out = make_double2(f.x - out.x, f.y - out.y);
            nrm = fma(out.x, out.x, fma(out.y, out.y, nrm));
            fnrm = fma(f.x, f.x, fma(f.y, f.y, fnrm));
          }
          Tout yo;
          yo.x = out.x;           // complex64 output: rounded after the FP64 norm
          yo.y = out.y;
          y[o] = yo;
        }
      }
      acc_a[s] = acc_b[s];
      apply_w(acc_a[s], w_cur, S);
      acc_b[s] = make_double2(0.0, 0.0);
      apply_w(acc_b[s], w_next, S);
    }
    if (it + 1 < nplanes) store_plane(b ^ 1, nxt);
    __syncthreads();
  };
  for (int it = 0; it < nplanes; it += 2) {
    step(it, va, vb);
    if (it + 1 < nplanes) step(it + 1, vb, va);
  }

  if (RESID) {
    for (int o = 32; o > 0; o >>= 1) nrm += __shfl_down(nrm, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = nrm;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int i = 0; i < kThreads / 64; ++i) t += red[i];
      partials[blockIdx.x] = t;
    }
    if (fpartials) {
      for (int o = 32; o > 0; o >>= 1) fnrm += __shfl_down(fnrm, o, 64);
      __syncthreads();
      if ((tid & 63) == 0) red[tid >> 6] = fnrm;
      __syncthreads();
      if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < kThreads / 64; ++i) t += red[i];
        fpartials[blockIdx.x] = t;
      }
    }
  }
}

}  // namespace

template <typename Tin, typename Tout, int kTZ>
hipError_t stencil_launch(h6_plan P, const Tin* x, Tout* y, const double2* F, double* partials,
                          int* nparts, hipStream_t s, double* fpartials) {
  const int nx = P->dims[0], ny = P->dims[1], nz = P->dims[2];
  const int ntx = (nx + kTX - 1) / kTX, nty = (ny + kTY - 1) / kTY, ntz = (nz + kTZ - 1) / kTZ;
  const int nwg = ntx * nty * ntz;
  const bool resid = F != nullptr;
  if (resid && nwg > kMaxPartials) return hipErrorInvalidValue;
  hipEvent_t ev;
  timing_begin(P, resid ? KC_STENCIL_RESID : KC_STENCIL, s, &ev);
  if (resid)
    hipLaunchKernelGGL((stencil_kernel<true, Tin, Tout, kTZ>), dim3(nwg), dim3(kThreads), 0, s, x, y, F,
                       partials, fpartials, P->d_stencil, nx, ny, nz, P->xmirror, P->ymirror, P->zlo_closure,
                       P->zhi_closure, ntx, nty, nwg, P->skip);
  else
    hipLaunchKernelGGL((stencil_kernel<false, Tin, Tout, kTZ>), dim3(nwg), dim3(kThreads), 0, s, x, y,
                       nullptr, nullptr, nullptr, P->d_stencil, nx, ny, nz, P->xmirror, P->ymirror,
                       P->zlo_closure, P->zhi_closure, ntx, nty, nwg, P->skip);
  timing_end(P, resid ? KC_STENCIL_RESID : KC_STENCIL, s, ev,
             double(P->N) * (sizeof(Tin) + sizeof(Tout) + (resid ? sizeof(double2) : 0)));
  if (nparts) *nparts = nwg;
  return hipGetLastError();
}

// the plan's z-chunk depth (set by the autotuner; 16 by default)
template <typename Tin, typename Tout>
hipError_t stencil_impl(h6_plan P, const Tin* x, Tout* y, const double2* F, double* partials,
                        int* nparts, hipStream_t s, double* fpartials = nullptr) {
  if (P->stencil_tz == 8) return stencil_launch<Tin, Tout, 8>(P, x, y, F, partials, nparts, s, fpartials);
  if (P->stencil_tz == 32) return stencil_launch<Tin, Tout, 32>(P, x, y, F, partials, nparts, s, fpartials);
  return stencil_launch<Tin, Tout, 16>(P, x, y, F, partials, nparts, s, fpartials);
}

hipError_t launch_stencil(h6_plan P, const double2* x, double2* y, const double2* F,
                          double* partials, int* nparts, hipStream_t s, double* fpartials) {
  return stencil_impl(P, x, y, F, partials, nparts, s, fpartials);
}

hipError_t launch_stencil_f32in(h6_plan P, const float2* x, double2* y, hipStream_t s) {
  return stencil_impl(P, x, y, static_cast<const double2*>(nullptr), nullptr, nullptr, s);
}

int stencil_workgroups(h6_plan P) {
  const int tz = P->stencil_tz == 8 || P->stencil_tz == 32 ? P->stencil_tz : 16;
  return ((P->dims[0] + kTX - 1) / kTX) * ((P->dims[1] + kTY - 1) / kTY) * ((P->dims[2] + tz - 1) / tz);
}

hipError_t launch_resid_f32out(h6_plan P, const double2* U, float2* r, const double2* F,
                               double* partials, int* nparts, hipStream_t s, double* fpartials) {
  return stencil_impl(P, U, r, F, partials, nparts, s, fpartials);
}

}  // namespace h6
