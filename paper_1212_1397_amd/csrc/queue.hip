// Device side of the queued batch (helmholtz6_solve_batch_queue): many
// flexible GMRES(m) solves (Section 2, eq. (AAP)) of problems that share a
// grid shape run on a few lanes, each lane a plan of that shape whose
// wavenumber-dependent tables are reloaded from the next problem of a
// device-side work queue when its current problem is done.  One captured
// graph holds every lane; a replay advances each lane by one restart cycle.
//
// Per lane and replay, in stream order:
//   residual r = F - A U into the first basis slot, |r|^2       (plan kernels)
//   lane_check_kernel    convergence test of the lane's problem; when done,
//                        its result is recorded and the next problem is
//                        taken from the queue (atomic head, longest first)
//   lane_refill_kernel   U of the finished problem copied out; F, U = 0,
//                        r_0 = F and the problem's stencil weights, z-solver
//                        parameters and segment starts copied in; |F|^2
//   lane_cycle_kernel    |F| of a new problem, the cycle's step budget,
//                        ||F|| and tolerance for the device Givens steps,
//                        and the stop flag (set for an idle lane)
//   restart cycle        (plan kernels: preconditioner, A, MGS, Givens, U += Z y)
//   lane_count_kernel    steps done
#include "h6_internal.h"

namespace h6 {
namespace {

constexpr int kQThreads = 256;

__global__ __launch_bounds__(64) void lane_check_kernel(QueueLane* L, const QueueEntry* __restrict__ q,
                                                        int* head, int count, const double* __restrict__ rnorm2,
                                                        QueueResult* res) {
  if (threadIdx.x != 0) return;
  if (L->idle) {
    L->skip_refill = 1;
    L->skip_fresh = 1;
    return;
  }
  L->out = L->pend;          // a problem finished by lane_cycle_kernel last replay
  L->pend = -1;
  L->fresh = 0;
  if (L->cur >= 0) {
    const QueueEntry& e = q[L->cur];
    const double rel = sqrt(fmax(*rnorm2, 0.0)) / L->normF;
    const bool ok = rel <= e.tol;
    if (ok || L->iters >= e.maxit || !isfinite(rel)) {
      QueueResult& r = res[e.result];
      r.iters = L->iters;
      r.rel_resid = rel;
      r.status = ok ? int(H6_OK) : (isfinite(rel) ? int(H6_NOT_CONVERGED) : int(H6_DIVERGED));
      L->out = L->cur;
      L->cur = -1;
    }
  }
  if (L->cur < 0) {
    const int nxt = atomicAdd(head, 1);
    if (nxt < count) {
      L->cur = nxt;
      L->fresh = 1;
      L->iters = 0;
    } else {
      L->idle = 1;
      *L->idle_mirror = 1;     // host-visible: the lane has no more work
    }
  }
  L->skip_refill = (L->out >= 0 || L->fresh) ? 0 : 1;
  L->skip_fresh = L->fresh ? 0 : 1;
}

__global__ __launch_bounds__(kQThreads) void lane_refill_kernel(LaneRefill a, const int* __restrict__ skip) {
  if (*skip) return;
  const QueueLane& L = *a.lane;
  double2* __restrict__ uo = L.out >= 0 ? a.q[L.out].U : nullptr;
  const QueueEntry* e = L.fresh ? &a.q[L.cur] : nullptr;
  const double2* __restrict__ fi = e ? e->F : nullptr;
  const size_t stride = size_t(gridDim.x) * kQThreads;
  const size_t g = blockIdx.x * size_t(kQThreads) + threadIdx.x;
  double acc = 0.0;
  for (size_t i = g; i < a.N; i += stride) {
    const double2 u = a.U[i];
    if (uo) uo[i] = u;
    if (fi) {
      const double2 f = fi[i];
      a.F[i] = f;
      a.V0[i] = f;
      a.U[i] = make_double2(0.0, 0.0);
      acc = fma(f.x, f.x, fma(f.y, f.y, acc));
    }
  }
  if (e) {
    const uint2* __restrict__ cs = static_cast<const uint2*>(e->cstart);
    uint2* __restrict__ cd = static_cast<uint2*>(a.cstart);
    for (size_t i = g; i < a.cstart_words; i += stride) cd[i] = cs[i];
    constexpr size_t kSt = sizeof(StencilTable) / sizeof(double);
    if (g < kSt) reinterpret_cast<double*>(a.stencil)[g] = reinterpret_cast<const double*>(e->stencil)[g];
    if (g < size_t(kZParams)) a.zparams[g] = e->zparams[g];
  }
  // |F|^2 partial of this block (r_0 = F from U = 0)
  __shared__ double red[kQThreads / 64];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kQThreads / 64; ++w) t += red[w];
    a.partials[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(64) void lane_cycle_kernel(QueueLane* L, const QueueEntry* __restrict__ q,
                                                        QueueResult* res, const double* __restrict__ rnorm2,
                                                        double* prm, int* stop, int* jdone, int m) {
  if (threadIdx.x != 0) return;
  *jdone = 0;
  if (L->idle || L->cur < 0) {
    *stop = 1;
    return;
  }
  const QueueEntry& e = q[L->cur];
  if (L->fresh) {
    L->normF = sqrt(fmax(*rnorm2, 0.0));
    // F = 0 (U = 0 is the solution), or a tolerance that U = 0 already meets
    if (!(L->normF > 0.0) || e.tol >= 1.0) {
      QueueResult& r = res[e.result];
      r.iters = 0;
      r.rel_resid = L->normF > 0.0 ? 1.0 : 0.0;
      r.status = int(H6_OK);
      L->pend = L->cur;      // U = 0 is copied out by the next replay's refill
      L->cur = -1;
      *stop = 1;
      return;
    }
  }
  prm[0] = double(min(m, e.maxit - L->iters));
  prm[1] = L->normF;
  prm[2] = e.tol;
  *stop = prm[0] >= 1.0 ? 0 : 1;
}

__global__ __launch_bounds__(64) void lane_count_kernel(QueueLane* L, const int* __restrict__ jdone) {
  if (threadIdx.x != 0) return;
  if (!L->idle && L->cur >= 0) L->iters += *jdone;
}

}  // namespace

hipError_t launch_lane_check(QueueLane* lane, const QueueEntry* q, int* head, int count, const double* rnorm2,
                             QueueResult* res, hipStream_t s) {
  hipLaunchKernelGGL(lane_check_kernel, dim3(1), dim3(64), 0, s, lane, q, head, count, rnorm2, res);
  return hipGetLastError();
}

hipError_t launch_lane_refill(const LaneRefill& a, hipStream_t s) {
  hipLaunchKernelGGL(lane_refill_kernel, dim3(kRedBlocks), dim3(kQThreads), 0, s, a,
                     static_cast<const int*>(&a.lane->skip_refill));
  return hipGetLastError();
}

hipError_t launch_lane_cycle(QueueLane* lane, const QueueEntry* q, QueueResult* res, const double* rnorm2,
                             double* prm, int* stop, int* jdone, int m, hipStream_t s) {
  hipLaunchKernelGGL(lane_cycle_kernel, dim3(1), dim3(64), 0, s, lane, q, res, rnorm2, prm, stop, jdone, m);
  return hipGetLastError();
}

hipError_t launch_lane_count(QueueLane* lane, const int* jdone, hipStream_t s) {
  hipLaunchKernelGGL(lane_count_kernel, dim3(1), dim3(64), 0, s, lane, jdone);
  return hipGetLastError();
}

}  // namespace h6
