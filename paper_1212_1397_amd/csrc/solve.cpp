// Host control loops of the solvers: right-preconditioned restarted GMRES(m)
// and flexible GMRES(m) (Section 2, eq. (AAP)), the SKS iteration (Section 2,
// Algorithm 1) in correction form, and Chebyshev acceleration (Section 2,
// Theorem 2) over the exact spectrum interval of eq. (3DEGV).
//
// Arnoldi: modified Gram-Schmidt in inverse compact WY form.  The basis is
// kept unnormalised on the device (q~_i = nu_i q_i), so no scaling pass is
// needed.  Step j:
//   z~ = A_p^{-1} q~_j,  w~ = A z~                      (w = w~ / nu_j)
//   one pass:  s~_i = <q~_i, w~>,  i <= j
//   device:    nu_j, row j of the Gram matrix G_{i,l} = <q_i, q_l>, and
//              h_i = s~_i / (nu_i nu_j) - sum_{l<i} G_{i,l} h_l   (the MGS
//              coefficients; one small kernel, no host round trip)
//   one pass:  w~ -= sum_i (nu_j h_i / nu_i) q~_i; |w~|^2 and the Gram row
//              <q~_i, w~> of the next basis vector
//   H(0..j, j) = h,  H(j+1, j) = nu_{j+1} / nu_j,
// followed by the complex Givens update of the least-squares problem on the
// host (FP64).  The host waits once per step, for h and |w~|^2; the first
// preconditioner pass of the next step is enqueued before that wait, so the
// device stays busy while the host decides whether to go on.  The cycle's
// stopping test uses the least-squares residual; convergence is declared on
// the true residual ||F - A U|| / ||F||, recomputed at every restart.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "h6_internal.h"

namespace h6 {
namespace {

// device scalar layout (in doubles from P->d_scal) and pinned host mirror
constexpr int kDots = 0;        // 2 (m + 1) doubles of block dot results
constexpr int kNorm = 1100;     // one norm (update pass: norm + 2 kGramMax Gram entries)
constexpr int kCoef = 1200;     // 2 (m + 1) doubles: update coefficients (double2)
constexpr int kY = 2000;        // 2 m doubles: least-squares coefficients (double2)
constexpr int kGram2 = 3000;    // Gram entries beyond kGramMax (2 m doubles)
constexpr int kNu = 3600;       // m + 1 doubles: basis norms nu_i
constexpr int kHcol = 4000;     // 2 (m + 1) doubles: Hessenberg column of the current step
constexpr int kJudge = 4600;    // 2 doubles: |q - A z|^2 without / with the learned correction
constexpr int kCycEst = 5000;   // whole-cycle graphs: m doubles of per-step residual estimates (host)
constexpr int kCycInt = 5300;   // steps done (an int in one double slot, host)
constexpr int kPrm = 5400;      // (steps allowed, ||F||, tol) for the device Givens steps
// host-mapped step mirror (P->h_step): the Hessenberg column (2 (m + 1) doubles
// from 0) and |w~|^2 (at kStepNorm), written by the step's own kernels
constexpr int kStepNorm = 2 * 258;
constexpr int kStepMirror = kStepNorm + 8;

struct Ctx {
  h6_plan P;
  hipStream_t s;
  size_t N;
  double* dev;      // P->d_scal as doubles
  double* host;     // P->h_pinned as doubles
};

h6_status ensure(h6_plan P, int method, int m) {
  const size_t vb = P->N * sizeof(double2);
  const size_t zb = P->N * (P->p.precision == H6_MIXED ? sizeof(float2) : sizeof(double2));
  auto grow = [&](void** ptr, int* cols, int want, size_t bytes) -> hipError_t {
    if (*cols >= want) return hipSuccess;
    (void)hipFree(*ptr);
    *ptr = nullptr;
    *cols = 0;
    hipError_t e = hipMalloc(ptr, bytes * size_t(want));
    if (e == hipSuccess) *cols = want;
    return e;
  };
  hipError_t e = hipSuccess;
  if (!P->ev_sync) e = hipEventCreateWithFlags(&P->ev_sync, hipEventDisableTiming);
  if (e == hipSuccess && !P->r) e = hipMalloc(reinterpret_cast<void**>(&P->r), vb);
  if (e == hipSuccess && !P->t) e = hipMalloc(reinterpret_cast<void**>(&P->t), vb);
  if (e == hipSuccess && method == H6_CHEBYSHEV)
    e = grow(reinterpret_cast<void**>(&P->V), &P->V_cols, 1, vb);     // the direction e
  if (e == hipSuccess && method != H6_SKS && method != H6_CHEBYSHEV) {
    e = grow(reinterpret_cast<void**>(&P->V), &P->V_cols, m + 1, vb);
    if (e == hipSuccess && P->gram_dim < m + 1) {
      (void)hipFree(P->d_gram);
      P->d_gram = nullptr;
      P->gram_dim = 0;
      e = hipMalloc(reinterpret_cast<void**>(&P->d_gram), sizeof(double2) * size_t(m + 1) * (m + 1));
      if (e == hipSuccess) P->gram_dim = m + 1;
    }
  }
  if (e == hipSuccess && method == H6_FGMRES) e = grow(&P->Z, &P->Z_cols, m, zb);
  if (e == hipSuccess && (method == H6_GMRES || method == H6_FGMRES) && !P->h_step) {
    e = hipHostMalloc(reinterpret_cast<void**>(&P->h_step), sizeof(double) * kStepMirror,
                      hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&P->d_step), P->h_step, 0);
  }
  if (e == hipSuccess && method == H6_SKS && P->parts_cap < stencil_workgroups(P)) {
    if (P->h_parts) (void)hipHostFree(P->h_parts);
    P->h_parts = P->d_parts = nullptr;
    P->parts_cap = 0;
    const int n = stencil_workgroups(P);
    e = hipHostMalloc(reinterpret_cast<void**>(&P->h_parts), 2 * sizeof(double) * size_t(n),
                      hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&P->d_parts), P->h_parts, 0);
    if (e == hipSuccess) P->parts_cap = n;
  }
  if (e == hipSuccess && P->use_graphs == 2 && (method == H6_GMRES || method == H6_FGMRES) &&
      P->givens_dim < m) {
    (void)hipFree(P->d_givens);
    P->d_givens = nullptr;
    P->givens_dim = 0;
    e = hipMalloc(reinterpret_cast<void**>(&P->d_givens), givens_bytes(m));
    if (e == hipSuccess) P->givens_dim = m;
  }
  if (e != hipSuccess) {
    P->last_error = std::string("workspace allocation failed: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? H6_ERR_ALLOC : H6_ERR_HIP;
  }
  return H6_OK;
}

// copy `count` doubles at `off` back to the pinned mirror; wait() blocks until
// they (and only the work enqueued before them) are done
h6_status fetch_async(Ctx& c, int off, int count) {
  h6_plan P = c.P;
  H6_TRY_HIP(hipMemcpyAsync(c.host + off, c.dev + off, sizeof(double) * count, hipMemcpyDeviceToHost, c.s));
  H6_TRY_HIP(hipEventRecord(P->ev_sync, c.s));
  return H6_OK;
}
h6_status wait(Ctx& c) {
  h6_plan P = c.P;
  H6_TRY_HIP(hipEventSynchronize(P->ev_sync));
  return H6_OK;
}
h6_status fetch(Ctx& c, int off, int count) {
  h6_status st = fetch_async(c, off, count);
  return st == H6_OK ? wait(c) : st;
}

// |v|^2 on the host (synchronises)
h6_status norm2(Ctx& c, const double2* v, double* out) {
  h6_plan P = c.P;
  hipEvent_t ev;
  timing_begin(P, KC_NORM, c.s, &ev);
  H6_TRY_HIP(launch_norm2(v, c.N, P->partials, c.dev + kNorm, c.s));
  timing_end(P, KC_NORM, c.s, ev, double(c.N) * sizeof(double2));
  h6_status st = fetch(c, kNorm, 1);
  *out = c.host[kNorm];
  return st;
}

// r = F - A U with |r|^2 into the device slot kNorm and on its way to the host
// (fetch_async: call wait() before reading c.host[kNorm])
h6_status residual_async(Ctx& c, const double2* F, const double2* U, double2* r) {
  h6_plan P = c.P;
  int nparts = 0;
  H6_TRY_HIP(launch_stencil(P, U, r, F, P->partials, &nparts, c.s));
  H6_TRY_HIP(launch_reduce_sum(P->partials, nparts, c.dev + kNorm, c.s));
  return fetch_async(c, kNorm, 1);
}

void record(h6_solve_info* info, int& nh, double v) {
  if (info->history && nh < info->history_len) info->history[nh++] = v;
}

// Complex Givens rotation (c real, s complex) with [c s; -conj(s) c] [a; b] = [r; 0], b real >= 0.
void givens(cplx a, double b, double& c, cplx& s, cplx& r) {
  if (b == 0.0) { c = 1.0; s = 0.0; r = a; return; }
  if (std::abs(a) == 0.0) { c = 0.0; s = 1.0; r = b; return; }
  const double t = std::hypot(std::abs(a), b);
  const cplx ph = a / std::abs(a);
  c = std::abs(a) / t;
  s = ph * b / t;
  r = ph * t;
}

h6_status upload_coefs(Ctx& c, int off, const std::vector<cplx>& v, int count) {
  h6_plan P = c.P;
  for (int i = 0; i < count; ++i) {
    c.host[off + 2 * i] = v[i].real();
    c.host[off + 2 * i + 1] = v[i].imag();
  }
  H6_TRY_HIP(hipMemcpyAsync(c.dev + off, c.host + off, sizeof(double) * 2 * count, hipMemcpyHostToDevice, c.s));
  return H6_OK;
}

// The kernels of one restart cycle of GMRES(m) / FGMRES(m) on c.s, with the
// Givens rotations on the device: steps j = 0..m-1 (preconditioner, A, MGS,
// Givens update), each returning at once while gs.stop is set, then
// y = R^{-1} g over the steps done and U += Z y (U += A_p^{-1} V y).  The
// cycle starts from the unnormalised residual in the first basis slot and
// |r|^2 in the kNorm slot, and reads (steps allowed, ||F||, tol) from kPrm.
hipError_t enqueue_cycle(Ctx& c, double2* U, int m, bool flex, bool mixed, const GivensState& gs) {
  h6_plan P = c.P;
  const size_t N = c.N;
  double* prm = c.dev + kPrm;
  hipError_t e = hipSuccess;
  P->skip = gs.stop;
  const double2* dcoef = reinterpret_cast<const double2*>(c.dev + kCoef);
  double2* dhcol = reinterpret_cast<double2*>(c.dev + kHcol);
  for (int j = 0; j < m && e == hipSuccess; ++j) {
    const double2* qj = P->V + size_t(j) * N;
    double2* w = P->V + size_t(j + 1) * N;
    if (mixed) {
      float2* z = static_cast<float2*>(P->Z) + size_t(j) * N;
      e = launch_pinv_f32out(P, qj, z, c.s, PINV_ALL);
      if (e == hipSuccess) e = launch_stencil_f32in(P, z, w, c.s);
    } else {
      double2* z = flex ? static_cast<double2*>(P->Z) + size_t(j) * N : P->t;
      e = launch_pinv(P, qj, z, c.s, PINV_ALL);
      if (e == hipSuccess) e = launch_stencil(P, z, w, nullptr, nullptr, nullptr, c.s);
    }
    if (e == hipSuccess) e = launch_block_dots(P->V, j + 1, w, N, P->partials, c.dev + kDots, c.s, gs.stop);
    if (e == hipSuccess && j > kGramMax)
      e = launch_block_dots(P->V + size_t(kGramMax) * N, j - kGramMax, qj, N, P->partials, c.dev + kGram2,
                            c.s, gs.stop);
    if (e == hipSuccess)
      e = launch_mgs_coef(j, c.dev + kDots, c.dev + kNorm, c.dev + kGram2, c.dev + kNu, P->d_gram, P->gram_dim,
                          dhcol, reinterpret_cast<double2*>(c.dev + kCoef), c.s, gs.stop);
    if (e == hipSuccess) e = launch_update_gram(w, P->V, dcoef, j + 1, N, P->partials, c.dev + kNorm, c.s, gs.stop);
    if (e == hipSuccess) e = launch_givens_step(j, c.dev + kNorm, c.dev + kNu, dhcol, gs, m, prm, c.s);
  }
  P->skip = nullptr;
  double2* dy = reinterpret_cast<double2*>(c.dev + kY);
  if (e == hipSuccess) e = launch_lsq_solve(m, gs, c.dev + kNu, dy, c.s);
  if (e == hipSuccess) {
    if (flex && mixed)
      e = launch_multi_axpy_f32(U, static_cast<float2*>(P->Z), dy, m, N, 1, c.s, gs.jdone);
    else if (flex)
      e = launch_multi_axpy(U, static_cast<double2*>(P->Z), dy, m, N, 1, c.s, gs.jdone);
    else {
      e = launch_multi_axpy(P->t, P->V, dy, m, N, 0, c.s, gs.jdone);
      if (e == hipSuccess) e = launch_pinv_acc(P, P->t, U, c.s);
    }
  }
  return e;
}

// GMRES / FGMRES with whole restart cycles as one captured HIP graph: every
// step's kernels (preconditioner, A, MGS) are followed by a one-thread
// Givens update of the least-squares problem on the device; when it meets
// the tolerance, the step budget or a breakdown it raises a device stop flag,
// and the kernels of the later steps return at once (no conditional nodes
// are needed).  The cycle ends with y = R^{-1} g and U += Z y (or
// U += A_p^{-1} V y) on the device, so the host waits once per cycle, for the
// true residual, the steps done and their estimates.
h6_status gmres_cycles(Ctx& c, const double2* F, double2* U, h6_solve_info* info, double normF) {
  h6_plan P = c.P;
  const int m = info->restart;
  const bool flex = info->method == H6_FGMRES;
  const bool mixed = P->p.precision == H6_MIXED;
  const size_t N = c.N;
  const GivensState gs = givens_state(P, m);
  double* prm = c.dev + kPrm;
  const GraphKey key{P->V, P->Z, U, m, int(flex), int(mixed), 2};
  if (!(key == P->graph_key)) {
    release_graphs(P);
    P->graph_key = key;
  }
  if (!P->cycle_graph) {
    hipGraph_t graph = nullptr;
    H6_TRY_HIP(hipStreamBeginCapture(c.s, hipStreamCaptureModeRelaxed));
    hipError_t e = enqueue_cycle(c, U, m, flex, mixed, gs);
    const hipError_t e2 = hipStreamEndCapture(c.s, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&P->cycle_graph, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    H6_TRY_HIP(e);
  }
  int nh = 0;
  h6_status st = residual_async(c, F, U, P->V);
  if (st == H6_OK) st = wait(c);
  if (st != H6_OK) return st;
  double beta2 = c.host[kNorm];
  info->iters = 0;
  while (true) {
    info->rel_resid = std::sqrt(beta2) / normF;
    if (!std::isfinite(info->rel_resid)) { info->history_len = nh; return H6_DIVERGED; }
    if (info->rel_resid <= info->tol) { info->history_len = nh; return H6_OK; }
    if (info->iters >= info->maxit) { info->history_len = nh; return H6_NOT_CONVERGED; }
    // cycle parameters and a cleared stop flag, outside the graph
    c.host[kPrm] = double(std::min(m, info->maxit - info->iters));
    c.host[kPrm + 1] = normF;
    c.host[kPrm + 2] = info->tol;
    H6_TRY_HIP(hipMemcpyAsync(prm, c.host + kPrm, 3 * sizeof(double), hipMemcpyHostToDevice, c.s));
    H6_TRY_HIP(launch_clear_int(gs.stop, c.s));
    H6_TRY_HIP(hipGraphLaunch(P->cycle_graph, c.s));
    H6_TRY_HIP(hipMemcpyAsync(c.host + kCycEst, gs.est, sizeof(double) * m, hipMemcpyDeviceToHost, c.s));
    H6_TRY_HIP(hipMemcpyAsync(c.host + kCycInt, gs.jdone, sizeof(int), hipMemcpyDeviceToHost, c.s));
    st = residual_async(c, F, U, P->V);
    if (st == H6_OK) st = wait(c);
    if (st != H6_OK) return st;
    int jd = 0;
    std::memcpy(&jd, c.host + kCycInt, sizeof(int));
    if (jd < 1 || jd > m) {
      P->last_error = "internal: whole-cycle graph reported " + std::to_string(jd) + " steps";
      return H6_ERR_HIP;
    }
    for (int j = 0; j < jd; ++j) record(info, nh, c.host[kCycEst + j]);
    info->iters += jd;
    beta2 = c.host[kNorm];
  }
}

h6_status gmres(Ctx& c, const double2* F, double2* U, h6_solve_info* info, double normF) {
  h6_plan P = c.P;
  const int m = info->restart;
  const bool flex = info->method == H6_FGMRES;
  const bool mixed = P->p.precision == H6_MIXED;   // implies flex (checked at the ABI)
  const size_t N = c.N;
  int nh = 0;
  // the residual goes straight into the first basis slot (unnormalised)
  h6_status st = residual_async(c, F, U, P->V);
  if (st == H6_OK) st = wait(c);
  if (st != H6_OK) return st;
  double beta2 = c.host[kNorm];
  std::vector<cplx> H(size_t(m + 1) * m), g(m + 1), sn(m);
  std::vector<double> cs(m), nu(m + 1);
  auto Hij = [&](int i, int j) -> cplx& { return H[size_t(i) * m + j]; };
  const double2* dcoef = reinterpret_cast<const double2*>(c.dev + kCoef);
  double2* dhcol = reinterpret_cast<double2*>(c.dev + kHcol);
  const double kh = P->k.real() * P->p.h;      // feature of the learned correction
  P->learned_steps = 0;
  // step graphs: valid while the workspace and the step shape are unchanged
  const bool graphs = P->use_graphs && !P->timing.enabled && !P->net;
  if (graphs && P->use_graphs == 2) return gmres_cycles(c, F, U, info, normF);
  if (graphs) {
    const GraphKey key{P->V, P->Z, nullptr, m, int(flex), int(mixed), 1};
    if (!(key == P->graph_key) || int(P->step_graphs.size()) < m) {
      release_graphs(P);
      P->graph_key = key;
      P->step_graphs.assign(m, nullptr);
    }
  }
  // preconditioner passes of step j (z_j = A_p^{-1} q~_j)
  auto pinv = [&](int j, int part) -> hipError_t {
    const double2* qj = P->V + size_t(j) * N;
    if (mixed) return launch_pinv_f32out(P, qj, static_cast<float2*>(P->Z) + size_t(j) * N, c.s, part);
    double2* z = flex ? static_cast<double2*>(P->Z) + size_t(j) * N : P->t;
    return launch_pinv(P, qj, z, c.s, part);
  };
  info->iters = 0;
  while (true) {
    const double beta = std::sqrt(beta2);
    info->rel_resid = beta / normF;
    if (!std::isfinite(info->rel_resid)) { info->history_len = nh; return H6_DIVERGED; }
    if (info->rel_resid <= info->tol) { info->history_len = nh; return H6_OK; }
    if (info->iters >= info->maxit) { info->history_len = nh; return H6_NOT_CONVERGED; }
    nu[0] = beta;
    std::fill(g.begin(), g.end(), cplx(0.0));
    g[0] = beta;
    int jdone = 0;
    bool first_done = false;          // first preconditioner pass of step j already enqueued
    bool use_net = false;             // this cycle applies the learned correction
    for (int j = 0; j < m; ++j) {
      double2* w = P->V + size_t(j + 1) * N;
      const double2* qj = P->V + size_t(j) * N;
      void* zj = flex ? (mixed ? static_cast<void*>(static_cast<float2*>(P->Z) + size_t(j) * N)
                               : static_cast<void*>(static_cast<double2*>(P->Z) + size_t(j) * N))
                      : static_cast<void*>(P->t);
      auto apply_A_z = [&](const void* z, double2* out) -> hipError_t {
        if (mixed) return launch_stencil_f32in(P, static_cast<const float2*>(z), out, c.s);
        return launch_stencil(P, static_cast<const double2*>(z), out, nullptr, nullptr, nullptr, c.s);
      };
      // the device part of the step after z_j = A_p^{-1} q_j and w = A z_j:
      // inner products, MGS coefficients, update with the Gram row; the
      // coefficient and update kernels also write h and |w~|^2 into the
      // host-mapped step mirror (no copies)
      auto orthogonalise = [&]() -> hipError_t {
        hipError_t e;
        hipEvent_t ev;
        timing_begin(P, KC_MGS_DOTS, c.s, &ev);
        if ((e = launch_block_dots(P->V, j + 1, w, N, P->partials, c.dev + kDots, c.s)) != hipSuccess) return e;
        // Gram entries of q_j beyond the kGramMax formed by the last update pass
        if (j > kGramMax &&
            (e = launch_block_dots(P->V + size_t(kGramMax) * N, j - kGramMax, P->V + size_t(j) * N, N,
                                   P->partials, c.dev + kGram2, c.s)) != hipSuccess)
          return e;
        timing_end(P, KC_MGS_DOTS, c.s, ev,
                   double(N) * sizeof(double2) * ((j + 2) + (j > kGramMax ? j - kGramMax + 1 : 0)));
        if ((e = launch_mgs_coef(j, c.dev + kDots, c.dev + kNorm, c.dev + kGram2, c.dev + kNu, P->d_gram,
                                 P->gram_dim, dhcol, reinterpret_cast<double2*>(c.dev + kCoef), c.s, nullptr,
                                 reinterpret_cast<double2*>(P->d_step))) != hipSuccess)
          return e;
        timing_begin(P, KC_MGS_UPDATE, c.s, &ev);
        if ((e = launch_update_gram(w, P->V, dcoef, j + 1, N, P->partials, c.dev + kNorm, c.s, nullptr,
                                    P->d_step + kStepNorm)) != hipSuccess)
          return e;
        timing_end(P, KC_MGS_UPDATE, c.s, ev, double(N) * sizeof(double2) * (j + 3));
        return hipSuccess;
      };
      if (graphs) {
        // the whole step is one captured graph per step index, replayed
        hipGraphExec_t& g = P->step_graphs[j];
        if (!g) {
          hipGraph_t graph = nullptr;
          H6_TRY_HIP(hipStreamBeginCapture(c.s, hipStreamCaptureModeRelaxed));
          hipError_t e = pinv(j, PINV_ALL);
          if (e == hipSuccess) e = apply_A_z(zj, w);
          if (e == hipSuccess) e = orthogonalise();
          const hipError_t e2 = hipStreamEndCapture(c.s, &graph);
          if (e == hipSuccess) e = e2;
          if (e == hipSuccess) e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
          if (graph) (void)hipGraphDestroy(graph);
          H6_TRY_HIP(e);
        }
        H6_TRY_HIP(hipGraphLaunch(g, c.s));
        H6_TRY_HIP(hipEventRecord(P->ev_sync, c.s));
        info->iters += 1;
      } else {
        H6_TRY_HIP(pinv(j, first_done ? PINV_REST : PINV_ALL));
        if (j == 0 && flex && P->net) {
          // acceptance test of the correction for this cycle: ||q - A z|| with and without it
          const size_t zb = N * (mixed ? sizeof(float2) : sizeof(double2));
          H6_TRY_HIP(apply_A_z(zj, w));
          H6_TRY_HIP(launch_diff_norm2(qj, w, N, P->partials, c.dev + kJudge, c.s));
          H6_TRY_HIP(hipMemcpyAsync(P->t, zj, zb, hipMemcpyDeviceToDevice, c.s));
          H6_TRY_HIP(net_apply_add(P->net, qj, kh, P->t, mixed, c.s));
          H6_TRY_HIP(apply_A_z(P->t, P->r));
          H6_TRY_HIP(launch_diff_norm2(qj, P->r, N, P->partials, c.dev + kJudge + 1, c.s));
          st = fetch(c, kJudge, 2);
          if (st != H6_OK) return st;
          use_net = c.host[kJudge + 1] <= c.host[kJudge];
          if (use_net) {
            H6_TRY_HIP(hipMemcpyAsync(zj, P->t, zb, hipMemcpyDeviceToDevice, c.s));
            H6_TRY_HIP(hipMemcpyAsync(w, P->r, N * sizeof(double2), hipMemcpyDeviceToDevice, c.s));
          }
        } else {
          if (use_net) H6_TRY_HIP(net_apply_add(P->net, qj, kh, zj, mixed, c.s));
          H6_TRY_HIP(apply_A_z(zj, w));
        }
        if (use_net) P->learned_steps += 1;
        info->iters += 1;
        H6_TRY_HIP(orthogonalise());
        H6_TRY_HIP(hipEventRecord(P->ev_sync, c.s));
        // meanwhile the device starts on step j + 1
        first_done = j + 1 < m && info->iters < info->maxit;
        if (first_done) H6_TRY_HIP(pinv(j + 1, PINV_FIRST));
      }
      st = wait(c);
      if (st != H6_OK) return st;
      nu[j + 1] = std::sqrt(std::max(P->h_step[kStepNorm], 0.0));
      for (int i = 0; i <= j; ++i) Hij(i, j) = cplx(P->h_step[2 * i], P->h_step[2 * i + 1]);
      const double hn = nu[j + 1] / nu[j];
      // previous rotations on column j
      for (int i = 0; i < j; ++i) {
        const cplx t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
        Hij(i + 1, j) = -std::conj(sn[i]) * Hij(i, j) + cs[i] * Hij(i + 1, j);
        Hij(i, j) = t;
      }
      double cr;
      cplx sr, rr;
      givens(Hij(j, j), hn, cr, sr, rr);
      cs[j] = cr;
      sn[j] = sr;
      Hij(j, j) = rr;
      g[j + 1] = -std::conj(sr) * g[j];
      g[j] = cr * g[j];
      jdone = j + 1;
      const double est = std::abs(g[j + 1]) / normF;
      record(info, nh, est);
      const bool breakdown = !(hn > 1e-300);
      if (est <= info->tol || info->iters >= info->maxit || breakdown || !std::isfinite(est)) break;
    }
    // y = R^{-1} g; the update uses the unnormalised vectors, so y_i / nu_i
    std::vector<cplx> y(jdone);
    for (int i = jdone - 1; i >= 0; --i) {
      cplx acc = g[i];
      for (int k = i + 1; k < jdone; ++k) acc -= Hij(i, k) * y[k];
      y[i] = acc / Hij(i, i);
    }
    for (int i = 0; i < jdone; ++i) y[i] /= nu[i];
    st = upload_coefs(c, kY, y, jdone);
    if (st != H6_OK) return st;
    const double2* dy = reinterpret_cast<const double2*>(c.dev + kY);
    hipEvent_t ev;
    if (flex) {
      timing_begin(P, KC_AXPY, c.s, &ev);
      if (mixed)
        H6_TRY_HIP(launch_multi_axpy_f32(U, static_cast<float2*>(P->Z), dy, jdone, N, 1, c.s));
      else
        H6_TRY_HIP(launch_multi_axpy(U, static_cast<double2*>(P->Z), dy, jdone, N, 1, c.s));
      timing_end(P, KC_AXPY, c.s, ev,
                 double(N) * (jdone * (mixed ? sizeof(float2) : sizeof(double2)) + 2 * sizeof(double2)));
    } else {
      timing_begin(P, KC_AXPY, c.s, &ev);
      H6_TRY_HIP(launch_multi_axpy(P->t, P->V, dy, jdone, N, 0, c.s));
      timing_end(P, KC_AXPY, c.s, ev, double(N) * sizeof(double2) * (jdone + 1));
      H6_TRY_HIP(launch_pinv_acc(P, P->t, U, c.s));
    }
    st = residual_async(c, F, U, P->V);
    if (st == H6_OK) st = wait(c);
    if (st != H6_OK) return st;
    beta2 = c.host[kNorm];
  }
}

// F = 0: the solution is U = 0 (whatever the initial guess)
h6_status zero_solution(Ctx& c, double2* U, h6_solve_info* info) {
  h6_plan P = c.P;
  H6_TRY_HIP(hipMemsetAsync(U, 0, c.N * sizeof(double2), c.s));
  H6_TRY_HIP(hipStreamSynchronize(c.s));
  info->iters = 0;
  info->rel_resid = 0.0;
  info->history_len = 0;
  return H6_OK;
}

// SKS, Algorithm 1, in correction form: U += A_p^{-1} r (the update is made
// by the last inverse transform pass), r = F - A U.  The first
// preconditioner pass of r is enqueued before the host waits for |r|, so the
// device stays busy during the convergence test.  In mixed plans r is stored
// in complex64 by the residual kernel (its norm is taken in FP64 first): the
// preconditioner's first pass would round it to complex64 on load anyway.
// The residual kernel writes its per-workgroup partial sums of |r|^2 straight
// into coherent pinned host memory, and the host adds them in workgroup
// order after the wait: no reduction kernel and no copy per iteration.  The
// first residual pass also sums |F|^2 (it reads F anyway), which replaces
// the separate norm pass of the other solvers.
h6_status sks(Ctx& c, const double2* F, double2* U, h6_solve_info* info, bool zero_guess) {
  h6_plan P = c.P;
  const bool mixed = P->p.precision == H6_MIXED;
  float2* r32 = reinterpret_cast<float2*>(P->r);
  int nparts = 0;
  if (!P->d_parts || stencil_workgroups(P) > P->parts_cap) {
    P->last_error = "internal: residual partials exceed their host array";
    return H6_ERR_HIP;
  }
  double* d_fparts = P->d_parts + P->parts_cap;
  auto resid = [&](bool with_f) -> h6_status {
    double* fp = with_f ? d_fparts : nullptr;
    if (mixed)
      H6_TRY_HIP(launch_resid_f32out(P, U, r32, F, P->d_parts, &nparts, c.s, fp));
    else
      H6_TRY_HIP(launch_stencil(P, U, P->r, F, P->d_parts, &nparts, c.s, fp));
    H6_TRY_HIP(hipEventRecord(P->ev_sync, c.s));
    return H6_OK;
  };
  auto host_sum = [&](const double* a) {
    double t = 0.0;
    for (int i = 0; i < nparts; ++i) t += a[i];
    return t;
  };
  auto pinv = [&](int part) -> hipError_t {
    return mixed ? launch_pinv_acc_f32in(P, r32, U, c.s, part) : launch_pinv_acc(P, P->r, U, c.s, part);
  };
  int nh = 0;
  info->iters = 0;
  double normF = -1.0;
  h6_status st = H6_OK;
  if (zero_guess) {
    // from U_0 = 0: r_0 = F, so the first step is U_1 = A_p^{-1} F, written
    // over U, then r_1; |F| comes from a norm pass enqueued behind them
    H6_TRY_HIP(launch_pinv(P, F, U, c.s, PINV_ALL));
    st = resid(false);
    if (st != H6_OK) return st;
    double normF2 = 0.0;
    st = norm2(c, F, &normF2);
    if (st != H6_OK) return st;
    normF = std::sqrt(normF2);
    if (normF == 0.0) return zero_solution(c, U, info);
    if (info->tol >= 1.0) {                     // U_0 = 0 already meets the tolerance
      st = zero_solution(c, U, info);
      info->rel_resid = 1.0;
      return st;
    }
    info->iters = 1;
  } else {
    st = resid(true);
  }
  if (st != H6_OK) return st;
  // The first pass of the next preconditioner application is enqueued before
  // the host waits for |r| (speculatively), except when the residual trend
  // (geometric: the last ratio of successive residuals) predicts that this
  // residual meets the tolerance.  Every return waits for the stream, so no
  // speculative pass is left running.
  double prev = -1.0, predicted = -1.0;
  auto finish = [&](h6_status s) -> h6_status {
    info->history_len = nh;
    if (hipStreamSynchronize(c.s) != hipSuccess) {
      P->last_error = "hipStreamSynchronize failed at the end of the SKS solve";
      return H6_ERR_HIP;
    }
    return s;
  };
  while (true) {
    const bool more = info->iters < info->maxit;
    const bool spec = more && !(predicted >= 0.0 && predicted <= info->tol);
    if (spec) H6_TRY_HIP(pinv(PINV_FIRST));
    st = wait(c);
    if (st != H6_OK) return st;
    if (normF < 0.0) {
      normF = std::sqrt(host_sum(P->h_parts + P->parts_cap));
      if (normF == 0.0) return zero_solution(c, U, info);
    }
    info->rel_resid = std::sqrt(host_sum(P->h_parts)) / normF;
    if (info->iters > 0) record(info, nh, info->rel_resid);
    if (info->rel_resid <= info->tol) return finish(H6_OK);
    if (!std::isfinite(info->rel_resid) || (info->iters > 0 && info->rel_resid > 1e4))
      return finish(H6_DIVERGED);
    if (!more) return finish(H6_NOT_CONVERGED);
    predicted = prev > 0.0 ? info->rel_resid * (info->rel_resid / prev) : -1.0;
    prev = info->rel_resid;
    if (!spec) H6_TRY_HIP(pinv(PINV_FIRST));
    H6_TRY_HIP(pinv(PINV_REST));
    st = resid(false);
    if (st != H6_OK) return st;
    info->iters += 1;
  }
}

// Chebyshev acceleration on A A_p^{-1} Y = F over the spectrum interval
// [alpha, beta] (theta = centre, delta = half width, sigma = theta / delta),
// written for U = A_p^{-1} Y with the direction e = A_p^{-1} d:
//   e_0 = A_p^{-1} r_0 / theta,  U_{k+1} = U_k + e_k,  r_{k+1} = F - A U_{k+1},
//   rho_{k+1} = 1 / (2 sigma - rho_k),  e_{k+1} = rho_{k+1} rho_k e_k + (2 rho_{k+1} / delta) A_p^{-1} r_{k+1}.
h6_status chebyshev(Ctx& c, const double2* F, double2* U, h6_solve_info* info, double normF) {
  h6_plan P = c.P;
  h6_status st = spectrum_bounds(P);
  if (st != H6_OK) return st;
  const double alpha = P->spec_lo, beta = P->spec_hi;
  if (!(alpha > 0.0 && beta > alpha)) {
    P->last_error = "Chebyshev acceleration needs a positive spectrum interval (lo > 0)";
    return H6_ERR_ARG;
  }
  const double theta = 0.5 * (alpha + beta), delta = 0.5 * (beta - alpha), sigma = theta / delta;
  double2* e = P->V;
  int nh = 0;
  st = residual_async(c, F, U, P->r);
  if (st == H6_OK) st = wait(c);
  if (st != H6_OK) return st;
  info->iters = 0;
  info->rel_resid = std::sqrt(c.host[kNorm]) / normF;
  if (info->rel_resid <= info->tol) { info->history_len = 0; return H6_OK; }
  double rho = 1.0 / sigma;
  H6_TRY_HIP(launch_pinv(P, P->r, P->t, c.s));
  H6_TRY_HIP(hipMemsetAsync(e, 0, c.N * sizeof(double2), c.s));
  H6_TRY_HIP(launch_cheb_update(e, P->t, U, 0.0, 1.0 / theta, c.N, c.s));   // e_0; U_1 = U_0 + e_0
  while (true) {
    st = residual_async(c, F, U, P->r);
    if (st == H6_OK) st = wait(c);
    if (st != H6_OK) return st;
    info->iters += 1;
    info->rel_resid = std::sqrt(c.host[kNorm]) / normF;
    record(info, nh, info->rel_resid);
    if (info->rel_resid <= info->tol) { info->history_len = nh; return H6_OK; }
    if (!std::isfinite(info->rel_resid) || info->rel_resid > 1e4) { info->history_len = nh; return H6_DIVERGED; }
    if (info->iters >= info->maxit) { info->history_len = nh; return H6_NOT_CONVERGED; }
    const double rho_next = 1.0 / (2.0 * sigma - rho);
    H6_TRY_HIP(launch_pinv(P, P->r, P->t, c.s));
    H6_TRY_HIP(launch_cheb_update(e, P->t, U, rho_next * rho, 2.0 * rho_next / delta, c.N, c.s));
    rho = rho_next;
  }
}

}  // namespace

void release_graphs(h6_plan P) {
  for (auto& g : P->step_graphs)
    if (g) (void)hipGraphExecDestroy(g);
  P->step_graphs.clear();
  if (P->cycle_graph) (void)hipGraphExecDestroy(P->cycle_graph);
  P->cycle_graph = nullptr;
  P->graph_key = GraphKey{};
}

h6_status run_solve(h6_plan P, const double2* F, double2* U, h6_solve_info* info, hipStream_t s) {
  h6_status st = ensure(P, info->method, info->restart);
  if (st != H6_OK) return st;
  const bool krylov = info->method == H6_GMRES || info->method == H6_FGMRES;
  if (P->use_graphs && krylov && !P->timing.enabled && !P->net) {
    // graph mode runs on the plan's own stream (capturable), after the
    // caller's pending work
    if (!P->gstream) H6_TRY_HIP(hipStreamCreateWithFlags(&P->gstream, hipStreamNonBlocking));
    if (!P->ev_order) H6_TRY_HIP(hipEventCreateWithFlags(&P->ev_order, hipEventDisableTiming));
    H6_TRY_HIP(hipEventRecord(P->ev_order, s));
    H6_TRY_HIP(hipStreamWaitEvent(P->gstream, P->ev_order, 0));
    s = P->gstream;
  }
  Ctx c{P, s, P->N, reinterpret_cast<double*>(P->d_scal), reinterpret_cast<double*>(P->h_pinned)};
  info->iters = 0;
  const bool zero_guess = info->zero_guess != 0;
  // |F| from its first residual pass, or from a norm pass from a zero guess
  if (info->method == H6_SKS) return sks(c, F, U, info, zero_guess);
  if (zero_guess) H6_TRY_HIP(hipMemsetAsync(U, 0, c.N * sizeof(double2), c.s));
  double normF2 = 0.0;
  st = norm2(c, F, &normF2);
  if (st != H6_OK) return st;
  const double normF = std::sqrt(normF2);
  if (normF == 0.0) return zero_solution(c, U, info);
  if (info->method == H6_CHEBYSHEV) return chebyshev(c, F, U, info, normF);
  return gmres(c, F, U, info, normF);
}

// Queued batch: problems grouped by grid shape (dims, faces, precision); per
// group a few lanes, each a plan of that shape with its own workspace and
// right-hand side / solution slots, and a device-side queue of the group's
// problems in decreasing order of estimated cost.  One captured graph holds
// every lane of every group (each lane forked onto its own stream); a replay
// advances each lane by one restart cycle, and the lanes themselves decide
// on the device when their problem is done and which problem comes next
// (queue.hip).  The host replays the graph until every lane reports an
// empty queue.  queue_create builds the lanes and the graph once;
// queue_solve fills the queue with the caller's vectors and tolerances and
// replays.
void queue_destroy(h6_queue Q) {
  if (!Q) return;
  if (Q->exec) (void)hipGraphExecDestroy(Q->exec);
  if (Q->graph) (void)hipGraphDestroy(Q->graph);
  for (QLane& l : Q->L) {
    if (l.join) (void)hipEventDestroy(l.join);
    if (l.s) (void)hipStreamDestroy(l.s);
    (void)hipFree(l.F);
    (void)hipFree(l.U);
    helmholtz6_destroy(l.P);
  }
  if (Q->fork) (void)hipEventDestroy(Q->fork);
  if (Q->s0) (void)hipStreamDestroy(Q->s0);
  (void)hipFree(Q->d_q);
  (void)hipFree(Q->d_head);
  (void)hipFree(Q->d_lanes);
  if (Q->h_res) (void)hipHostFree(Q->h_res);
  if (Q->h_idle) (void)hipHostFree(Q->h_idle);
  delete Q;
}

h6_status queue_create(h6_plan* plans, int count, int m, int lanes, h6_queue* out, std::string& err) {
  *out = nullptr;
  if (m < 1 || m > 256) { err = "restart must be in 1..256"; return H6_ERR_ARG; }
  for (int i = 0; i < count; ++i)
    if (!plans[i]) { err = "null plan"; return H6_ERR_ARG; }
  h6_queue Q = new h6_queue_s();
  Q->m = m;
  Q->count = count;
  Q->plans.assign(plans, plans + count);
  h6_status st = H6_OK;
  auto fail = [&](const std::string& what, hipError_t e) {
    err = what + ": " + hipGetErrorString(e);
    st = e == hipErrorOutOfMemory ? H6_ERR_ALLOC : H6_ERR_HIP;
    queue_destroy(Q);
    return st;
  };
  // groups of one grid shape, each in decreasing order of estimated cost
  using Key = std::tuple<int, int, int, int, int, int, int, int, int, int>;
  std::map<Key, std::vector<int>> groups;
  std::vector<double> cost(count);
  for (int i = 0; i < count; ++i) {
    const h6_plan P = plans[i];
    const double kh = std::abs(P->k) * P->p.h;
    cost[i] = double(P->N) * (1.0 + 40.0 * kh * kh);
    groups[Key{P->dims[0], P->dims[1], P->dims[2], P->p.bc[0], P->p.bc[2], P->p.bc[4], P->p.bc[5],
               P->p.precision, P->xmirror, P->ymirror}].push_back(i);
  }
  for (auto& kv : groups) {
    std::vector<int>& ids = kv.second;
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    Q->goff.push_back(int(Q->order.size()));
    Q->gcount.push_back(int(ids.size()));
    Q->order.insert(Q->order.end(), ids.begin(), ids.end());
    const int nl = std::min(lanes, int(ids.size()));
    for (int l = 0; l < nl; ++l) {
      Q->L.emplace_back();
      QLane& ln = Q->L.back();
      ln.group = int(Q->goff.size()) - 1;
      const h6_plan src = plans[ids[0]];
      h6_status s1 = helmholtz6_setup(&src->p, nullptr, &ln.P);
      if (s1 != H6_OK) {
        err = "lane plan setup failed";
        queue_destroy(Q);
        return s1;
      }
      // the kernel variants chosen for the group's plans (transform path and
      // width where the lane plan has that path's tables)
      ln.P->stencil_tz = src->stencil_tz;
      for (int a = 0; a < 2; ++a) {
        const int f = src->ax[a].fast;
        if (f == 0 || (f == 1 && ln.P->ax[a].rader_mem) || (f == 2 && ln.P->ax[a].blue_mem)) {
          ln.P->ax[a].fast = f;
          ln.P->ax[a].lines = src->ax[a].lines;
        }
      }
      ln.P->use_graphs = 2;                           // device least-squares state
      s1 = ensure(ln.P, H6_FGMRES, m);
      if (s1 != H6_OK) {
        err = ln.P->last_error;
        queue_destroy(Q);
        return s1;
      }
      const size_t vb = ln.P->N * sizeof(double2);
      hipError_t e = hipMalloc(reinterpret_cast<void**>(&ln.F), vb);
      if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ln.U), vb);
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ln.join, hipEventDisableTiming);
      if (e != hipSuccess) return fail("lane allocation", e);
    }
  }
  const int nl = int(Q->L.size());
  {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&Q->d_q), sizeof(QueueEntry) * count);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&Q->d_head), sizeof(int) * Q->goff.size());
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&Q->h_res), sizeof(QueueResult) * count,
                                           hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&Q->d_res), Q->h_res, 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&Q->h_idle), sizeof(int) * nl,
                                           hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&Q->d_idle), Q->h_idle, 0);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&Q->d_lanes), sizeof(QueueLane) * nl);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&Q->s0, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&Q->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail("queue set-up", e);
  }
  // capture: every lane forked from s0 onto its own stream
  hipError_t e = hipStreamBeginCapture(Q->s0, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) e = hipEventRecord(Q->fork, Q->s0);
  for (int l = 0; l < nl && e == hipSuccess; ++l) {
    QLane& ln = Q->L[l];
    h6_plan P = ln.P;
    QueueLane* lane = Q->d_lanes + l;
    const QueueEntry* q = Q->d_q + Q->goff[ln.group];
    const int qn = Q->gcount[ln.group];
    Ctx c{P, ln.s, P->N, reinterpret_cast<double*>(P->d_scal), reinterpret_cast<double*>(P->h_pinned)};
    const GivensState gs = givens_state(P, m);
    const bool mixed = P->p.precision == H6_MIXED;
    e = hipStreamWaitEvent(ln.s, Q->fork, 0);
    int nparts = 0;
    P->skip = &lane->idle;
    if (e == hipSuccess) e = launch_stencil(P, ln.U, P->V, ln.F, P->partials, &nparts, ln.s);
    P->skip = nullptr;
    if (e == hipSuccess) e = launch_reduce_sum_skip(P->partials, nparts, c.dev + kNorm, &lane->idle, ln.s);
    if (e == hipSuccess) e = launch_lane_check(lane, q, Q->d_head + ln.group, qn, c.dev + kNorm, Q->d_res, ln.s);
    if (e == hipSuccess) {
      const size_t cst_bytes = size_t(z_segments(P->dims[2], mixed)) * P->dims[0] * P->dims[1] *
                               (mixed ? sizeof(float2) : sizeof(double2));
      const LaneRefill a{lane, q, ln.F, ln.U, P->V, P->d_stencil, P->d_cstart, P->d_zparams, P->N,
                         cst_bytes / 8, P->partials};
      e = launch_lane_refill(a, ln.s);
    }
    if (e == hipSuccess)
      e = launch_reduce_sum_skip(P->partials, kRedBlocks, c.dev + kNorm, &lane->skip_fresh, ln.s);
    if (e == hipSuccess)
      e = launch_lane_cycle(lane, q, Q->d_res, c.dev + kNorm, c.dev + kPrm, gs.stop, gs.jdone, m, ln.s);
    if (e == hipSuccess) e = enqueue_cycle(c, ln.U, m, true, mixed, gs);
    if (e == hipSuccess) e = launch_lane_count(lane, gs.jdone, ln.s);
    if (e == hipSuccess) e = hipEventRecord(ln.join, ln.s);
    if (e == hipSuccess) e = hipStreamWaitEvent(Q->s0, ln.join, 0);
  }
  const hipError_t e2 = hipStreamEndCapture(Q->s0, &Q->graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&Q->exec, Q->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return fail("queue graph capture", e);
  *out = Q;
  return H6_OK;
}

h6_status queue_solve(h6_queue Q, const double2* const* F, double2* const* U, h6_solve_info* infos,
                      h6_status* statuses, std::string& err) {
  const int count = Q->count, nl = int(Q->L.size()), m = Q->m;
  std::vector<QueueEntry> entries(count);
  for (int k = 0; k < count; ++k) {
    const int i = Q->order[k];
    const h6_solve_info& in = infos[i];
    if (!F[i] || !U[i] || F[i] == U[i]) { err = "null or aliased vector"; return H6_ERR_ARG; }
    if (in.method != H6_FGMRES || in.restart != m || in.maxit < 1 || !(in.tol >= 0.0)) {
      err = "the queued batch runs flexible GMRES with the queue's restart length, maxit >= 1 and tol >= 0";
      return H6_ERR_ARG;
    }
    const h6_plan P = Q->plans[i];
    entries[k] = QueueEntry{F[i], U[i], P->d_stencil, P->d_cstart, P->d_zparams, in.tol, in.maxit, i};
  }
  for (int i = 0; i < count; ++i) Q->h_res[i] = QueueResult{0, int(H6_ERR_HIP), 0.0};
  std::vector<QueueLane> init(nl);
  for (int l = 0; l < nl; ++l) {
    Q->h_idle[l] = 0;
    init[l] = QueueLane{-1, -1, -1, 0, 0, 1, 1, 0, 0.0, Q->d_idle + l};
  }
  hipError_t e = hipMemcpyAsync(Q->d_q, entries.data(), sizeof(QueueEntry) * count, hipMemcpyHostToDevice, Q->s0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(Q->d_lanes, init.data(), sizeof(QueueLane) * nl, hipMemcpyHostToDevice, Q->s0);
  if (e == hipSuccess) e = hipMemsetAsync(Q->d_head, 0, sizeof(int) * Q->goff.size(), Q->s0);
  for (int l = 0; l < nl && e == hipSuccess; ++l) {    // the lanes start from empty slots
    const size_t vb = Q->L[l].P->N * sizeof(double2);
    e = hipMemsetAsync(Q->L[l].F, 0, vb, Q->s0);
    if (e == hipSuccess) e = hipMemsetAsync(Q->L[l].U, 0, vb, Q->s0);
  }
  // replays until every lane found its queue empty (bounded by the step budgets)
  long long bound = 2;
  for (int i = 0; i < count; ++i) bound += (infos[i].maxit + m - 1) / m + 2;
  bool drained = false;
  for (long long rep = 0; rep < bound && e == hipSuccess; ++rep) {
    e = hipGraphLaunch(Q->exec, Q->s0);
    if (e == hipSuccess) e = hipStreamSynchronize(Q->s0);
    if (e != hipSuccess) break;
    drained = true;
    for (int l = 0; l < nl; ++l) drained = drained && Q->h_idle[l] != 0;
    if (drained) break;
  }
  if (e != hipSuccess) {
    err = std::string("queue replay: ") + hipGetErrorString(e);
    return H6_ERR_HIP;
  }
  if (!drained) {
    err = "internal: the queued batch did not drain within its step budget";
    return H6_ERR_HIP;
  }
  h6_status st = H6_OK;
  for (int i = 0; i < count; ++i) {
    statuses[i] = h6_status(Q->h_res[i].status);
    infos[i].iters = Q->h_res[i].iters;
    infos[i].rel_resid = Q->h_res[i].rel_resid;
    infos[i].history_len = 0;
    if (statuses[i] < 0 && st == H6_OK) st = statuses[i];
  }
  return st;
}

}  // namespace h6
