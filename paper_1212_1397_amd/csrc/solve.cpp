// Host control loops of the solvers: right-preconditioned restarted GMRES(m)
// and flexible GMRES(m) with modified Gram-Schmidt Arnoldi (Section 2,
// eq. (AAP)), and the SKS iteration (Section 2, Algorithm 1) in correction
// form.  All vector work is enqueued on the caller's stream; per Arnoldi step
// only the Hessenberg column (j + 2 complex values) crosses to the host, where
// the complex Givens QR update and the least-squares residual estimate are
// computed in FP64.  The stopping test of a cycle uses the least-squares
// estimate; convergence is declared on the true residual ||F - A U|| / ||F||,
// recomputed at every restart.
#include <cmath>
#include <vector>

#include "h6_internal.h"

namespace h6 {
namespace {

struct Ctx {
  h6_plan P;
  hipStream_t s;
  size_t N;
  double2* d_h;       // device Hessenberg column / scratch scalars
  double2* d_y;       // device least-squares coefficients
  double2* d_norm;    // device norm slot
  double2* d_beta;    // device slot holding beta^2 at a cycle start
};

// pinned host slots: [0, 300) Hessenberg column, 300 beta^2, [320, 576) y
constexpr int kPinH = 0, kPinBeta = 300, kPinY = 320;

h6_status ensure(h6_plan P, int method, int m) {
  const size_t vb = P->N * sizeof(double2);
  auto grow = [&](void** ptr, int* cols, int want) -> hipError_t {
    if (*cols >= want) return hipSuccess;
    (void)hipFree(*ptr);
    *ptr = nullptr;
    *cols = 0;
    hipError_t e = hipMalloc(ptr, vb * size_t(want));
    if (e == hipSuccess) *cols = want;
    return e;
  };
  hipError_t e = hipSuccess;
  if (!P->r) e = hipMalloc(reinterpret_cast<void**>(&P->r), vb);
  if (e == hipSuccess && !P->t) e = hipMalloc(reinterpret_cast<void**>(&P->t), vb);
  if (e == hipSuccess && method != H6_SKS)
    e = grow(reinterpret_cast<void**>(&P->V), &P->V_cols, m + 1);
  if (e == hipSuccess && method == H6_FGMRES) e = grow(&P->Z, &P->Z_cols, m);
  if (e != hipSuccess) {
    P->last_error = std::string("workspace allocation failed: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? H6_ERR_ALLOC : H6_ERR_HIP;
  }
  return H6_OK;
}

// |v|^2 of a device vector into host (synchronises)
h6_status norm2(Ctx& c, const double2* v, double* out) {
  h6_plan P = c.P;
  hipEvent_t ev;
  timing_begin(P, KC_NORM, c.s, &ev);
  H6_TRY_HIP(launch_norm2_partials(v, c.N, P->partials, c.s));
  H6_TRY_HIP(launch_reduce(P->partials, kRedBlocks, 2, c.d_norm, c.s));
  timing_end(P, KC_NORM, c.s, ev);
  H6_TRY_HIP(hipMemcpyAsync(P->h_pinned, c.d_norm, sizeof(double2), hipMemcpyDeviceToHost, c.s));
  H6_TRY_HIP(hipStreamSynchronize(c.s));
  *out = P->h_pinned[0].x;
  return H6_OK;
}

// r = F - A U and |r|^2 on the host (synchronises)
h6_status residual(Ctx& c, const double2* F, const double2* U, double2* r, double* out) {
  h6_plan P = c.P;
  int nparts = 0;
  H6_TRY_HIP(launch_stencil(P, U, r, F, P->partials, &nparts, c.s));
  H6_TRY_HIP(launch_reduce(P->partials, nparts, 1, c.d_norm, c.s));
  H6_TRY_HIP(hipMemcpyAsync(P->h_pinned, c.d_norm, sizeof(double2), hipMemcpyDeviceToHost, c.s));
  H6_TRY_HIP(hipStreamSynchronize(c.s));
  *out = P->h_pinned[0].x;
  return H6_OK;
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

h6_status gmres(Ctx& c, const double2* F, double2* U, h6_solve_info* info, double normF) {
  h6_plan P = c.P;
  const int m = info->restart;
  const bool flex = info->method == H6_FGMRES;
  const size_t N = c.N;
  int nh = 0;
  double beta2 = 0.0;
  h6_status st = residual(c, F, U, P->r, &beta2);
  if (st != H6_OK) return st;
  std::vector<cplx> H(size_t(m + 1) * m), g(m + 1), sn(m);
  std::vector<double> cs(m);
  auto Hij = [&](int i, int j) -> cplx& { return H[size_t(i) * m + j]; };
  info->iters = 0;
  while (true) {
    const double beta = std::sqrt(beta2);
    info->rel_resid = beta / normF;
    if (!std::isfinite(info->rel_resid)) { info->history_len = nh; return H6_DIVERGED; }
    if (info->rel_resid <= info->tol) { info->history_len = nh; return H6_OK; }
    if (info->iters >= info->maxit) { info->history_len = nh; return H6_NOT_CONVERGED; }
    // v_0 = r / beta
    P->h_pinned[kPinBeta] = make_double2(beta2, 0.0);
    H6_TRY_HIP(hipMemcpyAsync(c.d_beta, P->h_pinned + kPinBeta, sizeof(double2), hipMemcpyHostToDevice, c.s));
    H6_TRY_HIP(launch_scale_inv_norm(P->V, P->r, c.d_beta, N, c.s));
    std::fill(g.begin(), g.end(), cplx(0.0));
    g[0] = beta;
    int jdone = 0;
    for (int j = 0; j < m; ++j) {
      double2* vj = P->V + size_t(j) * N;
      double2* w = P->V + size_t(j + 1) * N;
      double2* z = flex ? static_cast<double2*>(P->Z) + size_t(j) * N : P->t;
      H6_TRY_HIP(launch_pinv(P, vj, z, c.s));
      H6_TRY_HIP(launch_stencil(P, z, w, nullptr, nullptr, nullptr, c.s));
      info->iters += 1;
      // modified Gram-Schmidt; kernel i applies the update of basis vector i-1
      // and forms the partial inner product with basis vector i
      hipEvent_t ev;
      timing_begin(P, KC_MGS, c.s, &ev);
      for (int i = 0; i <= j; ++i) {
        const double2* vprev = i > 0 ? P->V + size_t(i - 1) * N : nullptr;
        H6_TRY_HIP(launch_mgs_step(w, vprev, c.d_h + (i > 0 ? i - 1 : 0), P->V + size_t(i) * N, N,
                                   P->partials, c.s));
        H6_TRY_HIP(launch_reduce(P->partials, kRedBlocks, 2, c.d_h + i, c.s));
      }
      H6_TRY_HIP(launch_axpy_norm(w, vj, c.d_h + j, N, P->partials, c.s));
      H6_TRY_HIP(launch_reduce(P->partials, kRedBlocks, 2, c.d_h + j + 1, c.s));
      timing_end(P, KC_MGS, c.s, ev);
      H6_TRY_HIP(hipMemcpyAsync(P->h_pinned + kPinH, c.d_h, sizeof(double2) * (j + 2), hipMemcpyDeviceToHost, c.s));
      H6_TRY_HIP(hipStreamSynchronize(c.s));
      const double2* hc = P->h_pinned + kPinH;
      for (int i = 0; i <= j; ++i) Hij(i, j) = cplx(hc[i].x, hc[i].y);
      const double hn2 = hc[j + 1].x;
      const double hn = std::sqrt(std::max(hn2, 0.0));
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
      const bool breakdown = !(hn > 1e-300 * beta);
      if (est <= info->tol || info->iters >= info->maxit || breakdown || j + 1 == m) break;
      // v_{j+1} = w / |w| (the device norm slot d_h[j+1] holds |w|^2)
      H6_TRY_HIP(launch_scale_inv_norm(w, w, c.d_h + j + 1, N, c.s));
    }
    // y = R^{-1} g
    std::vector<cplx> y(jdone);
    for (int i = jdone - 1; i >= 0; --i) {
      cplx acc = g[i];
      for (int k = i + 1; k < jdone; ++k) acc -= Hij(i, k) * y[k];
      y[i] = acc / Hij(i, i);
    }
    for (int i = 0; i < jdone; ++i) P->h_pinned[kPinY + i] = make_double2(y[i].real(), y[i].imag());
    H6_TRY_HIP(hipMemcpyAsync(c.d_y, P->h_pinned + kPinY, sizeof(double2) * jdone, hipMemcpyHostToDevice, c.s));
    hipEvent_t ev;
    if (flex) {
      timing_begin(P, KC_AXPY, c.s, &ev);
      H6_TRY_HIP(launch_multi_axpy(U, static_cast<double2*>(P->Z), c.d_y, jdone, N, 1, c.s));
      timing_end(P, KC_AXPY, c.s, ev);
    } else {
      timing_begin(P, KC_AXPY, c.s, &ev);
      H6_TRY_HIP(launch_multi_axpy(P->t, P->V, c.d_y, jdone, N, 0, c.s));
      timing_end(P, KC_AXPY, c.s, ev);
      H6_TRY_HIP(launch_pinv(P, P->t, P->r, c.s));
      timing_begin(P, KC_AXPY, c.s, &ev);
      H6_TRY_HIP(launch_add(U, P->r, N, c.s));
      timing_end(P, KC_AXPY, c.s, ev);
    }
    st = residual(c, F, U, P->r, &beta2);
    if (st != H6_OK) return st;
  }
}

// SKS, Algorithm 1, in correction form: U += A_p^{-1} r, r = F - A U.
h6_status sks(Ctx& c, const double2* F, double2* U, h6_solve_info* info, double normF) {
  h6_plan P = c.P;
  int nh = 0;
  double r2 = 0.0;
  h6_status st = residual(c, F, U, P->r, &r2);
  if (st != H6_OK) return st;
  info->iters = 0;
  while (true) {
    info->rel_resid = std::sqrt(r2) / normF;
    if (info->rel_resid <= info->tol) { info->history_len = nh; return H6_OK; }
    if (!std::isfinite(info->rel_resid) || (info->iters > 0 && info->rel_resid > 1e4)) {
      info->history_len = nh;
      return H6_DIVERGED;
    }
    if (info->iters >= info->maxit) { info->history_len = nh; return H6_NOT_CONVERGED; }
    H6_TRY_HIP(launch_pinv(P, P->r, P->t, c.s));
    hipEvent_t ev;
    timing_begin(P, KC_AXPY, c.s, &ev);
    H6_TRY_HIP(launch_add(U, P->t, c.N, c.s));
    timing_end(P, KC_AXPY, c.s, ev);
    st = residual(c, F, U, P->r, &r2);
    if (st != H6_OK) return st;
    info->iters += 1;
    record(info, nh, std::sqrt(r2) / normF);
  }
}

}  // namespace

h6_status run_solve(h6_plan P, const double2* F, double2* U, h6_solve_info* info, hipStream_t s) {
  h6_status st = ensure(P, info->method, info->restart);
  if (st != H6_OK) return st;
  Ctx c{P, s, P->N, P->d_scal + 64, P->d_scal + 512, P->d_scal + 8, P->d_scal + 16};
  if (info->method != H6_SKS && info->restart + 2 > 448) return H6_ERR_ARG;
  double normF2 = 0.0;
  st = norm2(c, F, &normF2);
  if (st != H6_OK) return st;
  const double normF = std::sqrt(normF2);
  info->iters = 0;
  if (normF == 0.0) {
    H6_TRY_HIP(hipMemsetAsync(U, 0, P->N * sizeof(double2), s));
    H6_TRY_HIP(hipStreamSynchronize(s));
    info->rel_resid = 0.0;
    info->history_len = 0;
    return H6_OK;
  }
  if (info->method == H6_SKS) return sks(c, F, U, info, normF);
  return gmres(c, F, U, info, normF);
}

}  // namespace h6
