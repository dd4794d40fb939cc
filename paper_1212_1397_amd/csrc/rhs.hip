// F = h^2-scaled compact right-hand side for a sum of Gaussian sources
//   f = sum_s a_s exp(-|x - c_s|^2 / (2 sigma^2)),
// one thread per unknown node.
//
// Interior part, eq. (scheme) right side times h^2 (mixed fourth-derivative
// coefficient h^4/180, the value that makes the scheme sixth order):
//   h^2 [ c_K f + (h^2/12)(1 - kappa/30) lap f + (h^4/360) lap^2 f
//         + (h^4/180)(f_xxyy + f_xxzz + f_yyzz) ].
// Neumann face with normal axis n (eq. (3DN), beta = 0): +- 2h R_N with
//   R_N = (h^2/6)(1 - kappa/20) f_n + (h^4/120) f_nnn + (7h^4/360)(f_n t1t1 + f_n t2t2)
// (+ on the low face, - on the high face).
// Sommerfeld z face (eqs. (3DIMP), (3DDISCS)): + e^{ikh} mu3 [2h Fbar + mu1 (h^5/3) Lbar]
// with fbar_m = d^m/dz'^m (e^{ikz'} f), Lbar = fbar_xxz + fbar_yyz and
//   Fbar = (h^2/6 + k^2h^4/45) fbar_1 - (ikh^4/90) fbar_2 + (h^4/120)(fbar_3 - Lbar),
// z' = z at the bottom face and z' = top - z at the top face.
//
// Gaussian derivatives: d^n/dx^n exp(-t^2/2), t = (x - c)/sigma, equals
// (-1/sigma)^n He_n(t) exp(-t^2/2) with the probabilists' Hermite polynomials.
#include "h6_internal.h"

namespace h6 {
namespace {

constexpr int kMaxSrc = 64;

struct RhsArgs {
  int nsrc;
  int n[3];        // interior counts
  int dims[3];     // unknown counts
  int qlo[3];      // q index of the first unknown per axis
  int face[6];
  double h, inv_sigma;
  double2 cK, c_lap, c_bil, c_mix;               // interior coefficients (already times h^2)
  double2 nN1, nN3, nNm;                         // Neumann R_N coefficients (times 2h)
  double2 ik, sA, sB, sC, e1mu3, mu1h5;          // Sommerfeld coefficients
  double cx[kMaxSrc], cy[kMaxSrc], cz[kMaxSrc];
  double2 amp[kMaxSrc];
};

__device__ __forceinline__ void gauss_derivs(double x, double c, double is, double g[5]) {
  const double t = (x - c) * is;
  const double e = exp(-0.5 * t * t);
  const double t2 = t * t;
  const double he[5] = {1.0, t, t2 - 1.0, t * (t2 - 3.0), t2 * t2 - 6.0 * t2 + 3.0};
  double s = 1.0;
  for (int k = 0; k < 5; ++k) {
    g[k] = s * he[k] * e;
    s *= -is;
  }
}

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 ca(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cs(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// index of the derivative combinations accumulated per node
enum {
  D000, D200, D020, D002, D400, D040, D004, D220, D202, D022,
  D100, D300, D120, D102, D010, D030, D210, D012, D001, D003, D201, D021, ND
};

__global__ __launch_bounds__(256) void rhs_kernel(RhsArgs a, double2* __restrict__ F) {
  const size_t N = size_t(a.dims[0]) * a.dims[1] * a.dims[2];
  const size_t idx = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
  if (idx >= N) return;
  const int i = int(idx % a.dims[0]);
  const int j = int((idx / a.dims[0]) % a.dims[1]);
  const int l = int(idx / (size_t(a.dims[0]) * a.dims[1]));
  const int q[3] = {i + a.qlo[0], j + a.qlo[1], l + a.qlo[2]};
  const double X = q[0] * a.h, Y = q[1] * a.h, Z = q[2] * a.h;
  double2 d[ND];
  for (int t = 0; t < ND; ++t) d[t] = make_double2(0.0, 0.0);
  for (int s = 0; s < a.nsrc; ++s) {
    double gx[5], gy[5], gz[5];
    gauss_derivs(X, a.cx[s], a.inv_sigma, gx);
    gauss_derivs(Y, a.cy[s], a.inv_sigma, gy);
    gauss_derivs(Z, a.cz[s], a.inv_sigma, gz);
    const double2 A = a.amp[s];
    const double v[ND] = {
        gx[0] * gy[0] * gz[0], gx[2] * gy[0] * gz[0], gx[0] * gy[2] * gz[0], gx[0] * gy[0] * gz[2],
        gx[4] * gy[0] * gz[0], gx[0] * gy[4] * gz[0], gx[0] * gy[0] * gz[4], gx[2] * gy[2] * gz[0],
        gx[2] * gy[0] * gz[2], gx[0] * gy[2] * gz[2], gx[1] * gy[0] * gz[0], gx[3] * gy[0] * gz[0],
        gx[1] * gy[2] * gz[0], gx[1] * gy[0] * gz[2], gx[0] * gy[1] * gz[0], gx[0] * gy[3] * gz[0],
        gx[2] * gy[1] * gz[0], gx[0] * gy[1] * gz[2], gx[0] * gy[0] * gz[1], gx[0] * gy[0] * gz[3],
        gx[2] * gy[0] * gz[1], gx[0] * gy[2] * gz[1]};
    for (int t = 0; t < ND; ++t) d[t] = ca(d[t], cs(A, v[t]));
  }
  const double2 lap = ca(ca(d[D200], d[D020]), d[D002]);
  const double2 mix = ca(ca(d[D220], d[D202]), d[D022]);
  const double2 quart = ca(ca(d[D400], d[D040]), d[D004]);
  // c_bil multiplies lap^2 f = quart + 2 mix; c_mix multiplies mix
  double2 Fv = ca(ca(cm(a.cK, d[D000]), cm(a.c_lap, lap)),
                  ca(cm(a.c_bil, ca(quart, cs(mix, 2.0))), cm(a.c_mix, mix)));

  // Neumann faces: normal derivative, its cube and the mixed terms
  const int dn[3][4] = {{D100, D300, D120, D102}, {D010, D030, D210, D012}, {D001, D003, D201, D021}};
  for (int ax = 0; ax < 3; ++ax)
    for (int side = 0; side < 2; ++side) {
      if (a.face[2 * ax + side] != H6_NEUMANN) continue;
      const bool on = side == 0 ? q[ax] == 0 : q[ax] == a.n[ax] + 1;
      if (!on) continue;
      double2 RN = ca(ca(cm(a.nN1, d[dn[ax][0]]), cm(a.nN3, d[dn[ax][1]])),
                      cm(a.nNm, ca(d[dn[ax][2]], d[dn[ax][3]])));
      Fv = ca(Fv, cs(RN, side == 0 ? 1.0 : -1.0));
    }
  // Sommerfeld z faces
  for (int side = 0; side < 2; ++side) {
    if (a.face[4 + side] != H6_SOMMERFELD) continue;
    const bool on = side == 0 ? q[2] == 0 : q[2] == a.n[2] + 1;
    if (!on) continue;
    const double sg = side == 0 ? 1.0 : -1.0;
    // z'-derivatives of f: f, f_z', f_z'z', f_z'z'z'
    const double2 f0 = d[D000], f1 = cs(d[D001], sg), f2 = d[D002], f3 = cs(d[D003], sg);
    const double2 ik = a.ik, ik2 = cm(ik, ik), ik3 = cm(ik2, ik);
    const double2 fb1 = ca(cm(ik, f0), f1);
    const double2 fb2 = ca(ca(cm(ik2, f0), cs(cm(ik, f1), 2.0)), f2);
    const double2 fb3 = ca(ca(cm(ik3, f0), cs(cm(ik2, f1), 3.0)), ca(cs(cm(ik, f2), 3.0), f3));
    const double2 Lb = ca(cm(ik, ca(d[D200], d[D020])), cs(ca(d[D201], d[D021]), sg));
    const double2 Fb = ca(ca(cm(a.sA, fb1), cs(cm(a.sB, fb2), -1.0)),
                          cm(a.sC, ca(fb3, cs(Lb, -1.0))));
    Fv = ca(Fv, cm(a.e1mu3, ca(cs(Fb, 2.0 * a.h), cm(a.mu1h5, Lb))));
  }
  F[idx] = Fv;
}

double2 d2(cplx c) { return make_double2(c.real(), c.imag()); }

}  // namespace

hipError_t launch_rhs(h6_plan P, int nsrc, const double* centres, const double* amps,
                      double sigma, double2* F, hipStream_t s) {
  if (nsrc > kMaxSrc) return hipErrorInvalidValue;
  RhsArgs a{};
  a.nsrc = nsrc;
  for (int ax = 0; ax < 3; ++ax) {
    a.n[ax] = P->p.n[ax];
    a.dims[ax] = P->dims[ax];
    a.qlo[ax] = P->p.bc[2 * ax] != H6_DIRICHLET ? 0 : 1;
  }
  for (int f = 0; f < 6; ++f) a.face[f] = P->p.bc[f];
  const double h = P->p.h;
  const cplx I(0.0, 1.0), k = P->k, kap = P->kappa, ikh = I * k * h;
  a.h = h;
  a.inv_sigma = 1.0 / sigma;
  const double h2 = h * h, h4 = h2 * h2;
  a.cK = d2(h2 * (1.0 - kap / 12.0 + kap * kap / 360.0));
  a.c_lap = d2(h2 * (h2 / 12.0) * (1.0 - kap / 30.0));
  a.c_bil = d2(cplx(h2 * h4 / 360.0));
  a.c_mix = d2(cplx(h2 * h4 / 180.0));
  a.nN1 = d2(2.0 * h * (h2 / 6.0) * (1.0 - kap / 20.0));
  a.nN3 = d2(cplx(2.0 * h * h4 / 120.0));
  a.nNm = d2(cplx(2.0 * h * 7.0 * h4 / 360.0));
  const cplx mu3 = 1.0 / (1.0 + (2.0 * ikh / 3.0) * (1.0 + 2.0 * kap / 15.0));
  const cplx mu1 = (ikh / 90.0 + (1.0 + kap / 30.0) / (6.0 * mu3)) / (1.0 + 2.0 * ikh / 3.0);
  a.ik = d2(I * k);
  a.sA = d2(h2 / 6.0 + k * k * h4 / 45.0);
  a.sB = d2(I * k * h4 / 90.0);
  a.sC = d2(cplx(h4 / 120.0));
  a.e1mu3 = d2(std::exp(ikh) * mu3);
  a.mu1h5 = d2(mu1 * h * h4 / 3.0);
  for (int i = 0; i < nsrc; ++i) {
    a.cx[i] = centres[3 * i];
    a.cy[i] = centres[3 * i + 1];
    a.cz[i] = centres[3 * i + 2];
    a.amp[i] = make_double2(amps[2 * i], amps[2 * i + 1]);
  }
  hipEvent_t ev;
  timing_begin(P, KC_RHS, s, &ev);
  const size_t nb = (P->N + 255) / 256;
  hipLaunchKernelGGL(rhs_kernel, dim3(unsigned(nb)), dim3(256), 0, s, a, F);
  timing_end(P, KC_RHS, s, ev, double(P->N) * sizeof(double2));
  return hipGetLastError();
}

}  // namespace h6
