// F = h^2-scaled compact right-hand side, one thread per unknown node, for
//  (a) a sum of Gaussian sources f = sum_s a_s exp(-|x - c_s|^2 / (2 sigma^2)),
//  (b) a separable source f = sum_s c_s X_s(x) Y_s(y) Z_s(z) given by samples of
//      each factor and its derivatives up to fourth order at the unknown nodes,
// and (c) the plane term of nonhomogeneous Dirichlet data on a z face, and
// (d) the data term of nonzero Neumann data on a Neumann face.
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
// Dirichlet data g on a z face: the unknown plane next to the face couples to
// the face plane through the in-plane operator G of eq. (scheme)'s delta_z^2
// term, G = I + (1 + kappa/30)/6 (D_x + D_y) + (1/30) D_x D_y (D = h^2 delta^2),
// so F -= G g on that plane.
// Neumann data beta = du/dn (n the face's axis, derivative along +n), eq.
// (3DN): the ghost relation carries -2h B with
//   B = (1 - kappa/6 + kappa^2/120) beta - (h^4/180)(beta_t1t1t2t2 + beta_t1^4 + beta_t2^4)
//       - (k^2 h^4/180)(beta_t1t1 + beta_t2t2),
// so the face's unknown plane gets F += 2h B (low face) or F -= 2h B (high face).
//
// Gaussian derivatives: d^n/dx^n exp(-t^2/2), t = (x - c)/sigma, equals
// (-1/sigma)^n He_n(t) exp(-t^2/2) with the probabilists' Hermite polynomials.
#include "h6_internal.h"

namespace h6 {
namespace {

constexpr int kMaxSrc = 64;

// grid and coefficient data shared by every source form
struct RhsCoef {
  int n[3];        // interior counts
  int dims[3];     // unknown counts
  int qlo[3];      // q index of the first unknown per axis
  int face[6];
  double h;
  double2 cK, c_lap, c_bil, c_mix;               // interior coefficients (already times h^2)
  double2 nN1, nN3, nNm;                         // Neumann R_N coefficients (times 2h)
  double2 ik, sA, sB, sC, e1mu3, mu1h5;          // Sommerfeld coefficients
};

struct RhsArgs {
  RhsCoef c;
  int nsrc;
  double inv_sigma;
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

// F at node q from the accumulated derivative combinations d[] of f there
__device__ double2 assemble(const RhsCoef& a, const double2 (&d)[ND], const int (&q)[3]) {
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
  return Fv;
}

// derivative orders (x, y, z) of each combination
__constant__ int kOrd[ND][3] = {
    {0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {4, 0, 0}, {0, 4, 0}, {0, 0, 4}, {2, 2, 0},
    {2, 0, 2}, {0, 2, 2}, {1, 0, 0}, {3, 0, 0}, {1, 2, 0}, {1, 0, 2}, {0, 1, 0}, {0, 3, 0},
    {2, 1, 0}, {0, 1, 2}, {0, 0, 1}, {0, 0, 3}, {2, 0, 1}, {0, 2, 1}};

__device__ __forceinline__ void node_of(const RhsCoef& a, size_t idx, int (&ijl)[3], int (&q)[3]) {
  ijl[0] = int(idx % a.dims[0]);
  ijl[1] = int((idx / a.dims[0]) % a.dims[1]);
  ijl[2] = int(idx / (size_t(a.dims[0]) * a.dims[1]));
  for (int ax = 0; ax < 3; ++ax) q[ax] = ijl[ax] + a.qlo[ax];
}

__global__ __launch_bounds__(256) void rhs_kernel(RhsArgs a, double2* __restrict__ F) {
  const size_t N = size_t(a.c.dims[0]) * a.c.dims[1] * a.c.dims[2];
  const size_t idx = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
  if (idx >= N) return;
  int ijl[3], q[3];
  node_of(a.c, idx, ijl, q);
  const double X = q[0] * a.c.h, Y = q[1] * a.c.h, Z = q[2] * a.c.h;
  double2 d[ND];
  for (int t = 0; t < ND; ++t) d[t] = make_double2(0.0, 0.0);
  for (int s = 0; s < a.nsrc; ++s) {
    double gx[5], gy[5], gz[5];
    gauss_derivs(X, a.cx[s], a.inv_sigma, gx);
    gauss_derivs(Y, a.cy[s], a.inv_sigma, gy);
    gauss_derivs(Z, a.cz[s], a.inv_sigma, gz);
    const double2 A = a.amp[s];
    for (int t = 0; t < ND; ++t)
      d[t] = ca(d[t], cs(A, gx[kOrd[t][0]] * gy[kOrd[t][1]] * gz[kOrd[t][2]]));
  }
  F[idx] = assemble(a.c, d, q);
}

// Separable source: tab[a] holds, per term s and derivative order o = 0..4,
// the samples of the axis-a factor at the dims[a] unknown nodes of axis a:
// tab[a][(s * 5 + o) * dims[a] + i].  coef[s] multiplies term s.
__global__ __launch_bounds__(256) void rhs_separable_kernel(RhsCoef a, int nterms,
                                                            const double2* __restrict__ coef,
                                                            const double2* __restrict__ tx,
                                                            const double2* __restrict__ ty,
                                                            const double2* __restrict__ tz,
                                                            double2* __restrict__ F) {
  const size_t N = size_t(a.dims[0]) * a.dims[1] * a.dims[2];
  const size_t idx = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
  if (idx >= N) return;
  int ijl[3], q[3];
  node_of(a, idx, ijl, q);
  double2 d[ND];
  for (int t = 0; t < ND; ++t) d[t] = make_double2(0.0, 0.0);
  for (int s = 0; s < nterms; ++s) {
    double2 gx[5], gy[5], gz[5];
    for (int o = 0; o < 5; ++o) {
      gx[o] = tx[size_t(s * 5 + o) * a.dims[0] + ijl[0]];
      gy[o] = ty[size_t(s * 5 + o) * a.dims[1] + ijl[1]];
      gz[o] = tz[size_t(s * 5 + o) * a.dims[2] + ijl[2]];
    }
    const double2 c = coef[s];
    for (int t = 0; t < ND; ++t)
      d[t] = ca(d[t], cm(c, cm(gx[kOrd[t][0]], cm(gy[kOrd[t][1]], gz[kOrd[t][2]]))));
  }
  F[idx] = assemble(a, d, q);
}

// Dirichlet data g (n'x x n'y, x fastest) on a z face: Fp -= G g on the
// adjacent unknown plane Fp.  D_x, D_y take the neighbour outside the unknown
// range as 0 next to a Dirichlet face and as the mirror value (index 1 or
// n' - 2) next to a Neumann face.
struct PlaneRule {
  int nx, ny;
  int xlo_n, xhi_n, ylo_n, yhi_n;   // 1 where that in-plane face is Neumann
};

// index of the neighbour of i (i = -1 or n) under the face rule, or -1 for a zero value
__device__ __forceinline__ int ext_index(int i, int n, int lo_n, int hi_n) {
  if (i >= 0 && i < n) return i;
  if (n < 2) return -1;
  if (i < 0) return lo_n ? 1 : -1;
  return hi_n ? n - 2 : -1;
}

__device__ __forceinline__ double2 dx_row(const double2* __restrict__ g, const PlaneRule& r, int i, int j) {
  const double2* row = g + size_t(j) * r.nx;
  const int im = ext_index(i - 1, r.nx, r.xlo_n, r.xhi_n), ip = ext_index(i + 1, r.nx, r.xlo_n, r.xhi_n);
  double2 v = cs(row[i], -2.0);
  if (im >= 0) v = ca(v, row[im]);
  if (ip >= 0) v = ca(v, row[ip]);
  return v;
}

__global__ __launch_bounds__(256) void dirichlet_plane_kernel(const double2* __restrict__ g,
                                                              double2* __restrict__ Fp, PlaneRule r,
                                                              double2 ca_, double cb) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= r.nx * r.ny) return;
  const int i = idx % r.nx, j = idx / r.nx;
  const int jm = ext_index(j - 1, r.ny, r.ylo_n, r.yhi_n), jp = ext_index(j + 1, r.ny, r.ylo_n, r.yhi_n);
  const double2 g0 = g[idx];
  const double2 dx0 = dx_row(g, r, i, j);
  // D_y g and D_y D_x g at (i, j)
  double2 dy = cs(g0, -2.0), dyx = cs(dx0, -2.0);
  if (jm >= 0) {
    dy = ca(dy, g[size_t(jm) * r.nx + i]);
    dyx = ca(dyx, dx_row(g, r, i, jm));
  }
  if (jp >= 0) {
    dy = ca(dy, g[size_t(jp) * r.nx + i]);
    dyx = ca(dyx, dx_row(g, r, i, jp));
  }
  const double2 Gg = ca(ca(g0, cm(ca_, ca(dx0, dy))), cs(dyx, cb));
  const double2 f = Fp[idx];
  Fp[idx] = make_double2(f.x - Gg.x, f.y - Gg.y);
}

double2 d2(cplx c) { return make_double2(c.real(), c.imag()); }

RhsCoef rhs_coef(h6_plan P) {
  RhsCoef a{};
  for (int ax = 0; ax < 3; ++ax) {
    a.n[ax] = P->p.n[ax];
    a.dims[ax] = P->dims[ax];
    a.qlo[ax] = P->p.bc[2 * ax] != H6_DIRICHLET ? 0 : 1;
  }
  for (int f = 0; f < 6; ++f) a.face[f] = P->p.bc[f];
  const double h = P->p.h;
  const cplx I(0.0, 1.0), k = P->k, kap = P->kappa, ikh = I * k * h;
  a.h = h;
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
  return a;
}

// Neumann data on face plane (axis ax, side): beta = sum_s coef[s] T1_s(t1) T2_s(t2)
// from tables tab1 / tab2 ([(s * 5 + o) * n_t + i], o = derivative order).
struct NeumannFace {
  int n1, n2;                 // unknowns along the tangential axes t1 < t2
  size_t s1, s2;              // strides of t1, t2 in the vector layout
  size_t base;                // offset of the face's unknown plane
  double2 a0, c4, c2;         // 2h (1 - kappa/6 + kappa^2/120), -2h h^4/180, -2h k^2 h^4/180 (signed)
};

__global__ __launch_bounds__(256) void neumann_data_kernel(NeumannFace fc, int nterms,
                                                           const double2* __restrict__ coef,
                                                           const double2* __restrict__ tab1,
                                                           const double2* __restrict__ tab2,
                                                           double2* __restrict__ F) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= fc.n1 * fc.n2) return;
  const int i1 = idx % fc.n1, i2 = idx / fc.n1;
  double2 d00 = make_double2(0, 0), d4 = make_double2(0, 0), d2 = make_double2(0, 0);
  for (int s = 0; s < nterms; ++s) {
    double2 a[5], b[5];
    for (int o = 0; o < 5; ++o) {
      a[o] = tab1[size_t(s * 5 + o) * fc.n1 + i1];
      b[o] = tab2[size_t(s * 5 + o) * fc.n2 + i2];
    }
    const double2 c = coef[s];
    d00 = ca(d00, cm(c, cm(a[0], b[0])));
    d4 = ca(d4, cm(c, ca(ca(cm(a[2], b[2]), cm(a[4], b[0])), cm(a[0], b[4]))));
    d2 = ca(d2, cm(c, ca(cm(a[2], b[0]), cm(a[0], b[2]))));
  }
  const double2 add = ca(ca(cm(fc.a0, d00), cm(fc.c4, d4)), cm(fc.c2, d2));
  const size_t o = fc.base + size_t(i1) * fc.s1 + size_t(i2) * fc.s2;
  const double2 f = F[o];
  F[o] = make_double2(f.x + add.x, f.y + add.y);
}

}  // namespace

hipError_t launch_rhs(h6_plan P, int nsrc, const double* centres, const double* amps,
                      double sigma, double2* F, hipStream_t s) {
  if (nsrc > kMaxSrc) return hipErrorInvalidValue;
  RhsArgs a{};
  a.c = rhs_coef(P);
  a.nsrc = nsrc;
  a.inv_sigma = 1.0 / sigma;
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

hipError_t launch_rhs_separable(h6_plan P, int nterms, const double* coef, const double* const tab[3],
                                double2* F, hipStream_t s) {
  // device copy of the coefficients and the three factor tables, in one
  // plan-owned buffer grown on demand
  const size_t total = size_t(nterms) * (1 + 5 * (size_t(P->dims[0]) + P->dims[1] + P->dims[2]));
  hipError_t e = hipSuccess;
  if (total * sizeof(double2) > P->sep_bytes) {
    (void)hipFree(P->d_sep);
    P->d_sep = nullptr;
    P->sep_bytes = 0;
    e = hipMalloc(&P->d_sep, total * sizeof(double2));
    if (e != hipSuccess) return e;
    P->sep_bytes = total * sizeof(double2);
  }
  double2* base = static_cast<double2*>(P->d_sep);
  const double2* dcoef = base;
  const double2* dtab[3];
  e = hipMemcpyAsync(base, coef, size_t(nterms) * sizeof(double2), hipMemcpyHostToDevice, s);
  size_t at = size_t(nterms);
  for (int ax = 0; ax < 3 && e == hipSuccess; ++ax) {
    const size_t cnt = size_t(nterms) * 5 * P->dims[ax];
    dtab[ax] = base + at;
    e = hipMemcpyAsync(base + at, tab[ax], cnt * sizeof(double2), hipMemcpyHostToDevice, s);
    at += cnt;
  }
  if (e != hipSuccess) return e;
  hipEvent_t ev;
  timing_begin(P, KC_RHS, s, &ev);
  const size_t nb = (P->N + 255) / 256;
  hipLaunchKernelGGL(rhs_separable_kernel, dim3(unsigned(nb)), dim3(256), 0, s, rhs_coef(P), nterms,
                     dcoef, dtab[0], dtab[1], dtab[2], F);
  timing_end(P, KC_RHS, s, ev, double(P->N) * sizeof(double2));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the host tables may be released once the call returns
  return hipStreamSynchronize(s);
}

hipError_t launch_rhs_dirichlet_z(h6_plan P, int side, const double2* g, double2* F, hipStream_t s) {
  PlaneRule r{};
  r.nx = P->dims[0];
  r.ny = P->dims[1];
  r.xlo_n = P->p.bc[0] == H6_NEUMANN;
  r.xhi_n = P->p.bc[1] == H6_NEUMANN;
  r.ylo_n = P->p.bc[2] == H6_NEUMANN;
  r.yhi_n = P->p.bc[3] == H6_NEUMANN;
  const size_t plane = size_t(r.nx) * r.ny;
  double2* Fp = F + (side == 0 ? size_t(0) : plane * (P->dims[2] - 1));
  const double2 ca_ = d2((1.0 + P->kappa / 30.0) / 6.0);
  const unsigned nb = unsigned((plane + 255) / 256);
  hipLaunchKernelGGL(dirichlet_plane_kernel, dim3(nb), dim3(256), 0, s, g, Fp, r, ca_, 1.0 / 30.0);
  return hipGetLastError();
}

hipError_t launch_rhs_neumann(h6_plan P, int face, int nterms, const double* coef, const double* t1,
                              const double* t2, double2* F, hipStream_t s) {
  const int ax = face / 2, side = face % 2;
  const int ta = ax == 0 ? 1 : 0, tb = ax == 2 ? 1 : 2;       // tangential axes, increasing
  const size_t stride[3] = {1, size_t(P->dims[0]), size_t(P->dims[0]) * P->dims[1]};
  NeumannFace fc{};
  fc.n1 = P->dims[ta];
  fc.n2 = P->dims[tb];
  fc.s1 = stride[ta];
  fc.s2 = stride[tb];
  fc.base = side == 0 ? 0 : stride[ax] * size_t(P->dims[ax] - 1);
  const double h = P->p.h, h4 = h * h * h * h;
  const cplx kap = P->kappa, k2 = P->k * P->k;
  const double sg = side == 0 ? 2.0 * h : -2.0 * h;
  fc.a0 = d2(sg * (1.0 - kap / 6.0 + kap * kap / 120.0));
  fc.c4 = d2(cplx(-sg * h4 / 180.0));
  fc.c2 = d2(-sg * k2 * h4 / 180.0);
  const size_t total = size_t(nterms) * (1 + 5 * (size_t(fc.n1) + fc.n2));
  hipError_t e = hipSuccess;
  if (total * sizeof(double2) > P->sep_bytes) {
    (void)hipFree(P->d_sep);
    P->d_sep = nullptr;
    P->sep_bytes = 0;
    e = hipMalloc(&P->d_sep, total * sizeof(double2));
    if (e != hipSuccess) return e;
    P->sep_bytes = total * sizeof(double2);
  }
  double2* base = static_cast<double2*>(P->d_sep);
  double2* d1 = base + nterms;
  double2* dt2 = d1 + size_t(nterms) * 5 * fc.n1;
  e = hipMemcpyAsync(base, coef, size_t(nterms) * sizeof(double2), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d1, t1, size_t(nterms) * 5 * fc.n1 * sizeof(double2), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dt2, t2, size_t(nterms) * 5 * fc.n2 * sizeof(double2), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  const unsigned nb = unsigned((size_t(fc.n1) * fc.n2 + 255) / 256);
  hipLaunchKernelGGL(neumann_data_kernel, dim3(nb), dim3(256), 0, s, fc, nterms, base, d1, dt2, F);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace h6
