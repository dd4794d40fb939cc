// C ABI of the helmholtz6 library: parameter validation, plan construction
// (coefficients of Section 3.1-3.3), workspace, status strings and timing.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <thread>
#include <new>

#include "h6_internal.h"
#include "h6net.h"

namespace h6 {

const char* const kKernelClassNames[KC_COUNT] = {
    "stencil", "stencil_resid", "xform_x", "xform_y", "tridiag_z", "mgs_dots", "mgs_update",
    "norm", "axpy", "rhs"};

namespace {

std::string g_setup_error;
std::mutex g_setup_mutex;

W9 to_w9(cplx alpha, cplx beta, cplx gamma) {
  cplx c = alpha - 4.0 * beta + 4.0 * gamma, e = beta - 2.0 * gamma, k = gamma;
  return W9{make_double2(c.real(), c.imag()), make_double2(e.real(), e.imag()),
            make_double2(k.real(), k.imag())};
}

W9 w9_lin(const W9& a, double sa, const W9& b, double sb) {
  auto f = [&](double2 x, double2 y) {
    return make_double2(sa * x.x + sb * y.x, sa * x.y + sb * y.y);
  };
  return W9{f(a.c, b.c), f(a.e, b.e), f(a.k, b.k)};
}

const W9 kZeroW9{make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};

// Stencil weights.  With D_a = h^2 delta_a^2 and kappa = (kh)^2, eq. (scheme)
// times h^2 is D_z G + P with
//   G = I + a (D_x + D_y) + (1/30) D_x D_y,            a = (1 + kappa/30) / 6,
//   P = D_x + D_y + a D_x D_y + kappa c_K I,           c_K = 1 - kappa/12 + kappa^2/360,
// so an interior row is G U_{l-1} + (P - 2G) U_l + G U_{l+1}.  A closure row
// replaces G U_ghost by G U_1 (Neumann, eq. (3DN)) or by Q U_1 + R U_0
// (Sommerfeld, eq. (3DDISCS)).
void build_stencil(h6_plan P) {
  const cplx I(0.0, 1.0);
  const cplx kap = P->kappa;
  const cplx kh = P->k * P->p.h;
  const cplx ikh = I * kh;
  const cplx a = (1.0 + kap / 30.0) / 6.0;
  const cplx cK = 1.0 - kap / 12.0 + kap * kap / 360.0;
  const W9 G = to_w9(1.0, a, 1.0 / 30.0);
  const W9 Pw = to_w9(kap * cK, 1.0, a);
  const W9 Pm2G = w9_lin(Pw, 1.0, G, -2.0);

  // Section 3.2.2: mu_3, mu_1 chosen to match the interior scheme.
  const cplx mu3 = 1.0 / (1.0 + (2.0 * ikh / 3.0) * (1.0 + 2.0 * kap / 15.0));
  const cplx mu1 = (ikh / 90.0 + (1.0 + kap / 30.0) / (6.0 * mu3)) / (1.0 + 2.0 * ikh / 3.0);
  const cplx q = std::exp(2.0 * ikh) * mu3;
  const W9 Q = to_w9(q * (1.0 - 2.0 * ikh / 3.0 - 4.0 * I * kh * kh * kh / 45.0),
                     q * (mu1 + (2.0 * ikh / 3.0) * (1.0 / 60.0 - mu1)), q / (30.0 * mu3));
  const cplx r = std::exp(ikh) * mu3;
  const W9 R = to_w9(r * (4.0 * ikh / 3.0) * (1.0 + 2.0 * kap / 15.0),
                     -r * (4.0 * ikh / 3.0) * (1.0 / 60.0 - mu1), 0.0);

  StencilTable& T = P->stencil;
  T.w[0][0] = G;
  T.w[0][1] = Pm2G;
  T.w[0][2] = G;
  const int lo = P->p.bc[4], hi = P->p.bc[5];
  // low-z closure row: ghost plane (offset -1) eliminated
  T.w[1][0] = kZeroW9;
  if (lo == H6_SOMMERFELD) {
    T.w[1][1] = w9_lin(Pm2G, 1.0, R, 1.0);
    T.w[1][2] = w9_lin(G, 1.0, Q, 1.0);
  } else {
    T.w[1][1] = Pm2G;
    T.w[1][2] = w9_lin(G, 2.0, G, 0.0);
  }
  // high-z closure row: ghost plane (offset +1) eliminated
  T.w[2][2] = kZeroW9;
  if (hi == H6_SOMMERFELD) {
    T.w[2][1] = w9_lin(Pm2G, 1.0, R, 1.0);
    T.w[2][0] = w9_lin(G, 1.0, Q, 1.0);
  } else {
    T.w[2][1] = Pm2G;
    T.w[2][0] = w9_lin(G, 2.0, G, 0.0);
  }
}

// lambda(m) = -4 sin^2(pi m / (2M)); modes m = 1..n (Dirichlet) or 0..M (Neumann).
std::vector<double> mode_lambdas(const AxisXform& a) {
  std::vector<double> l(a.L);
  for (int i = 0; i < a.L; ++i) {
    const int m = a.neumann ? i : i + 1;
    const double s = std::sin(M_PI * m / (2.0 * a.M));
    l[i] = -4.0 * s * s;
  }
  return l;
}

// Basis matrices of the dense transforms of one axis (xform_dense.hip), in
// the compute precision R, folded by their reflection symmetry: for the
// forward then the inverse matrix W, We[j][p] = W[2j][p] (p < ceil(L/2)) and
// Wo[j][p] = W[2j+1][p] (p < floor(L/2)), each [Hm][Hk] row-major and
// zero-padded (Hm a multiple of 32, Hk of kDenseKChunk).  Inverse: W_mq = sin(pi (q+1)(m+1) / M) (sine basis) or
// cos(pi q m / M) (cosine basis); forward W^{-1} = (2/M) W (sine) or
// (2/M) C W C, C = diag(1/2, 1, .., 1, 1/2) (cosine).  Angles are reduced
// modulo 2M in integers.
template <typename T>
hipError_t upload(T** dst, const std::vector<T>& v, hipStream_t s);

template <typename R>
hipError_t build_dense(AxisXform& ax, hipStream_t s) {
  const int L = ax.L, M = ax.M, h = L / 2, H = L - h;
  ax.Hm = (H + 31) / 32 * 32;
  ax.Hk = (H + kDenseKChunk - 1) / kDenseKChunk * kDenseKChunk;
  const size_t one = size_t(ax.Hm) * ax.Hk;
  std::vector<R> hv(4 * one, R(0));     // [direction][parity][Hm][Hk]
  for (int m = 0; m < L; ++m)
    for (int q = 0; q < ((m & 1) ? h : H); ++q) {
      double inv, fwd;
      if (!ax.neumann) {
        const long long t = (long long)(q + 1) * (m + 1) % (2 * M);
        inv = std::sin(M_PI * double(t) / M);
        fwd = (2.0 / M) * inv;
      } else {
        const long long t = (long long)q * m % (2 * M);
        inv = std::cos(M_PI * double(t) / M);
        const double cq = (q == 0 || q == L - 1) ? 0.5 : 1.0, sm = (m == 0 || m == L - 1) ? 0.5 : 1.0;
        fwd = (2.0 / M) * sm * cq * inv;
      }
      const size_t at = size_t(m & 1) * one + size_t(m >> 1) * ax.Hk + q;
      hv[at] = R(fwd);
      hv[2 * one + at] = R(inv);
    }
  R* d = nullptr;
  const hipError_t e = upload(&d, hv, s);
  ax.wmat = d;
  return e;
}

// T_z of eq. (3DAP): tridiag(1, -2, 1), corner entry 2 next to a Neumann or
// Sommerfeld face (beta_z = 1), diagonal + 2ikh on a Sommerfeld face.
void z_tridiagonal(h6_plan P, std::vector<cplx>& sub, std::vector<cplx>& diag,
                   std::vector<cplx>& sup) {
  const int L = P->dims[2];
  sub.assign(L, 1.0);
  sup.assign(L, 1.0);
  diag.assign(L, -2.0);
  sub[0] = 0.0;
  sup[L - 1] = 0.0;
  const cplx alpha = cplx(0.0, 2.0) * P->k * P->p.h;
  if (P->p.bc[4] != H6_DIRICHLET && L > 1) {
    sup[0] = 2.0;
    if (P->p.bc[4] == H6_SOMMERFELD) diag[0] += alpha;
  }
  if (P->p.bc[5] != H6_DIRICHLET && L > 1) {
    sub[L - 1] = 2.0;
    if (P->p.bc[5] == H6_SOMMERFELD) diag[L - 1] += alpha;
  }
}

// Gaussian elimination of every z system T_z + (kappa + lx + ly) I: a pivot
// below 1e-12 (4 + |shift|) or non-finite means A_p is singular.  Records
// c'_{r0-1}, the value entering each of the kZSegs segments of rows
// [r0, r0 + S), S = ceil(n'z / kZSegs), for the partitioned device solver.
bool factor_modes(h6_plan P, const std::vector<double>& lx, const std::vector<double>& ly,
                  const std::vector<cplx>& sub, const std::vector<cplx>& diag,
                  const std::vector<cplx>& sup, std::vector<cplx>& cstart, std::string& where) {
  const int L = P->dims[2];
  const size_t nmodes = lx.size() * ly.size();
  const int segs = z_segments(L, P->p.precision == H6_MIXED);
  const int S = (L + segs - 1) / segs;
  cstart.assign(size_t(segs) * nmodes, cplx(0.0));
  for (size_t j = 0; j < ly.size(); ++j)
    for (size_t i = 0; i < lx.size(); ++i) {
      const size_t mode = i + lx.size() * j;
      const cplx shift = P->kappa + lx[i] + ly[j];
      const double tol = 1e-12 * (4.0 + std::abs(shift));
      cplx cprev = 0.0;
      for (int l = 0; l < L; ++l) {
        if (l % S == 0) cstart[size_t(l / S) * nmodes + mode] = cprev;
        const cplx piv = diag[l] + shift - (l > 0 ? sub[l] * cprev : cplx(0.0));
        if (!std::isfinite(piv.real()) || !std::isfinite(piv.imag()) || std::abs(piv) <= tol) {
          where = "zero pivot in z row " + std::to_string(l) + " of mode (" + std::to_string(i) +
                  ", " + std::to_string(j) + ")";
          return true;
        }
        cprev = sup[l] / piv;
      }
    }
  return false;
}

// Tables of the Bluestein path (xform_bluestein.hip) for odd M <= 255:
// c_q = exp(-i pi q^2 / M) (q^2 taken mod 2M, the period of c), the spectrum
// FFT_P(b) / P of b_j = conj(c_j) for |j| < M laid out cyclically (computed as
// a plain DFT in long double), the FFT twiddles and sin / cos(pi q / M), in
// double and in single precision, in one device allocation.
hipError_t build_bluestein(AxisXform& ax, hipStream_t s) {
  const int M = ax.M, P = bluestein_length(M);
  std::vector<double2> chirp(M), bhat(P), tw(P);
  std::vector<double> sq(M), cq(M);
  std::vector<std::complex<long double>> b(P, 0.0L);
  for (int q = 0; q < M; ++q) {
    const long double ang = -M_PIl * (long double)((long long)q * q % (2LL * M)) / M;
    chirp[q] = make_double2(double(cosl(ang)), double(sinl(ang)));
    const std::complex<long double> bj(cosl(ang), -sinl(ang));      // conj(c_q)
    b[q] = bj;
    if (q > 0) b[P - q] = bj;
    sq[q] = std::sin(M_PI * q / M);
    cq[q] = std::cos(M_PI * q / M);
  }
  // FFT_P(b) as a plain DFT over the nonzero b_j (j < M and j > P - M), with
  // exp(-2 pi i t / P) tabulated once (t = j k mod P)
  std::vector<std::complex<long double>> wp(P);
  for (int t = 0; t < P; ++t) {
    const long double ang = -2.0L * M_PIl * (long double)t / P;
    wp[t] = std::complex<long double>(cosl(ang), sinl(ang));
  }
  std::vector<int> nz;
  for (int j = 0; j < P; ++j)
    if (b[j] != std::complex<long double>(0.0L)) nz.push_back(j);
  for (int k = 0; k < P; ++k) {
    std::complex<long double> acc = 0.0L;
    for (int j : nz) acc += b[j] * wp[(long long)j * k % P];
    bhat[k] = make_double2(double(acc.real() / P), double(acc.imag() / P));
  }
  for (int t = 0; t < P; ++t)
    tw[t] = make_double2(std::cos(-2.0 * M_PI * t / P), std::sin(-2.0 * M_PI * t / P));
  // layout (16-byte aligned pieces)
  auto al = [](size_t x) { return (x + 15) / 16 * 16; };
  const size_t o_ch = 0, o_bh = o_ch + al(M * sizeof(double2)), o_tw = o_bh + al(P * sizeof(double2));
  const size_t o_s = o_tw + al(P * sizeof(double2)), o_c = o_s + al(M * sizeof(double));
  const size_t o_chf = o_c + al(M * sizeof(double)), o_bhf = o_chf + al(M * sizeof(float2));
  const size_t o_twf = o_bhf + al(P * sizeof(float2)), o_sf = o_twf + al(P * sizeof(float2));
  const size_t o_cf = o_sf + al(M * sizeof(float)), bytes = o_cf + al(M * sizeof(float));
  std::vector<char> host(bytes, 0);
  auto put = [&](size_t off, const void* src, size_t n) { std::memcpy(host.data() + off, src, n); };
  std::vector<float2> chf(M), bhf(P), twf(P);
  std::vector<float> sf(M), cf(M);
  for (int q = 0; q < M; ++q) {
    chf[q] = make_float2(float(chirp[q].x), float(chirp[q].y));
    sf[q] = float(sq[q]);
    cf[q] = float(cq[q]);
  }
  for (int k = 0; k < P; ++k) {
    bhf[k] = make_float2(float(bhat[k].x), float(bhat[k].y));
    twf[k] = make_float2(float(tw[k].x), float(tw[k].y));
  }
  put(o_ch, chirp.data(), M * sizeof(double2));
  put(o_bh, bhat.data(), P * sizeof(double2));
  put(o_tw, tw.data(), P * sizeof(double2));
  put(o_s, sq.data(), M * sizeof(double));
  put(o_c, cq.data(), M * sizeof(double));
  put(o_chf, chf.data(), M * sizeof(float2));
  put(o_bhf, bhf.data(), P * sizeof(float2));
  put(o_twf, twf.data(), P * sizeof(float2));
  put(o_sf, sf.data(), M * sizeof(float));
  put(o_cf, cf.data(), M * sizeof(float));
  char* mem = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&mem), bytes);
  if (e != hipSuccess) return e;
  ax.blue_mem = mem;
  e = hipMemcpyAsync(mem, host.data(), bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  BluesteinTables& t = ax.blue;
  t.M = M;
  t.P = P;
  t.chirp = reinterpret_cast<const double2*>(mem + o_ch);
  t.bhat = reinterpret_cast<const double2*>(mem + o_bh);
  t.tw = reinterpret_cast<const double2*>(mem + o_tw);
  t.sin_q = reinterpret_cast<const double*>(mem + o_s);
  t.cos_q = reinterpret_cast<const double*>(mem + o_c);
  t.chirp_f = reinterpret_cast<const float2*>(mem + o_chf);
  t.bhat_f = reinterpret_cast<const float2*>(mem + o_bhf);
  t.tw_f = reinterpret_cast<const float2*>(mem + o_twf);
  t.sin_f = reinterpret_cast<const float*>(mem + o_sf);
  t.cos_f = reinterpret_cast<const float*>(mem + o_cf);
  return e;
}

// Tables of the Rader path for a prime M with M - 1 = 256 (xform_rader.hip).
hipError_t build_rader(AxisXform& ax, hipStream_t s) {
  const int M = ax.M, P1 = M - 1;
  auto powmod = [M](long long b, long long e) {
    long long r = 1;
    b %= M;
    while (e > 0) {
      if (e & 1) r = r * b % M;
      b = b * b % M;
      e >>= 1;
    }
    return int(r);
  };
  int g = 2;                                   // primitive root: g^((M-1)/2) != 1 (M-1 = 2^8)
  while (powmod(g, P1 / 2) == 1) ++g;
  const int ginv = powmod(g, M - 2);
  std::vector<int> pin(P1), pout(P1);
  for (int a = 0; a < P1; ++a) {
    pin[a] = powmod(ginv, a);
    pout[a] = powmod(g, a);
  }
  std::vector<double2> kf(P1), tw(256);
  for (int k = 0; k < P1; ++k) {
    long double re = 0.0L, im = 0.0L;
    for (int c = 0; c < P1; ++c) {
      // K[c] = exp(-2 pi i g^c / M), times exp(-2 pi i c k / (M-1))
      const long double ang = -2.0L * M_PIl * ((long double)pout[c] / M + (long double)((c * (long long)k) % P1) / P1);
      re += cosl(ang);
      im += sinl(ang);
    }
    kf[k] = make_double2(double(re / P1), double(im / P1));
  }
  for (int t = 0; t < 256; ++t)
    tw[t] = make_double2(std::cos(-2.0 * M_PI * t / 256.0), std::sin(-2.0 * M_PI * t / 256.0));
  std::vector<double> sa(P1), ca(P1);
  std::vector<int> slot_of_q(M + 1, -1);
  for (int a = 0; a < P1; ++a) {
    sa[a] = std::sin(M_PI * pin[a] / M);
    ca[a] = std::cos(M_PI * pin[a] / M);
    slot_of_q[pin[a]] = a;
  }
  slot_of_q[0] = P1;          // cosine-basis end nodes
  slot_of_q[M] = P1 + 1;
  std::vector<int> slot_d(M - 1), slot_n(M + 1);
  for (int p = 0; p < M - 1; ++p) slot_d[p] = slot_of_q[p + 1];
  for (int p = 0; p <= M; ++p) slot_n[p] = slot_of_q[p];
  std::vector<float2> kff(P1), twf(256);
  std::vector<float> saf(P1), caf(P1);
  for (int k = 0; k < P1; ++k) kff[k] = make_float2(float(kf[k].x), float(kf[k].y));
  for (int t = 0; t < 256; ++t) twf[t] = make_float2(float(tw[t].x), float(tw[t].y));
  for (int a = 0; a < P1; ++a) {
    saf[a] = float(sa[a]);
    caf[a] = float(ca[a]);
  }
  const size_t bytes = 2 * P1 * sizeof(int) + 2 * P1 * sizeof(double2) + 2 * P1 * sizeof(double) +
                       (2 * M + 1) * sizeof(int) + 2 * P1 * sizeof(float2) + 2 * P1 * sizeof(float) +
                       16 * 16;
  char* mem = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&mem), bytes + 64);
  if (e != hipSuccess) return e;
  ax.rader_mem = mem;
  std::vector<char> host(bytes + 64, 0);
  size_t off = 0;
  auto put = [&](const void* src, size_t n) {
    off = (off + 15) & ~size_t(15);
    std::memcpy(host.data() + off, src, n);
    const size_t at = off;
    off += n;
    return mem + at;
  };
  ax.rader.kf = reinterpret_cast<const double2*>(put(kf.data(), P1 * sizeof(double2)));
  ax.rader.tw256 = reinterpret_cast<const double2*>(put(tw.data(), 256 * sizeof(double2)));
  ax.rader.sin_a = reinterpret_cast<const double*>(put(sa.data(), P1 * sizeof(double)));
  ax.rader.cos_a = reinterpret_cast<const double*>(put(ca.data(), P1 * sizeof(double)));
  ax.rader.slot_d = reinterpret_cast<const int*>(put(slot_d.data(), (M - 1) * sizeof(int)));
  ax.rader.slot_n = reinterpret_cast<const int*>(put(slot_n.data(), (M + 1) * sizeof(int)));
  ax.rader.perm_in = reinterpret_cast<const int*>(put(pin.data(), P1 * sizeof(int)));
  ax.rader.perm_out = reinterpret_cast<const int*>(put(pout.data(), P1 * sizeof(int)));
  ax.rader.kf_f = reinterpret_cast<const float2*>(put(kff.data(), P1 * sizeof(float2)));
  ax.rader.tw_f = reinterpret_cast<const float2*>(put(twf.data(), 256 * sizeof(float2)));
  ax.rader.sin_f = reinterpret_cast<const float*>(put(saf.data(), P1 * sizeof(float)));
  ax.rader.cos_f = reinterpret_cast<const float*>(put(caf.data(), P1 * sizeof(float)));
  if (off > bytes + 64) return hipErrorInvalidValue;
  e = hipMemcpyAsync(mem, host.data(), off, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  ax.fast = 1;
  return hipStreamSynchronize(s);
}

void free_plan(h6_plan P) {
  if (!P) return;
  release_graphs(P);
  (void)hipFree(P->d_givens);
  if (P->gstream) (void)hipStreamDestroy(P->gstream);
  if (P->ev_order) (void)hipEventDestroy(P->ev_order);
  for (auto& a : P->ax) (void)hipFree(a.rader_mem);
  for (auto& a : P->ax) (void)hipFree(a.blue_mem);
  (void)hipFree(P->d_stencil);
  (void)hipFree(P->d_lambda_x);
  (void)hipFree(P->d_lambda_y);
  for (auto& a : P->ax) (void)hipFree(a.wmat);
  (void)hipFree(P->d_cstart);
  (void)hipFree(P->d_zparams);
  for (void* w : P->w_pc) (void)hipFree(w);
  (void)hipFree(P->V);
  (void)hipFree(P->Z);
  (void)hipFree(P->r);
  (void)hipFree(P->t);
  (void)hipFree(P->partials);
  (void)hipFree(P->d_scal);
  (void)hipFree(P->d_gram);
  (void)hipFree(P->d_sep);
  if (P->ev_sync) (void)hipEventDestroy(P->ev_sync);
  if (P->h_pinned) (void)hipHostFree(P->h_pinned);
  if (P->h_parts) (void)hipHostFree(P->h_parts);
  if (P->h_step) (void)hipHostFree(P->h_step);
  for (hipEvent_t e : P->timing.pool) (void)hipEventDestroy(e);
  for (auto& pe : P->timing.pending) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  delete P;
}

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& v, hipStream_t s) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

h6_status setup_impl(const h6_params* p, hipStream_t s, h6_plan* out, std::string& err) {
  *out = nullptr;
  if (!p) { err = "params is NULL"; return H6_ERR_ARG; }
  for (int a = 0; a < 3; ++a)
    if (p->n[a] < 1 || p->n[a] > 100000) { err = "n[a] must be in 1..100000"; return H6_ERR_ARG; }
  if (!(p->h > 0.0) || !std::isfinite(p->h)) { err = "h must be positive and finite"; return H6_ERR_ARG; }
  if (!std::isfinite(p->k_re) || !std::isfinite(p->k_im)) { err = "k must be finite"; return H6_ERR_ARG; }
  for (int f = 0; f < 6; ++f)
    if (p->bc[f] < H6_DIRICHLET || p->bc[f] > H6_SOMMERFELD) { err = "bad bc code"; return H6_ERR_ARG; }
  if (p->precision != H6_FP64 && p->precision != H6_MIXED) { err = "bad precision"; return H6_ERR_ARG; }
  for (int a = 0; a < 2; ++a) {
    if (p->bc[2 * a] == H6_SOMMERFELD || p->bc[2 * a + 1] == H6_SOMMERFELD) {
      err = "Sommerfeld faces are supported on z only";
      return H6_ERR_UNSUPPORTED_BC;
    }
    if (p->bc[2 * a] != p->bc[2 * a + 1]) {
      err = "x and y faces must be a Dirichlet or a Neumann pair";
      return H6_ERR_UNSUPPORTED_BC;
    }
  }
  h6_plan P = new (std::nothrow) h6_plan_s();
  if (!P) { err = "host allocation failed"; return H6_ERR_ALLOC; }
  P->p = *p;
  for (int a = 0; a < 3; ++a)
    P->dims[a] = p->n[a] + (p->bc[2 * a] != H6_DIRICHLET) + (p->bc[2 * a + 1] != H6_DIRICHLET);
  P->N = size_t(P->dims[0]) * P->dims[1] * P->dims[2];
  if (P->dims[2] > kMaxZ) {
    err = "n'z = " + std::to_string(P->dims[2]) + " exceeds the z-solver limit of " + std::to_string(kMaxZ);
    free_plan(P);
    return H6_ERR_ARG;
  }
  if (P->N > (size_t(1) << 31)) { err = "grid too large"; free_plan(P); return H6_ERR_ARG; }
  P->xmirror = p->bc[0] == H6_NEUMANN;
  P->ymirror = p->bc[2] == H6_NEUMANN;
  P->zlo_closure = p->bc[4] != H6_DIRICHLET;
  P->zhi_closure = p->bc[5] != H6_DIRICHLET;
  P->k = cplx(p->k_re, p->k_im);
  P->kappa = (P->k * p->h) * (P->k * p->h);
  build_stencil(P);
  for (int a = 0; a < 2; ++a) {
    P->ax[a].L = P->dims[a];
    P->ax[a].M = p->n[a] + 1;
    P->ax[a].neumann = p->bc[2 * a] == H6_NEUMANN;
    if (P->ax[a].L > kMaxLine) {
      err = std::string("n'") + (a == 0 ? "x" : "y") + " = " + std::to_string(P->ax[a].L) +
            " exceeds the transform limit of " + std::to_string(kMaxLine);
      free_plan(P);
      return H6_ERR_ARG;
    }
  }
  std::vector<double> lx = mode_lambdas(P->ax[0]), ly = mode_lambdas(P->ax[1]);
  std::vector<cplx> sub, diag, sup;
  z_tridiagonal(P, sub, diag, sup);
  std::string where;
  std::vector<cplx> cstart;
  if (factor_modes(P, lx, ly, sub, diag, sup, cstart, where)) {
    err = "preconditioner is singular: " + where;
    free_plan(P);
    return H6_ERR_SINGULAR;
  }
  for (int l = 0; l < P->dims[2]; ++l)      // the device z solver takes the off-diagonals as real
    if (sub[l].imag() != 0.0 || sup[l].imag() != 0.0) {
      err = "internal: complex z off-diagonal";
      free_plan(P);
      return H6_ERR_ARG;
    }
  {
    const int L = P->dims[2];
    for (int l = 0; l < L; ++l)           // inner rows are (1, -2, 1)
      if ((l > 0 && l < L - 1) && (sub[l] != 1.0 || sup[l] != 1.0 || diag[l] != -2.0)) {
        err = "internal: z tridiagonal inner row";
        free_plan(P);
        return H6_ERR_ARG;
      }
    const double o0 = L > 1 ? sup[0].real() : 1.0, ol = L > 1 ? sub[L - 1].real() : 1.0;
    P->zends = ZEnds{diag[0].real(), diag[0].imag(), 1.0 / o0, diag[L - 1].real(), diag[L - 1].imag(), 1.0 / ol};
  }
  hipError_t e = hipSuccess;
  std::vector<StencilTable> st(1, P->stencil);
  if (e == hipSuccess) e = upload(&P->d_stencil, st, s);
  {
    const ZEnds& z = P->zends;
    std::vector<double> zp = {P->kappa.real(), P->kappa.imag(), z.b0_re, z.b0_im, z.s0, z.bl_re, z.bl_im, z.sl};
    static_assert(kZParams == 8, "z-solver parameter block");
    if (e == hipSuccess) e = upload(&P->d_zparams, zp, s);
  }
  if (e == hipSuccess) e = upload(&P->d_lambda_x, lx, s);
  if (e == hipSuccess) e = upload(&P->d_lambda_y, ly, s);
  for (int a = 0; a < 2 && e == hipSuccess; ++a)
    e = p->precision == H6_MIXED ? build_dense<float>(P->ax[a], s) : build_dense<double>(P->ax[a], s);
  if (e == hipSuccess) {
    if (p->precision == H6_MIXED) {
      std::vector<float2> cf(cstart.size());
      for (size_t i = 0; i < cf.size(); ++i) cf[i] = make_float2(float(cstart[i].real()), float(cstart[i].imag()));
      e = upload(reinterpret_cast<float2**>(&P->d_cstart), cf, s);
    } else {
      std::vector<double2> cd(cstart.size());
      for (size_t i = 0; i < cd.size(); ++i) cd[i] = make_double2(cstart[i].real(), cstart[i].imag());
      e = upload(reinterpret_cast<double2**>(&P->d_cstart), cd, s);
    }
  }
  for (int a = 0; a < 2 && e == hipSuccess; ++a) {
    if (P->ax[a].M == kRaderM && !std::getenv("H6_DENSE_TRANSFORMS")) e = build_rader(P->ax[a], s);
    else if (bluestein_ok(P->ax[a].M) && P->ax[a].L <= 256 && !std::getenv("H6_DENSE_TRANSFORMS")) {
      e = build_bluestein(P->ax[a], s);
      // untuned default: the chirp-z path where its FFT length is nearly all
      // signal (2M - 2 >= 15/16 P; measured faster there), else the dense
      // product; the autotuner times both
      const int M = P->ax[a].M;
      if (e == hipSuccess && 16 * (2 * M - 2) >= 15 * bluestein_length(M)) P->ax[a].fast = 2;
    }
    P->ax[a].lines = a == 0 ? 4 : 16;     // untuned default: best on gfx950 at 256^3
  }
  const size_t elem = p->precision == H6_MIXED ? sizeof(float2) : sizeof(double2);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipMalloc(&P->w_pc[i], P->N * elem);
  if (e == hipSuccess) e = hipMalloc(&P->partials, sizeof(double) * 2 * kMaxPartials);
  if (e == hipSuccess) e = hipMalloc(&P->d_scal, sizeof(double2) * kScal);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&P->h_pinned), sizeof(double2) * kScal);
  if (e == hipSuccess) {
    // device address of the fixed work space of helmholtz6_apply_Pinv_noalloc
    // on this device (looked up once per device)
    void* ws = nullptr;
    e = static_work_address(&ws);
  }
  if (e != hipSuccess) {
    err = std::string("device setup failed: ") + hipGetErrorString(e);
    const bool oom = e == hipErrorOutOfMemory;
    free_plan(P);
    return oom ? H6_ERR_ALLOC : H6_ERR_HIP;
  }
  *out = P;
  return H6_OK;
}

}  // namespace

void timing_begin(h6_plan P, int cls, hipStream_t s, hipEvent_t* a) {
  (void)cls;
  *a = nullptr;
  if (!P->timing.enabled) return;
  if (P->timing.pool.empty()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return;
    P->timing.pool.push_back(ev);
  }
  *a = P->timing.pool.back();
  P->timing.pool.pop_back();
  (void)hipEventRecord(*a, s);
}

void timing_end(h6_plan P, int cls, hipStream_t s, hipEvent_t a, double bytes) {
  if (!P->timing.enabled || !a) return;
  hipEvent_t b;
  if (P->timing.pool.empty()) {
    if (hipEventCreate(&b) != hipSuccess) { P->timing.pool.push_back(a); return; }
  } else {
    b = P->timing.pool.back();
    P->timing.pool.pop_back();
  }
  (void)hipEventRecord(b, s);
  P->timing.pending.push_back({a, b, cls, bytes});
}

}  // namespace h6

using namespace h6;

namespace h6 {

// Extreme eigenvalues of A A_p^{-1} over all Dirichlet sine modes: with
// mu_a = -4 sin^2(m pi / (2 M_a)) the eigenvalues of D_a, A = D_z G + P has
//   lambda = mu_z (1 + a (mu_x + mu_y) + mu_x mu_y / 30) + mu_x + mu_y + a mu_x mu_y + kappa c_K
// (a = (1 + kappa/30)/6, c_K = 1 - kappa/12 + kappa^2/360; eq. (3DEGV)) and
// A_p has lambda^p = mu_x + mu_y + mu_z + kappa.
h6_status spectrum_bounds(h6_plan P) {
  if (P->spec_done) return P->spec_status;
  P->spec_done = true;
  P->spec_status = H6_ERR_ARG;
  for (int f = 0; f < 6; ++f)
    if (P->p.bc[f] != H6_DIRICHLET) {
      P->last_error = "spectrum bounds need Dirichlet faces";
      return P->spec_status;
    }
  if (P->p.k_im != 0.0) {
    P->last_error = "spectrum bounds need a real k";
    return P->spec_status;
  }
  const double kap = P->kappa.real();
  const double a = (1.0 + kap / 30.0) / 6.0, cK = 1.0 - kap / 12.0 + kap * kap / 360.0;
  std::vector<double> mu[3];
  for (int ax = 0; ax < 3; ++ax) {
    const int n = P->dims[ax];
    for (int m = 1; m <= n; ++m) {
      const double s = std::sin(M_PI * m / (2.0 * (n + 1)));
      mu[ax].push_back(-4.0 * s * s);
    }
  }
  double lo = INFINITY, hi = -INFINITY;
  for (double mz : mu[2])
    for (double my : mu[1])
      for (double mx : mu[0]) {
        const double lam = mz * (1.0 + a * (mx + my) + mx * my / 30.0) + mx + my + a * mx * my + kap * cK;
        const double r = lam / (mx + my + mz + kap);
        lo = std::min(lo, r);
        hi = std::max(hi, r);
      }
  if (!std::isfinite(lo) || !std::isfinite(hi)) {
    P->last_error = "spectrum bounds are not finite (k^2 on the 7-point spectrum)";
    return P->spec_status;
  }
  P->spec_lo = lo;
  P->spec_hi = hi;
  P->spec_status = H6_OK;
  return H6_OK;
}

// Autotuner: time the kernel variants on the plan's grid and keep the fastest.
h6_status autotune(h6_plan P, const char* cache_path, hipStream_t s) {
  char devname[256] = "unknown";
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      std::snprintf(devname, sizeof devname, "%s", prop.gcnArchName);
  }
  char key[512];
  std::snprintf(key, sizeof key, "h6tune3 %s %d %d %d %d", devname, P->dims[0], P->dims[1], P->dims[2],
                P->p.precision);
  const bool can_x = P->ax[0].rader_mem != nullptr, can_y = P->ax[1].rader_mem != nullptr;
  // transform variant code of the cache (0 dense, 1 Rader, 2 Bluestein) -> the variants this plan has
  auto fast_code = [&](int ax, int code) {
    if (code == 1 && P->ax[ax].rader_mem) return 1;
    if (code == 2 && P->ax[ax].blue_mem) return 2;
    return 0;
  };
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[600];
      while (std::fgets(line, sizeof line, f)) {
        int tz = 0, xf = 0, yf = 0, xl = 0, yl = 0;
        const size_t kl = std::strlen(key);
        if (std::strncmp(line, key, kl) == 0 && line[kl] == ' ' &&
            std::sscanf(line + kl, " tz=%d xfast=%d yfast=%d xlines=%d ylines=%d", &tz, &xf, &yf, &xl,
                        &yl) == 5 &&
            (tz == 8 || tz == 16 || tz == 32) && rader_lines_ok(0, xl) && rader_lines_ok(1, yl)) {
          std::fclose(f);
          P->stencil_tz = tz;
          P->ax[0].fast = fast_code(0, xf);
          P->ax[1].fast = fast_code(1, yf);
          P->ax[0].lines = xl;
          P->ax[1].lines = yl;
          return H6_OK;
        }
      }
      std::fclose(f);
    }
  }
  void *a = nullptr, *b = nullptr;
  const size_t vb = P->N * sizeof(double2);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(a);
    (void)hipFree(b);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&a, vb) != hipSuccess || hipMalloc(&b, vb) != hipSuccess ||
      hipMemsetAsync(a, 0, vb, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    P->last_error = "autotune: workspace allocation failed";
    return H6_ERR_ALLOC;
  }
  const bool timing = P->timing.enabled;
  P->timing.enabled = false;
  auto time_it = [&](auto&& fn) -> double {     // best of 3 after a warm-up
    fn();
    double best = 1e30;
    for (int r = 0; r < 3; ++r) {
      (void)hipEventRecord(e0, s);
      fn();
      (void)hipEventRecord(e1, s);
      float ms = 0.f;
      if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
        best = std::min(best, double(ms));
    }
    return best;
  };
  const double2* x = static_cast<const double2*>(a);
  double2* y = static_cast<double2*>(b);
  int best_tz = 16;
  double best_ms = 1e30;
  for (int tz : {8, 16, 32}) {
    P->stencil_tz = tz;
    const double ms = time_it([&] { (void)launch_stencil(P, x, y, nullptr, nullptr, nullptr, s); });
    if (ms < best_ms) { best_ms = ms; best_tz = tz; }
  }
  P->stencil_tz = best_tz;
  // per transform axis: the Rader path at each supported workgroup width
  // against the dense sums, timed inside the whole A_p^{-1}
  for (int ax = 0; ax < 2; ++ax) {
    if (!(ax == 0 ? can_x : can_y)) continue;
    P->ax[ax].fast = 0;
    double best = time_it([&] { (void)launch_pinv(P, x, y, s); });
    int best_lines = 0;
    for (int lines : {4, 8, 16}) {
      if (!rader_lines_ok(ax, lines)) continue;
      P->ax[ax].fast = 1;
      P->ax[ax].lines = lines;
      const double ms = time_it([&] { (void)launch_pinv(P, x, y, s); });
      if (ms < best) { best = ms; best_lines = lines; }
    }
    P->ax[ax].fast = best_lines ? 1 : 0;
    P->ax[ax].lines = best_lines ? best_lines : (ax == 0 ? 4 : 16);
  }
  // the Bluestein path against the dense product (odd M <= 255)
  for (int ax = 0; ax < 2; ++ax) {
    if (!P->ax[ax].blue_mem) continue;
    P->ax[ax].fast = 0;
    const double dense = time_it([&] { (void)launch_pinv(P, x, y, s); });
    P->ax[ax].fast = 2;
    const double blue = time_it([&] { (void)launch_pinv(P, x, y, s); });
    P->ax[ax].fast = blue <= dense ? 2 : 0;
  }
  P->timing.enabled = timing;
  const hipError_t err = hipStreamSynchronize(s);
  cleanup();
  if (err != hipSuccess) {
    P->last_error = std::string("autotune: ") + hipGetErrorString(err);
    return H6_ERR_HIP;
  }
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s tz=%d xfast=%d yfast=%d xlines=%d ylines=%d\n", key, P->stencil_tz,
                   int(P->ax[0].fast), int(P->ax[1].fast), P->ax[0].lines, P->ax[1].lines);
      std::fclose(f);
    }
  }
  return H6_OK;
}

}  // namespace h6

extern "C" {

h6_status helmholtz6_setup(const h6_params* p, void* hip_stream, h6_plan* out) {
  if (!out) return H6_ERR_ARG;
  std::string err;
  h6_status st;
  try {
    st = setup_impl(p, static_cast<hipStream_t>(hip_stream), out, err);
  } catch (...) {
    st = H6_ERR_ALLOC;
    err = "exception during setup";
    *out = nullptr;
  }
  std::lock_guard<std::mutex> g(g_setup_mutex);
  g_setup_error = err;
  return st;
}

h6_status helmholtz6_dims(h6_plan P, int dims[3]) {
  if (!P || !dims) return H6_ERR_ARG;
  for (int a = 0; a < 3; ++a) dims[a] = P->dims[a];
  return H6_OK;
}

h6_status helmholtz6_apply_A(h6_plan P, const void* x, void* y, void* hip_stream) {
  if (!P) return H6_ERR_ARG;
  P->last_error.clear();
  if (!x || !y || x == y) { P->last_error = "x, y must be distinct non-null pointers"; return H6_ERR_ARG; }
  H6_TRY_HIP(launch_stencil(P, static_cast<const double2*>(x), static_cast<double2*>(y), nullptr,
                            nullptr, nullptr, static_cast<hipStream_t>(hip_stream)));
  return H6_OK;
}

h6_status helmholtz6_apply_Pinv(h6_plan P, const void* r, void* z, void* hip_stream) {
  if (!P) return H6_ERR_ARG;
  P->last_error.clear();
  if (!r || !z || r == z) { P->last_error = "r, z must be distinct non-null pointers"; return H6_ERR_ARG; }
  H6_TRY_HIP(launch_pinv(P, static_cast<const double2*>(r), static_cast<double2*>(z),
                         static_cast<hipStream_t>(hip_stream)));
  return H6_OK;
}

h6_status helmholtz6_apply_Pinv_noalloc(h6_plan P, const void* r, void* z, void* hip_stream) {
  if (!P) return H6_ERR_ARG;
  P->last_error.clear();
  if (!r || !z || r == z) { P->last_error = "r, z must be distinct non-null pointers"; return H6_ERR_ARG; }
  const size_t elem = P->p.precision == H6_MIXED ? sizeof(float2) : sizeof(double2);
  const size_t vec = (P->N * elem + 255) / 256 * 256;
  if (2 * vec > kStaticWorkBytes) {
    P->last_error = "apply_Pinv_noalloc: this grid needs " + std::to_string(2 * vec) +
                    " bytes of work space, more than the fixed " + std::to_string(kStaticWorkBytes) +
                    " bytes (use helmholtz6_apply_Pinv)";
    return H6_ERR_ARG;
  }
  void* base = nullptr;
  H6_TRY_HIP(static_work_address(&base));
  void* ws[2] = {base, static_cast<unsigned char*>(base) + vec};
  // no timing events here (creating one may allocate)
  const bool timed = P->timing.enabled;
  P->timing.enabled = false;
  const hipError_t e = launch_pinv_ws(P, static_cast<const double2*>(r), static_cast<double2*>(z), ws,
                                      static_cast<hipStream_t>(hip_stream));
  P->timing.enabled = timed;
  H6_TRY_HIP(e);
  return H6_OK;
}

h6_status helmholtz6_rhs_gaussians(h6_plan P, int nsrc, const double* centres, const double* amps,
                                   double sigma, void* F, void* hip_stream) {
  if (!P) return H6_ERR_ARG;
  P->last_error.clear();
  if (!F || nsrc < 0 || nsrc > 64 || (nsrc > 0 && (!centres || !amps)) || !(sigma > 0.0)) {
    P->last_error = "bad rhs arguments";
    return H6_ERR_ARG;
  }
  H6_TRY_HIP(launch_rhs(P, nsrc, centres, amps, sigma, static_cast<double2*>(F),
                        static_cast<hipStream_t>(hip_stream)));
  return H6_OK;
}

h6_status helmholtz6_rhs_separable(h6_plan P, int nterms, const double* coef, const double* tx,
                                   const double* ty, const double* tz, void* F, void* hip_stream) {
  if (!P) return H6_ERR_ARG;
  P->last_error.clear();
  if (!F || nterms < 0 || nterms > 1024 || (nterms > 0 && (!coef || !tx || !ty || !tz))) {
    P->last_error = "bad rhs_separable arguments";
    return H6_ERR_ARG;
  }
  if (nterms == 0) {
    H6_TRY_HIP(hipMemsetAsync(F, 0, P->N * sizeof(double2), static_cast<hipStream_t>(hip_stream)));
    return H6_OK;
  }
  const double* tab[3] = {tx, ty, tz};
  H6_TRY_HIP(launch_rhs_separable(P, nterms, coef, tab, static_cast<double2*>(F),
                                  static_cast<hipStream_t>(hip_stream)));
  return H6_OK;
}

h6_status helmholtz6_rhs_dirichlet_z(h6_plan P, int side, const void* g, void* F, void* hip_stream) {
  if (!P) return H6_ERR_ARG;
  P->last_error.clear();
  if (!g || !F || (side != 0 && side != 1)) {
    P->last_error = "bad rhs_dirichlet_z arguments";
    return H6_ERR_ARG;
  }
  if (P->p.bc[4 + side] != H6_DIRICHLET) {
    P->last_error = "Dirichlet data given for a z face that is not Dirichlet";
    return H6_ERR_ARG;
  }
  H6_TRY_HIP(launch_rhs_dirichlet_z(P, side, static_cast<const double2*>(g), static_cast<double2*>(F),
                                    static_cast<hipStream_t>(hip_stream)));
  return H6_OK;
}

h6_status helmholtz6_rhs_neumann(h6_plan P, int face, int nterms, const double* coef, const double* t1,
                                 const double* t2, void* F, void* hip_stream) {
  if (!P) return H6_ERR_ARG;
  P->last_error.clear();
  if (!F || face < 0 || face > 5 || nterms < 0 || nterms > 1024 || (nterms > 0 && (!coef || !t1 || !t2))) {
    P->last_error = "bad rhs_neumann arguments";
    return H6_ERR_ARG;
  }
  if (P->p.bc[face] != H6_NEUMANN) {
    P->last_error = "Neumann data given for a face that is not Neumann";
    return H6_ERR_ARG;
  }
  if (nterms == 0) return H6_OK;
  H6_TRY_HIP(launch_rhs_neumann(P, face, nterms, coef, t1, t2, static_cast<double2*>(F),
                                static_cast<hipStream_t>(hip_stream)));
  return H6_OK;
}

h6_status helmholtz6_solve(h6_plan P, const void* F, void* U, h6_solve_info* info,
                           void* hip_stream) {
  if (!P) return H6_ERR_ARG;
  P->last_error.clear();
  if (!F || !U || !info || F == U) { P->last_error = "bad solve arguments"; return H6_ERR_ARG; }
  const bool krylov = info->method == H6_GMRES || info->method == H6_FGMRES;
  if (info->method < H6_GMRES || info->method > H6_CHEBYSHEV || info->maxit < 1 || !(info->tol >= 0.0) ||
      (krylov && (info->restart < 1 || info->restart > 256)) ||
      (info->history_len < 0) || (info->history_len > 0 && !info->history)) {
    P->last_error = "bad solve info";
    return H6_ERR_ARG;
  }
  if (P->p.precision == H6_MIXED && info->method == H6_GMRES) {
    P->last_error = "mixed precision needs FGMRES or SKS (the preconditioner is inexact)";
    return H6_ERR_ARG;
  }
  try {
    return run_solve(P, static_cast<const double2*>(F), static_cast<double2*>(U), info,
                     static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    P->last_error = "exception during solve";
    return H6_ERR_ALLOC;
  }
}

h6_status helmholtz6_profile(h6_plan P, int enable) {
  if (!P) return H6_ERR_ARG;
  P->timing.enabled = enable != 0;
  return H6_OK;
}

h6_status helmholtz6_kernel_time(h6_plan P, const char* name, int reset, double* ms,
                                 long long* launches, double* bytes) {
  if (!P || !name) return H6_ERR_ARG;
  int cls = -1;
  for (int i = 0; i < KC_COUNT; ++i)
    if (std::strcmp(name, kKernelClassNames[i]) == 0) cls = i;
  if (cls < 0) { P->last_error = "unknown kernel class"; return H6_ERR_ARG; }
  for (auto& pe : P->timing.pending) {
    float t = 0.f;
    if (hipEventSynchronize(pe.b) == hipSuccess && hipEventElapsedTime(&t, pe.a, pe.b) == hipSuccess) {
      P->timing.ms[pe.cls] += t;
      P->timing.launches[pe.cls] += 1;
      P->timing.bytes[pe.cls] += pe.bytes;
    }
    P->timing.pool.push_back(pe.a);
    P->timing.pool.push_back(pe.b);
  }
  P->timing.pending.clear();
  if (ms) *ms = P->timing.ms[cls];
  if (launches) *launches = P->timing.launches[cls];
  if (bytes) *bytes = P->timing.bytes[cls];
  if (reset) {
    P->timing.ms[cls] = 0.0;
    P->timing.launches[cls] = 0;
    P->timing.bytes[cls] = 0.0;
  }
  return H6_OK;
}

void helmholtz6_destroy(h6_plan P) { free_plan(P); }

const char* helmholtz6_status_string(h6_status s) {
  switch (s) {
    case H6_OK: return "ok";
    case H6_NOT_CONVERGED: return "not converged (maxit reached)";
    case H6_DIVERGED: return "diverged";
    case H6_ERR_ARG: return "invalid argument";
    case H6_ERR_UNSUPPORTED_BC: return "unsupported boundary-condition pattern";
    case H6_ERR_ALLOC: return "allocation failed";
    case H6_ERR_HIP: return "HIP runtime error";
    case H6_ERR_SINGULAR: return "preconditioner singular (k^2 on the 7-point spectrum)";
  }
  return "unknown status";
}

h6_status helmholtz6_solve_batch(h6_plan* plans, const void* const* F, void* const* U,
                                 h6_solve_info* infos, h6_status* statuses, int count, int nstreams) {
  if (count < 0 || nstreams < 1 || nstreams > 16 || (count > 0 && (!plans || !F || !U || !infos || !statuses)))
    return H6_ERR_ARG;
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return H6_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return H6_ERR_ARG;
  }
  if (count == 0) return H6_OK;
  // longest first: unknowns times an iteration estimate growing with kh
  std::vector<int> order(count);
  std::vector<double> cost(count);
  for (int i = 0; i < count; ++i) {
    const double kh = std::abs(plans[i]->k) * plans[i]->p.h;
    cost[i] = double(plans[i]->N) * (1.0 + 40.0 * kh * kh);
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return H6_ERR_HIP;
  const int nt = std::min(nstreams, count);
  std::vector<hipStream_t> streams(nt, nullptr);
  for (int t = 0; t < nt; ++t)
    if (hipStreamCreateWithFlags(&streams[t], hipStreamNonBlocking) != hipSuccess) {
      for (int u = 0; u < t; ++u) (void)hipStreamDestroy(streams[u]);
      return H6_ERR_HIP;
    }
  std::atomic<int> next{0};
  auto worker = [&](int t) {
    (void)hipSetDevice(dev);
    for (int q = next.fetch_add(1); q < count; q = next.fetch_add(1)) {
      const int i = order[q];
      statuses[i] = helmholtz6_solve(plans[i], F[i], U[i], &infos[i], streams[t]);
    }
  };
  std::vector<std::thread> threads;
  for (int t = 1; t < nt; ++t) threads.emplace_back(worker, t);
  worker(0);
  for (auto& th : threads) th.join();
  for (auto s : streams) (void)hipStreamDestroy(s);
  for (int i = 0; i < count; ++i)
    if (statuses[i] < 0) return statuses[i];
  return H6_OK;
}

h6_status helmholtz6_queue_create(h6_plan* plans, int count, int restart, int lanes, h6_queue* out) {
  if (!out) return H6_ERR_ARG;
  *out = nullptr;
  if (!plans || count < 1 || lanes < 1 || lanes > 16) return H6_ERR_ARG;
  std::string err;
  h6_status st;
  try {
    st = queue_create(plans, count, restart, lanes, out, err);
  } catch (...) {
    st = H6_ERR_ALLOC;
    err = "exception while creating the queue";
  }
  if (st != H6_OK) {
    std::lock_guard<std::mutex> g(g_setup_mutex);
    g_setup_error = err;
  }
  return st;
}

h6_status helmholtz6_queue_solve(h6_queue Q, const void* const* F, void* const* U, h6_solve_info* infos,
                                 h6_status* statuses) {
  if (!Q) return H6_ERR_ARG;
  Q->last_error.clear();
  if (!F || !U || !infos || !statuses) {
    Q->last_error = "null array";
    return H6_ERR_ARG;
  }
  try {
    return queue_solve(Q, reinterpret_cast<const double2* const*>(F), reinterpret_cast<double2* const*>(U), infos,
                       statuses, Q->last_error);
  } catch (...) {
    Q->last_error = "exception in the queued solve";
    return H6_ERR_ALLOC;
  }
}

const char* helmholtz6_queue_last_error(h6_queue Q) {
  if (!Q) {
    std::lock_guard<std::mutex> g(g_setup_mutex);
    return g_setup_error.c_str();
  }
  return Q->last_error.c_str();
}

void helmholtz6_queue_destroy(h6_queue Q) { queue_destroy(Q); }

h6_status helmholtz6_solve_batch_queue(h6_plan* plans, const void* const* F, void* const* U,
                                       h6_solve_info* infos, h6_status* statuses, int count, int lanes) {
  if (!plans || !F || !U || !infos || !statuses || count < 0 || lanes < 1 || lanes > 16) return H6_ERR_ARG;
  if (count == 0) return H6_OK;
  for (int i = 0; i < count; ++i)
    if (!plans[i]) return H6_ERR_ARG;
  h6_queue Q = nullptr;
  h6_status st = helmholtz6_queue_create(plans, count, infos[0].restart, lanes, &Q);
  if (st != H6_OK) {
    plans[0]->last_error = helmholtz6_queue_last_error(nullptr);
    return st;
  }
  st = helmholtz6_queue_solve(Q, F, U, infos, statuses);
  if (st < 0) plans[0]->last_error = Q->last_error;
  helmholtz6_queue_destroy(Q);
  return st;
}

h6_status helmholtz6_set_graphs(h6_plan P, int enable) {
  if (!P) return H6_ERR_ARG;
  if (enable < 0 || enable > 2) {
    P->last_error = "set_graphs: mode must be 0, 1 or 2";
    return H6_ERR_ARG;
  }
  if (enable != P->use_graphs) release_graphs(P);
  P->use_graphs = enable;
  return H6_OK;
}

h6_status helmholtz6_autotune(h6_plan P, const char* cache_path, void* hip_stream) {
  if (!P) return H6_ERR_ARG;
  return autotune(P, cache_path, static_cast<hipStream_t>(hip_stream));
}

h6_status helmholtz6_spectrum_bounds(h6_plan P, double* lo, double* hi) {
  if (!P || !lo || !hi) return H6_ERR_ARG;
  const h6_status st = spectrum_bounds(P);
  if (st != H6_OK) return st;
  *lo = P->spec_lo;
  *hi = P->spec_hi;
  return H6_OK;
}

double helmholtz6_psi_order(double r1_h, double r2_h, double r1_gh, double r2_gh, double gamma) {
  if (!(r1_h > 0.0 && r2_h > 0.0 && r1_gh > 0.0 && r2_gh > 0.0 && gamma > 1.0)) return std::nan("");
  return (std::log(r2_gh / r1_gh) - std::log(r2_h / r1_h)) / std::log(gamma);
}

h6_status helmholtz6_attach_net(h6_plan P, h6_net net) {
  if (!P) return H6_ERR_ARG;
  if (net && !net_matches(net, P->dims)) {
    P->last_error = "network grid does not match the plan's dims";
    return H6_ERR_ARG;
  }
  P->net = net;
  return H6_OK;
}

h6_status helmholtz6_learned_steps(h6_plan P, int* steps) {
  if (!P || !steps) return H6_ERR_ARG;
  *steps = P->learned_steps;
  return H6_OK;
}

const char* helmholtz6_last_error(h6_plan P) {
  if (!P) {
    std::lock_guard<std::mutex> g(g_setup_mutex);
    return g_setup_error.c_str();
  }
  return P->last_error.c_str();
}

}  // extern "C"
