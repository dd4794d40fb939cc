// Device helpers of the line transforms (xform_rader.hip, xform_bluestein.hip):
// complex arithmetic on float2 / double2 and an in-register FFT of length 16.
#pragma once

#include <hip/hip_runtime.h>

namespace h6 {
namespace fftdev {

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

template <typename R>
__device__ __forceinline__ typename V2<R>::T mk2(R a, R b) {
  typename V2<R>::T v;
  v.x = a;
  v.y = b;
  return v;
}

template <typename D, typename S>
__device__ __forceinline__ D cv(S v) {
  D d;
  d.x = v.x;
  d.y = v.y;
  return d;
}

template <typename R>
__device__ __forceinline__ typename V2<R>::T add(typename V2<R>::T a, typename V2<R>::T b) { return mk2<R>(a.x + b.x, a.y + b.y); }
template <typename R>
__device__ __forceinline__ typename V2<R>::T sub(typename V2<R>::T a, typename V2<R>::T b) { return mk2<R>(a.x - b.x, a.y - b.y); }
template <typename R>
__device__ __forceinline__ typename V2<R>::T mul(typename V2<R>::T a, typename V2<R>::T b) {
  return mk2<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__device__ __forceinline__ typename V2<R>::T scl(typename V2<R>::T a, R s) { return mk2<R>(a.x * s, a.y * s); }

// radix-4 butterfly; forward uses w4 = -i, inverse w4 = +i
template <typename R, bool INV>
__device__ __forceinline__ void fft4(typename V2<R>::T& a0, typename V2<R>::T& a1, typename V2<R>::T& a2, typename V2<R>::T& a3) {
  const typename V2<R>::T s0 = add<R>(a0, a2), s1 = sub<R>(a0, a2), s2 = add<R>(a1, a3), d = sub<R>(a1, a3);
  const typename V2<R>::T s3 = INV ? mk2<R>(-d.y, d.x) : mk2<R>(d.y, -d.x);
  a0 = add<R>(s0, s2);
  a2 = sub<R>(s0, s2);
  a1 = add<R>(s1, s3);
  a3 = sub<R>(s1, s3);
}

// In-register FFT of length 16 (natural order in and out), 16 = 4 x 4.
template <typename R, bool INV>
__device__ __forceinline__ void fft16(typename V2<R>::T (&v)[16]) {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
  constexpr double c2 = 0.70710678118654752440;
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) fft4<R, INV>(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]);
  // twiddles w16^{n1 k2} on element n1 + 4 k2; w16 = e^{-+ 2 pi i / 16}
  const R sg = INV ? R(1) : R(-1);
  const typename V2<R>::T w1 = mk2<R>(R(c1), sg * R(s1)), w2 = mk2<R>(R(c2), sg * R(c2)),
           w3 = mk2<R>(R(s1), sg * R(c1)), w6 = mk2<R>(-R(c2), sg * R(c2)),
           w9 = mk2<R>(-R(c1), -sg * R(s1));
  const typename V2<R>::T w4 = mk2<R>(R(0), sg);
  v[1 + 4 * 1] = mul<R>(v[1 + 4 * 1], w1);
  v[1 + 4 * 2] = mul<R>(v[1 + 4 * 2], w2);
  v[1 + 4 * 3] = mul<R>(v[1 + 4 * 3], w3);
  v[2 + 4 * 1] = mul<R>(v[2 + 4 * 1], w2);
  v[2 + 4 * 2] = mul<R>(v[2 + 4 * 2], w4);
  v[2 + 4 * 3] = mul<R>(v[2 + 4 * 3], w6);
  v[3 + 4 * 1] = mul<R>(v[3 + 4 * 1], w3);
  v[3 + 4 * 2] = mul<R>(v[3 + 4 * 2], w6);
  v[3 + 4 * 3] = mul<R>(v[3 + 4 * 3], w9);
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) fft4<R, INV>(v[4 * k2], v[4 * k2 + 1], v[4 * k2 + 2], v[4 * k2 + 3]);
  // X[4 k1 + k2] sits at v[k1 + 4 k2]: transpose the 4 x 4 index grid
  typename V2<R>::T t[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[4 * k1 + k2] = v[k1 + 4 * k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = t[i];
}


}  // namespace fftdev
}  // namespace h6
