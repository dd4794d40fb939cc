// Fast transform path for odd period parameters M = n + 1 up to 255 (other
// than 257): device tables and launchers (see xform_bluestein.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace h6 {

struct BluesteinTables {
  int M = 0;                       // period parameter (odd, <= 255)
  int P = 0;                       // convolution length: 256 (M <= 129) or 512
  const double2* chirp = nullptr;  // c_q = exp(-i pi q^2 / M), q = 0..M-1
  const double2* bhat = nullptr;   // FFT_P(b) / P, b_j = conj(c_j) for |j| < M (cyclic), 0 elsewhere
  const double2* tw = nullptr;     // exp(-2 pi i t / P), t = 0..P-1
  const double* sin_q = nullptr;   // sin(pi q / M), q = 0..M-1
  const double* cos_q = nullptr;   // cos(pi q / M), q = 0..M-1
  const float2* chirp_f = nullptr; // the same tables rounded to single precision (complex64 path)
  const float2* bhat_f = nullptr;
  const float2* tw_f = nullptr;
  const float* sin_f = nullptr;
  const float* cos_f = nullptr;
};

// Largest M of the path and the convolution length it needs: the lags k - q
// of the convolution take the 2M - 2 values 1 - M .. M - 2 (y_0 = 0), so a
// cyclic length P >= 2M - 2 holds them without wrap-around.
constexpr int kBluesteinMaxM = 255;
inline int bluestein_length(int M) { return 2 * M - 2 <= 256 ? 256 : 512; }
inline bool bluestein_ok(int M) { return M >= 3 && M <= kBluesteinMaxM && (M & 1); }

// Same conventions as launch_rader_x / launch_rader_y (forward: W^{-1},
// inverse: W; accumulate: out += result, x lines with a complex128 output only).
template <typename R, typename Tin, typename Tout>
hipError_t launch_bluestein_x(bool neumann, bool inverse, const Tin* in, Tout* out, int nlines, int L,
                              const BluesteinTables& tab, hipStream_t s, int accumulate,
                              const int* skip = nullptr);
template <typename R, typename T>
hipError_t launch_bluestein_y(bool neumann, bool inverse, const T* in, T* out, int nx, int L, int nz,
                              const BluesteinTables& tab, hipStream_t s, const int* skip = nullptr);

}  // namespace h6
