// Fast transform path for the period parameter M = 257 (n = 256): device
// tables and launchers (see xform_rader.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace h6 {

struct RaderTables {
  const int* perm_in;      // g^{-a} mod M, a = 0..M-2
  const int* perm_out;     // g^{b} mod M,  b = 0..M-2
  const double2* kf;       // FFT_{M-1} of w^{g^c} (w = e^{-2 pi i / M}), divided by M-1
  const double2* tw256;    // e^{-2 pi i t / 256}
  const double* sin_a;     // sin(pi g^{-a} / M), a = 0..M-2
  const double* cos_a;     // cos(pi g^{-a} / M), a = 0..M-2
  const int* slot_d;       // LDS slot of array index p of a sine-basis line (node q = p + 1)
  const int* slot_n;       // LDS slot of array index p of a cosine-basis line (node q = p)
  const float2* kf_f;      // kf, tw256, sin_a, cos_a rounded to single precision (complex64 path)
  const float2* tw_f;
  const float* sin_f;
  const float* cos_f;
};

constexpr int kRaderM = 257;

// Lines per workgroup supported per axis (x: 4, 8; y: 8, 16).
bool rader_lines_ok(int axis, int lines);

// accumulate != 0 (inverse transforms with a complex128 output only): out += result.
// lines: lines (x) or columns (y) per workgroup, one of rader_lines_ok's values.
// skip: device flag; when nonzero the kernels return at once (whole-cycle graphs).
template <typename R, typename Tin, typename Tout>
hipError_t launch_rader_x(bool neumann, bool inverse, const Tin* in, Tout* out, int nlines, int L,
                          const RaderTables& tab, hipStream_t s, int accumulate, int lines,
                          const int* skip = nullptr);
template <typename R, typename T>
hipError_t launch_rader_y(bool neumann, bool inverse, const T* in, T* out, int nx, int L, int nz,
                          const RaderTables& tab, hipStream_t s, int lines, const int* skip = nullptr);

}  // namespace h6
