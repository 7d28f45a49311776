// Shared device/host definitions of the pst HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pst {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return cpx<T>{a.re + b.re, a.im + b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return cpx<T>{a.re - b.re, a.im - b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, T s) {
  return cpx<T>{a.re * s, a.im * s};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return cpx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmul_conj(cpx<T> a, cpx<T> b) {
  return cpx<T>{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conj(cpx<T> a) {
  return cpx<T>{a.re, -a.im};
}
template <typename T>
__host__ __device__ __forceinline__ T norm2(cpx<T> a) {
  return a.re * a.re + a.im * a.im;
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) {
  return cpx<T>{-a.im, a.re};
}

// cos and sin of 2*pi*m/16 as compile-time constants.
__host__ __device__ constexpr double c16_first_octant(int m) {
  // m in 0..4: cos(2 pi m / 16)
  return m == 0 ? 1.0
       : m == 1 ? 0.92387953251128675613
       : m == 2 ? 0.70710678118654752440
       : m == 3 ? 0.38268343236508977173
       : 0.0;
}
__host__ __device__ constexpr double cos16(int m) {
  m = ((m % 16) + 16) % 16;
  return m <= 4 ? c16_first_octant(m)
       : m <= 8 ? -c16_first_octant(8 - m)
       : m <= 12 ? -c16_first_octant(m - 8)
       : c16_first_octant(16 - m);
}
__host__ __device__ constexpr double sin16(int m) { return cos16(m - 4); }

__host__ __device__ constexpr double cos_const(double ang) {
  // only called with ang = 2 pi m / 16
  return cos16((int)(ang * 16.0 / (2.0 * 3.14159265358979323846) + 0.5));
}
__host__ __device__ constexpr double sin_const(double ang) {
  return sin16((int)(ang * 16.0 / (2.0 * 3.14159265358979323846) + 0.5));
}

}  // namespace pst
