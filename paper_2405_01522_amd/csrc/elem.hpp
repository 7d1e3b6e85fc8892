// Element-type helpers so the ACE kernels serve real (float, double) and complex
// (C2<float>, C2<double>) orbitals with one body each.
#pragma once

#include "common.hpp"

namespace ace {

template <typename E>
struct Elem;
template <>
struct Elem<float> {
  typedef float real;
  typedef double wide;
  static constexpr bool cplx = false;
};
template <>
struct Elem<double> {
  typedef double real;
  typedef double wide;
  static constexpr bool cplx = false;
};
template <>
struct Elem<C2<float>> {
  typedef float real;
  typedef C2<double> wide;
  static constexpr bool cplx = true;
};
template <>
struct Elem<C2<double>> {
  typedef double real;
  typedef C2<double> wide;
  static constexpr bool cplx = true;
};

__host__ __device__ __forceinline__ float e_conj(float a) { return a; }
__host__ __device__ __forceinline__ double e_conj(double a) { return a; }
template <typename T>
__host__ __device__ __forceinline__ C2<T> e_conj(C2<T> a) { return {a.r, -a.i}; }

__host__ __device__ __forceinline__ float e_mul(float a, float b) { return a * b; }
__host__ __device__ __forceinline__ double e_mul(double a, double b) { return a * b; }
template <typename T>
__host__ __device__ __forceinline__ C2<T> e_mul(C2<T> a, C2<T> b) { return cmul(a, b); }

// conj(a) * b
__host__ __device__ __forceinline__ float e_mulc(float a, float b) { return a * b; }
__host__ __device__ __forceinline__ double e_mulc(double a, double b) { return a * b; }
template <typename T>
__host__ __device__ __forceinline__ C2<T> e_mulc(C2<T> a, C2<T> b) { return cmulc(a, b); }

__host__ __device__ __forceinline__ float e_add(float a, float b) { return a + b; }
__host__ __device__ __forceinline__ double e_add(double a, double b) { return a + b; }
template <typename T>
__host__ __device__ __forceinline__ C2<T> e_add(C2<T> a, C2<T> b) { return cadd(a, b); }

__host__ __device__ __forceinline__ float e_neg(float a) { return -a; }
__host__ __device__ __forceinline__ double e_neg(double a) { return -a; }
template <typename T>
__host__ __device__ __forceinline__ C2<T> e_neg(C2<T> a) { return {-a.r, -a.i}; }

template <typename E>
__host__ __device__ __forceinline__ E e_zero() {
  return E{};
}

// widen / narrow between the storage element and its FP64 counterpart
__host__ __device__ __forceinline__ double e_wide(float a) { return a; }
__host__ __device__ __forceinline__ double e_wide(double a) { return a; }
template <typename T>
__host__ __device__ __forceinline__ C2<double> e_wide(C2<T> a) { return {double(a.r), double(a.i)}; }

template <typename E>
__host__ __device__ __forceinline__ E e_narrow(typename Elem<E>::wide a);
template <>
__host__ __device__ __forceinline__ float e_narrow<float>(double a) { return (float)a; }
template <>
__host__ __device__ __forceinline__ double e_narrow<double>(double a) { return a; }
template <>
__host__ __device__ __forceinline__ C2<float> e_narrow<C2<float>>(C2<double> a) {
  return {(float)a.r, (float)a.i};
}
template <>
__host__ __device__ __forceinline__ C2<double> e_narrow<C2<double>>(C2<double> a) { return a; }

__host__ __device__ __forceinline__ double e_re(double a) { return a; }
__host__ __device__ __forceinline__ double e_re(C2<double> a) { return a.r; }
__host__ __device__ __forceinline__ bool e_finite(double a) { return isfinite(a); }
__host__ __device__ __forceinline__ bool e_finite(C2<double> a) { return isfinite(a.r) && isfinite(a.i); }
__host__ __device__ __forceinline__ double e_abs2(double a) { return a * a; }
__host__ __device__ __forceinline__ double e_abs2(C2<double> a) { return a.r * a.r + a.i * a.i; }
__host__ __device__ __forceinline__ double e_scale(double a, double s) { return a * s; }
__host__ __device__ __forceinline__ C2<double> e_scale(C2<double> a, double s) { return {a.r * s, a.i * s}; }
__host__ __device__ __forceinline__ double e_sub(double a, double b) { return a - b; }
__host__ __device__ __forceinline__ C2<double> e_sub(C2<double> a, C2<double> b) { return csub(a, b); }

}  // namespace ace
