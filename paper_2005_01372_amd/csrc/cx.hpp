// Interleaved complex numbers for the HIP kernels (re, im adjacent in memory).
#pragma once
#include <hip/hip_runtime.h>

template <typename T>
struct alignas(2 * sizeof(T)) Cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ Cx<T> cx(T r, T i) { return Cx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator*(T s, Cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> conjx(Cx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ Cx<T> cmul_conj(Cx<T> a, Cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__host__ __device__ __forceinline__ Cx<T> mul_mi(Cx<T> a) {
  if constexpr (INV) return {-a.im, a.re};
  else return {a.im, -a.re};
}
template <typename T>
__host__ __device__ __forceinline__ T norm2(Cx<T> a) { return a.re * a.re + a.im * a.im; }

template <typename T>
__host__ __device__ __forceinline__ Cx<T> czero() { return {T(0), T(0)}; }

template <typename To, typename Ti>
__host__ __device__ __forceinline__ Cx<To> ccast(Cx<Ti> a) { return {To(a.re), To(a.im)}; }
