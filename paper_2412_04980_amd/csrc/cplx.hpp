// Complex arithmetic on interleaved (re, im) pairs, shared by the device
// kernels and the host solver of the MADP library.
#pragma once
#include <hip/hip_runtime.h>

namespace hm {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};
using c64 = cx<float>;
using c128 = cx<double>;

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { cx<T> z; z.re = r; z.im = i; return z; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk(s * a.re, s * a.im); }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// a / b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  T d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cx<To> cvt(cx<Ti> a) { return mk<To>((To)a.re, (To)a.im); }

}  // namespace hm
