// Complex arithmetic for the axis-pass kernels (interleaved re, im).
#pragma once
#include <hip/hip_runtime.h>

namespace lpt2 {

template <typename T>
struct alignas(2 * sizeof(T)) Cx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ Cx<T> mk(T a, T b) {
  Cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> scale(Cx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> conj(Cx<T> a) { return mk(a.x, -a.y); }
// a * (s i) for s = +1 or -1
template <int S, typename T>
__host__ __device__ __forceinline__ Cx<T> mul_si(Cx<T> a) {
  return S > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> zero() { return mk(T(0), T(0)); }

}  // namespace lpt2
