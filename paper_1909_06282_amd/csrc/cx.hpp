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

// Streaming (non-temporal) global accesses: data that one pass touches once
// goes through the caches without displacing what is reused (the radial
// tables the x passes gather).
template <typename T>
__device__ __forceinline__ void st_nt(Cx<T>* p, Cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));
}
template <typename T>
__device__ __forceinline__ Cx<T> ld_nt(const Cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 w = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return mk(w.x, w.y);
}

}  // namespace lpt2
