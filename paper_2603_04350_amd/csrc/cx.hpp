// Complex arithmetic helpers shared by every kernel of the library.
//
// cx<T> is a two-component value type aligned to its full size so that one
// element is one 16-byte (fp64) or 8-byte (fp32) vector load or store.
#pragma once
#include <hip/hip_runtime.h>

namespace expdiag {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T re, T im) {
  cx<T> r;
  r.x = re;
  r.y = im;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return mk(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return mk(a.x - b.x, a.y - b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, T s) {
  return mk(a.x * s, a.y * s);
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) {
  return mk(a.x, -a.y);
}
// multiply by +i (S = +1) or -i (S = -1)
template <int S, typename T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {
  if constexpr (S > 0)
    return mk(-a.y, a.x);
  else
    return mk(a.y, -a.x);
}
template <typename TO, typename TI>
__device__ __forceinline__ cx<TO> cvt(cx<TI> a) {
  return mk(static_cast<TO>(a.x), static_cast<TO>(a.y));
}
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) {
  return a.x * a.x + a.y * a.y;
}

// Accesses through pointers read from job tables.  The compiler cannot see
// where such a pointer points and would emit flat instructions (which also
// count against the LDS wait counter); every such pointer is device global
// memory, and these say so.
template <typename T>
using gmem = __attribute__((address_space(1))) T;

// (The host compilation pass only type-checks device bodies and has no
// address space 1, so it sees the plain access.)
template <typename T>
__device__ __forceinline__ T gld(const T* p, long i) {
#if __HIP_DEVICE_COMPILE__
  return ((const gmem<T>*)p)[i];
#else
  return p[i];
#endif
}
template <typename T>
__device__ __forceinline__ void gst(T* p, long i, T v) {
#if __HIP_DEVICE_COMPILE__
  ((gmem<T>*)p)[i] = v;
#else
  p[i] = v;
#endif
}

}  // namespace expdiag
