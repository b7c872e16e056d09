// Shared device-side helpers of the TTSH library: complex arithmetic and
// reductions.  gfx950 only; wavefronts are 64 lanes wide.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ttsh {

template <class T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};

template <class T>
__device__ __forceinline__ C2<T> mk(T x, T y) {
  C2<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <class T>
__device__ __forceinline__ C2<T> operator+(C2<T> a, C2<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <class T>
__device__ __forceinline__ C2<T> operator-(C2<T> a, C2<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <class T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return mk(a.x * s, a.y * s); }
template <class T>
__device__ __forceinline__ C2<T> conj(C2<T> a) { return mk(a.x, -a.y); }
// multiply by i^DIR for DIR = +1 (i) or -1 (-i)
template <int DIR, class T>
__device__ __forceinline__ C2<T> mul_i(C2<T> a) {
  return DIR > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

template <class D, class S>
__device__ __forceinline__ C2<D> cvt(C2<S> a) { return mk<D>((D)a.x, (D)a.y); }

// Sum over the 64 lanes of a wavefront for lanes whose index differs only in
// the bits at and above `from` (from a power of two); lanes that share the low
// bits end up with the same total.
template <class T>
__device__ __forceinline__ T wave_sum_from(T v, int from) {
  for (int o = from; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace ttsh
