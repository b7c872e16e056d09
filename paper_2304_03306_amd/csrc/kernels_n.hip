// Full-array transforms for one grid size, TTSH_N (defined on the compiler
// command line: 64, 128, 256, 512, 1024 or 2048), used by the set-up and read-out
// paths.
#include "fft_full.hpp"
#include "launch.hpp"

#ifndef TTSH_N
#error "define TTSH_N"
#endif

namespace ttsh {
namespace {

constexpr int N = TTSH_N;
constexpr int TT = N / kFftE;
template <class T, int DIR>
hipError_t fft2_t(void* p, int batch, const void* tw, hipStream_t s) {
  C2<T>* a = (C2<T>*)p;
  constexpr int RPB = FullFft<N>::RPB, CPB = FullFft<N>::CPB;
  const int rows = batch * N;
  hipLaunchKernelGGL((fft_rows<N, DIR, T>), dim3((rows + RPB - 1) / RPB), dim3(RPB * TT), 0, s, a,
                     rows, (const C2<T>*)tw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fft_cols<N, DIR, T>), dim3((rows + CPB - 1) / CPB), dim3(CPB * TT), 0, s, a,
                     rows, (const C2<T>*)tw);
  return hipGetLastError();
}

hipError_t fft2(void* a, int batch, int dir, int fp64, const void* tw, hipStream_t s) {
  if (fp64) return dir < 0 ? fft2_t<double, -1>(a, batch, tw, s) : fft2_t<double, +1>(a, batch, tw, s);
  return dir < 0 ? fft2_t<float, -1>(a, batch, tw, s) : fft2_t<float, +1>(a, batch, tw, s);
}

}  // namespace

#define TTSH_CAT2(a, b) a##b
#define TTSH_CAT(a, b) TTSH_CAT2(a, b)
const SizeOps* TTSH_CAT(ops_, TTSH_N)() {
  static const SizeOps ops = {fft2};
  return &ops;
}

}  // namespace ttsh
