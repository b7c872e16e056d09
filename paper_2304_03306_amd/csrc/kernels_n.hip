// Kernel instantiations and launchers for one grid size, TTSH_N (defined on
// the compiler command line: 64, 128, 256, 512 or 1024).  Splitting by N keeps
// every translation unit small enough to compile in parallel.
#include "fft_full.hpp"
#include "launch.hpp"
#include "step.hpp"

#ifndef TTSH_N
#error "define TTSH_N"
#endif

namespace ttsh {
namespace {

constexpr int N = TTSH_N;
constexpr int TT = N / kFftE;
constexpr size_t kMaxLds = 65536;

template <class T, int RP>
constexpr bool row_valid() {
  return (RP * TT) % 64 == 0 && RP * TT <= 1024 && RP <= N / 2 &&
         (size_t)RP * 3 * Padded<N>::value * sizeof(C2<T>) +
                 (size_t)(RP * TT / 64) * RP * 4 * sizeof(T) <=
             kMaxLds;
}
template <class T, int TC>
constexpr bool col_valid() {
  return (TC * TT) % 64 == 0 && TC * TT <= 1024 && TC <= N / 4 + 1 &&
         ColSmem<N, TC, T, true>::bytes <= kMaxLds;
}

template <class T, bool GW, int RP>
hipError_t row_launch(const PassArgs& a, hipStream_t s) {
  if constexpr (row_valid<T, RP>()) {
    RowCoef<T> c{(T)a.beta, (T)a.gamma_v, (T)a.lambda0, (T)a.gamma_w};
    hipLaunchKernelGGL((row_pass<N, RP, T, GW>), dim3(N / (2 * RP), a.n), dim3(RP * TT), 0, s,
                       (const C2<T>*)a.X_in, (C2<T>*)a.Y, (const T*)a.K, (T*)a.rowsum,
                       (const C2<T>*)a.tw, c);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <class T, bool GW>
hipError_t row_dispatch(const PassArgs& a, hipStream_t s) {
  switch (a.rp) {
    case 1: return row_launch<T, GW, 1>(a, s);
    case 2: return row_launch<T, GW, 2>(a, s);
    case 4: return row_launch<T, GW, 4>(a, s);
    case 8: return row_launch<T, GW, 8>(a, s);
    case 16: return row_launch<T, GW, 16>(a, s);
    case 32: return row_launch<T, GW, 32>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t row(const PassArgs& a, hipStream_t s) {
  if (a.prec == 64) return a.gw ? row_dispatch<double, true>(a, s) : row_dispatch<double, false>(a, s);
  return a.gw ? row_dispatch<float, true>(a, s) : row_dispatch<float, false>(a, s);
}

template <class T, class S, bool GW, int TC, int MODE>
hipError_t col_launch(const PassArgs& a, hipStream_t s) {
  if constexpr (col_valid<T, TC>()) {
    constexpr int MP = N / 4 + 1;
    LinCoef lc{a.alpha, a.gamma0, a.gamma2, a.dt, a.dt_over_N, a.scheme};
    hipLaunchKernelGGL((col_pass<N, TC, T, S, GW, MODE>), dim3((MP + TC - 1) / TC, a.n),
                       dim3(TC * TT), 0, s, (const C2<T>*)a.Y, (C2<T>*)a.X_out, (C2<S>*)a.st,
                       (const T*)a.rowsum, a.dk, (const C2<T>*)a.tw, lc);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <class T, class S, bool GW, int MODE>
hipError_t col_dispatch(const PassArgs& a, hipStream_t s) {
  switch (a.tc) {
    case 1: return col_launch<T, S, GW, 1, MODE>(a, s);
    case 2: return col_launch<T, S, GW, 2, MODE>(a, s);
    case 4: return col_launch<T, S, GW, 4, MODE>(a, s);
    case 8: return col_launch<T, S, GW, 8, MODE>(a, s);
    case 16: return col_launch<T, S, GW, 16, MODE>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <class T, class S, int MODE>
hipError_t col_mode(const PassArgs& a, hipStream_t s) {
  // MODE 1 never reads Y, so the gamma_w variant is irrelevant there
  if (MODE == 0 && a.gw) return col_dispatch<T, S, true, MODE>(a, s);
  return col_dispatch<T, S, false, MODE>(a, s);
}

hipError_t col(const PassArgs& a, int mode, hipStream_t s) {
  if (a.prec == 64) return mode ? col_mode<double, double, 1>(a, s) : col_mode<double, double, 0>(a, s);
  if (a.prec == 96) return mode ? col_mode<float, double, 1>(a, s) : col_mode<float, double, 0>(a, s);
  return mode ? col_mode<float, float, 1>(a, s) : col_mode<float, float, 0>(a, s);
}

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

template <class T>
unsigned row_opts_t() {
  return (row_valid<T, 1>() ? 1u : 0u) | (row_valid<T, 2>() ? 2u : 0u) |
         (row_valid<T, 4>() ? 4u : 0u) | (row_valid<T, 8>() ? 8u : 0u) |
         (row_valid<T, 16>() ? 16u : 0u) | (row_valid<T, 32>() ? 32u : 0u);
}
template <class T>
unsigned col_opts_t() {
  return (col_valid<T, 1>() ? 1u : 0u) | (col_valid<T, 2>() ? 2u : 0u) |
         (col_valid<T, 4>() ? 4u : 0u) | (col_valid<T, 8>() ? 8u : 0u) |
         (col_valid<T, 16>() ? 16u : 0u);
}
unsigned row_options(int prec, int) { return prec == 64 ? row_opts_t<double>() : row_opts_t<float>(); }
unsigned col_options(int prec, int) { return prec == 64 ? col_opts_t<double>() : col_opts_t<float>(); }

}  // namespace

#define TTSH_CAT2(a, b) a##b
#define TTSH_CAT(a, b) TTSH_CAT2(a, b)
const SizeOps* TTSH_CAT(ops_, TTSH_N)() {
  static const SizeOps ops = {row, col, fft2, row_options, col_options};
  return &ops;
}

}  // namespace ttsh
