// Launchers of the multi-size step kernels for one arithmetic (TTSH_PREC =
// 32: FP32 with FP32 state, 64: FP64, 96: FP32 with FP64 state) and one
// workgroup size (TTSH_BS = 64, 128 or 256), both set on the compiler command
// line.  The row pass does not depend on the state type, so the FP32-state
// build also serves the FP64-state one.
#include "launch.hpp"
#include "step_multi.hpp"

#include <algorithm>

#if !defined(TTSH_PREC) || !defined(TTSH_BS)
#error "define TTSH_PREC and TTSH_BS"
#endif

namespace ttsh {
namespace {

#if TTSH_PREC == 64
using T = double;
using S = double;
#elif TTSH_PREC == 96
using T = float;
using S = double;
#else
using T = float;
using S = float;
#endif
constexpr int BS = TTSH_BS;

// dynamic LDS of a launch: the largest tile footprint over the classes present
template <class F>
size_t lds_bytes(const MultiArgs& a, F of) {
  size_t m = 0;
  for (int q = 0; q < a.ncls; ++q) m = std::max(m, (size_t)of(a.c[q].N));
  return m;
}

#if TTSH_PREC != 96
hipError_t row(const MultiArgs& a, int gw, hipStream_t s) {
  const int grid = a.start[a.ncls];
  const size_t lds = lds_bytes(a, row_smem_of<T, BS>);
  if (lds == 0) return hipErrorInvalidValue;
  if (gw)
    hipLaunchKernelGGL((row_multi<T, true, BS>), dim3(grid), dim3(BS), lds, s, a);
  else
    hipLaunchKernelGGL((row_multi<T, false, BS>), dim3(grid), dim3(BS), lds, s, a);
  return hipGetLastError();
}
#endif

template <bool GW, int MODE>
void col_multi_launch(const MultiArgs& a, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((col_multi<T, S, GW, MODE, BS>), dim3(a.start[a.ncls]), dim3(BS), lds, s, a);
}

// mode: 0 one-stage step, 1 state -> X only, 2 / 3 the ETD2RK stages, 4..7
// the ETDRK4 stages
hipError_t col(const MultiArgs& a, int gw, int mode, hipStream_t s) {
  const size_t lds = gw && mode != 1 ? lds_bytes(a, col_smem_of<T, BS, true>) : lds_bytes(a, col_smem_of<T, BS, false>);
  if (lds == 0) return hipErrorInvalidValue;
  switch (mode * 2 + (gw ? 1 : 0)) {
    case 0: col_multi_launch<false, 0>(a, lds, s); break;
    case 1: col_multi_launch<true, 0>(a, lds, s); break;
    case 2: case 3: col_multi_launch<false, 1>(a, lds, s); break;
    case 4: col_multi_launch<false, 2>(a, lds, s); break;
    case 5: col_multi_launch<true, 2>(a, lds, s); break;
    case 6: col_multi_launch<false, 3>(a, lds, s); break;
    case 7: col_multi_launch<true, 3>(a, lds, s); break;
    case 8: col_multi_launch<false, 4>(a, lds, s); break;
    case 9: col_multi_launch<true, 4>(a, lds, s); break;
    case 10: col_multi_launch<false, 5>(a, lds, s); break;
    case 11: col_multi_launch<true, 5>(a, lds, s); break;
    case 12: col_multi_launch<false, 6>(a, lds, s); break;
    case 13: col_multi_launch<true, 6>(a, lds, s); break;
    case 14: col_multi_launch<false, 7>(a, lds, s); break;
    case 15: col_multi_launch<true, 7>(a, lds, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// the arguments of class q alone
MultiArgs only(const MultiArgs& a, int q) {
  MultiArgs o = a;
  o.ncls = 1;
  o.c[0] = a.c[q];
  o.start[0] = 0;
  o.start[1] = a.start[q + 1] - a.start[q];
  return o;
}

template <int N>
hipError_t row_one_n(const MultiArgs& o, int gw, hipStream_t s) {
  if constexpr (row_smem_n<T, BS, N>() > 0) {
    const size_t lds = (row_smem_n<T, BS, N>());
    if (gw)
      hipLaunchKernelGGL((row_one<N, T, true, BS>), dim3(o.start[1]), dim3(BS), lds, s, o);
    else
      hipLaunchKernelGGL((row_one<N, T, false, BS>), dim3(o.start[1]), dim3(BS), lds, s, o);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N, bool GW, int MODE>
void col_one_launch(const MultiArgs& o, hipStream_t s) {
  hipLaunchKernelGGL((col_one<N, T, S, GW, MODE, BS>), dim3(o.start[1]), dim3(BS), (col_smem_n<T, BS, GW, N>()), s,
                     o);
}

template <int N>
hipError_t col_one_n(const MultiArgs& o, int gw, int mode, hipStream_t s) {
  if constexpr (col_smem_n<T, BS, true, N>() > 0) {
    switch (mode * 2 + (gw ? 1 : 0)) {
      case 0: col_one_launch<N, false, 0>(o, s); break;
      case 1: col_one_launch<N, true, 0>(o, s); break;
      case 2: case 3: col_one_launch<N, false, 1>(o, s); break;
      case 4: col_one_launch<N, false, 2>(o, s); break;
      case 5: col_one_launch<N, true, 2>(o, s); break;
      case 6: col_one_launch<N, false, 3>(o, s); break;
      case 7: col_one_launch<N, true, 3>(o, s); break;
      case 8: col_one_launch<N, false, 4>(o, s); break;
      case 9: col_one_launch<N, true, 4>(o, s); break;
      case 10: col_one_launch<N, false, 5>(o, s); break;
      case 11: col_one_launch<N, true, 5>(o, s); break;
      case 12: col_one_launch<N, false, 6>(o, s); break;
      case 13: col_one_launch<N, true, 6>(o, s); break;
      case 14: col_one_launch<N, false, 7>(o, s); break;
      case 15: col_one_launch<N, true, 7>(o, s); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

#if TTSH_PREC != 96
hipError_t row_split(const MultiArgs& a, int gw, hipStream_t s) {
  for (int q = 0; q < a.ncls; ++q) {
    const MultiArgs o = only(a, q);
    hipError_t e = hipErrorInvalidValue;
    switch (o.c[0].N) {
      case 64: e = row_one_n<64>(o, gw, s); break;
      case 128: e = row_one_n<128>(o, gw, s); break;
      case 256: e = row_one_n<256>(o, gw, s); break;
      case 512: e = row_one_n<512>(o, gw, s); break;
      case 1024: e = row_one_n<1024>(o, gw, s); break;
      case 2048: e = row_one_n<2048>(o, gw, s); break;
      default: break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
#endif

hipError_t col_split(const MultiArgs& a, int gw, int mode, hipStream_t s) {
  for (int q = 0; q < a.ncls; ++q) {
    const MultiArgs o = only(a, q);
    hipError_t e = hipErrorInvalidValue;
    switch (o.c[0].N) {
      case 64: e = col_one_n<64>(o, gw, mode, s); break;
      case 128: e = col_one_n<128>(o, gw, mode, s); break;
      case 256: e = col_one_n<256>(o, gw, mode, s); break;
      case 512: e = col_one_n<512>(o, gw, mode, s); break;
      case 1024: e = col_one_n<1024>(o, gw, mode, s); break;
      case 2048: e = col_one_n<2048>(o, gw, mode, s); break;
      default: break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

#define TTSH_CAT4(a, b, c, d) a##b##c##d
#define TTSH_NAME(p, b) TTSH_CAT4(multi_ops_, p, _, b)
const MultiOps* TTSH_NAME(TTSH_PREC, TTSH_BS)() {
#if TTSH_PREC != 96
  static const MultiOps ops = {row, col, row_split, col_split};
#else
  static const MultiOps ops = {nullptr, col, nullptr, col_split};
#endif
  return &ops;
}

}  // namespace ttsh
