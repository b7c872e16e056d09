// The time-step passes for the paper's production grid sizes, TTSH_N = 4096
// or 8192 points per side (set on the compiler command line with TTSH_PREC):
// one workgroup of N/8 threads (512 or 1024) carries one row pair (row pass)
// or one column (column pass), so that a whole length-N transform of the
// three fields stays in LDS (FP32: 2 x 8704 complex entries, 139 KB at 8192,
// within the 160 KB a gfx950 workgroup addresses; FP64 fits up to 4096).
// The tile bodies are those of every other size; only the workgroup size
// differs, and these sizes always run one launch per size class.
#include "launch.hpp"
#include "step_multi.hpp"

#if !defined(TTSH_N) || !defined(TTSH_PREC)
#error "define TTSH_N and TTSH_PREC"
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
constexpr int N = TTSH_N;
constexpr int BS = N / 8;
static_assert(row_smem_n<T, BS, N>() > 0 && col_smem_n<T, BS, true, N>() > 0, "tiles must fit the LDS");

hipError_t row(const MultiArgs& o, int gw, hipStream_t s) {
  constexpr size_t lds = row_smem_n<T, BS, N>();
  if (gw)
    hipLaunchKernelGGL((row_one<N, T, true, BS>), dim3(o.start[1]), dim3(BS), lds, s, o);
  else
    hipLaunchKernelGGL((row_one<N, T, false, BS>), dim3(o.start[1]), dim3(BS), lds, s, o);
  return hipGetLastError();
}

template <bool GW, int MODE>
void col_launch(const MultiArgs& o, hipStream_t s) {
  hipLaunchKernelGGL((col_one<N, T, S, GW, MODE, BS>), dim3(o.start[1]), dim3(BS), (col_smem_n<T, BS, GW, N>()), s, o);
}

hipError_t col(const MultiArgs& o, int gw, int mode, hipStream_t s) {
  switch (mode * 2 + (gw ? 1 : 0)) {
    case 0: col_launch<false, 0>(o, s); break;
    case 1: col_launch<true, 0>(o, s); break;
    case 2: case 3: col_launch<false, 1>(o, s); break;
    case 4: col_launch<false, 2>(o, s); break;
    case 5: col_launch<true, 2>(o, s); break;
    case 6: col_launch<false, 3>(o, s); break;
    case 7: col_launch<true, 3>(o, s); break;
    case 8: col_launch<false, 4>(o, s); break;
    case 9: col_launch<true, 4>(o, s); break;
    case 10: col_launch<false, 5>(o, s); break;
    case 11: col_launch<true, 5>(o, s); break;
    case 12: col_launch<false, 6>(o, s); break;
    case 13: col_launch<true, 6>(o, s); break;
    case 14: col_launch<false, 7>(o, s); break;
    case 15: col_launch<true, 7>(o, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

#define TTSH_CAT4(a, b, c, d) a##b##c##d
#define TTSH_NAME(n, p) TTSH_CAT4(big_ops_, n, _, p)
const BigOps* TTSH_NAME(TTSH_N, TTSH_PREC)() {
  static const BigOps ops = {row, col};
  return &ops;
}

}  // namespace ttsh
