// The time-step passes of the FP32 arithmetic (FP32 transforms and state)
// with a non-default transform schedule (TTSH_SCH, see fft.hpp) for one
// workgroup size (TTSH_BS): the row pass and the one-stage column pass, each
// as one launch over every size class.  These are the kernels the autotuner
// tries beside the default-schedule ones of step_multi.hip; the data layout
// does not depend on the schedule, so any other pass (set-up, the
// Runge-Kutta stages) may keep the default.
#include "launch.hpp"
#include "step_multi.hpp"

#include <algorithm>

#if !defined(TTSH_SCH) || !defined(TTSH_BS)
#error "define TTSH_SCH and TTSH_BS"
#endif

namespace ttsh {
namespace {

using T = float;
constexpr int BS = TTSH_BS;
constexpr int SCH = TTSH_SCH;

template <class F>
size_t lds_bytes(const MultiArgs& a, F of) {
  size_t m = 0;
  for (int q = 0; q < a.ncls; ++q) m = std::max(m, (size_t)of(a.c[q].N));
  return m;
}

hipError_t row(const MultiArgs& a, int gw, hipStream_t s) {
  const size_t lds = lds_bytes(a, row_smem_of<T, BS, SCH>);
  if (lds == 0) return hipErrorInvalidValue;
  if (gw)
    hipLaunchKernelGGL((row_multi<T, true, BS, SCH>), dim3(a.start[a.ncls]), dim3(BS), lds, s, a);
  else
    hipLaunchKernelGGL((row_multi<T, false, BS, SCH>), dim3(a.start[a.ncls]), dim3(BS), lds, s, a);
  return hipGetLastError();
}

hipError_t col(const MultiArgs& a, int gw, hipStream_t s) {
  const size_t lds = gw ? lds_bytes(a, col_smem_of<T, BS, true, SCH>) : lds_bytes(a, col_smem_of<T, BS, false, SCH>);
  if (lds == 0) return hipErrorInvalidValue;
  if (gw)
    hipLaunchKernelGGL((col_multi<T, T, true, 0, BS, SCH>), dim3(a.start[a.ncls]), dim3(BS), lds, s, a);
  else
    hipLaunchKernelGGL((col_multi<T, T, false, 0, BS, SCH>), dim3(a.start[a.ncls]), dim3(BS), lds, s, a);
  return hipGetLastError();
}

}  // namespace

#define TTSH_CAT4(a, b, c, d) a##b##c##d
#define TTSH_NAME(b, c) TTSH_CAT4(sched_ops_, b, _, c)
const SchedOps* TTSH_NAME(TTSH_BS, TTSH_SCH)() {
  static const SchedOps ops = {row, col};
  return &ops;
}

}  // namespace ttsh
