// Host-side launch interface between the runtime (ttsh_capi.hip) and the
// kernels compiled once per grid size (kernels_n.hip built with -DTTSH_N=...).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ttsh {

struct MultiArgs;

// Full-array transforms compiled per grid size (set-up and read-out paths).
struct SizeOps {
  // unnormalised 2D transform of `batch` N x N complex arrays in place;
  // dir = -1 forward, +1 inverse; fp64 selects double (else float) data
  hipError_t (*fft2)(void* a, int batch, int dir, int fp64, const void* tw, hipStream_t);
};

// Time-step passes over every size class of a context, compiled per
// arithmetic and workgroup size.  row is null for the FP64-state arithmetic
// (its row pass is the FP32 one).
struct MultiOps {
  hipError_t (*row)(const MultiArgs&, int gw, hipStream_t);
  hipError_t (*col)(const MultiArgs&, int gw, int mode, hipStream_t);
  // the same passes as one launch per size class
  hipError_t (*row_split)(const MultiArgs&, int gw, hipStream_t);
  hipError_t (*col_split)(const MultiArgs&, int gw, int mode, hipStream_t);
};

// The FP32 row pass and one-stage column pass with a non-default transform
// schedule, one launch over every size class (autotuner candidates).
struct SchedOps {
  hipError_t (*row)(const MultiArgs&, int gw, hipStream_t);
  hipError_t (*col)(const MultiArgs&, int gw, hipStream_t);
};
// schedules compiled besides the default, in the order the autotuner tries them
constexpr int kNumSchedVariants = 5;
constexpr int kSchedVariants[kNumSchedVariants] = {6, 10, 9, 7, 11};  // 2 PAD + SMALL_FIRST
const SchedOps* sched_ops(int bs, int sch);  // null for the default schedule or an unknown one

// The passes of one size class of the paper's production sizes (4096, 8192),
// whose workgroups have N/8 threads: `o` holds that class alone (c[0]).
struct BigOps {
  hipError_t (*row)(const MultiArgs& o, int gw, hipStream_t);
  hipError_t (*col)(const MultiArgs& o, int gw, int mode, hipStream_t);
};
constexpr int kMaxBlockN = 2048;  // the largest size served by the 64..256-thread kernels
const BigOps* big_ops(int N, int prec);  // null where the tiles do not fit (8192 in FP64)

const SizeOps* size_ops(int N);
// record `msg` as the calling thread's last error (ttsh_last_error) and return code
int record_error(int code, const char* msg);
const MultiOps* multi_ops(int prec, int bs);

}  // namespace ttsh
