// Host-side launch interface between the runtime (ttsh_capi.hip) and the
// kernels compiled once per grid size (kernels_n.hip built with -DTTSH_N=...).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ttsh {

// Everything one launch of the row or column pass needs for a group of
// instances that share the grid size N (arrays start at the first instance of
// the group; consecutive instances are contiguous).
struct PassArgs {
  int N;        // grid points per side
  int n;        // instances in this launch (grid.y)
  int prec;     // 32, 64 or 96 (FP32 with FP64 state)
  int gw;       // 1 if gamma_w != 0 (third forward transform)
  int rp, tc;   // row pairs / columns per workgroup
  const void* X_in;  // row pass reads X
  void* X_out;       // column pass writes X
  void* Y;
  void* st;
  const void* K;
  void* rowsum;
  const double* dk;
  const void* tw;    // twiddles e^{-2 pi i j/N} in the run precision
  double beta, gamma_v, lambda0, gamma_w;
  double alpha, gamma0, gamma2, dt, dt_over_N;
  int scheme;
};

struct SizeOps {
  // time-step passes; return hipSuccess or the launch error
  hipError_t (*row)(const PassArgs&, hipStream_t);
  hipError_t (*col)(const PassArgs&, int mode, hipStream_t);
  // unnormalised 2D transform of `batch` N x N complex arrays in place;
  // dir = -1 forward, +1 inverse; fp64 selects double (else float) data
  hipError_t (*fft2)(void* a, int batch, int dir, int fp64, const void* tw, hipStream_t);
  // tile options that compile for this N (bit i set: 2^i is valid)
  unsigned (*row_options)(int prec, int gw);
  unsigned (*col_options)(int prec, int gw);
};

const SizeOps* size_ops(int N);

}  // namespace ttsh
