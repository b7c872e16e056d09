// One launch per pass for every instance of a context, whatever its mix of
// grid sizes.  Workgroups have a fixed size BS; an instance of size N is cut
// into tiles of BS threads: RP = BS/(N/8) row pairs per row-pass tile and
// TC = BS/(N/8) columns per column-pass tile, so every tile carries the same
// amount of data (16 BS grid points of the row pass, 8 BS of the column pass)
// and the LDS footprint is the same for every N.  Workgroup b finds its size
// class from prefix sums of the per-class tile counts, then its instance and
// tile; the class test is uniform across the workgroup.
#pragma once

#include "step.hpp"

namespace ttsh {

constexpr int kMaxClasses = 6;

struct ClassArgs {
  int N;       // grid points per side
  int n;       // instances in the class (contiguous in every array below)
  int tiles;   // tiles per instance in this pass
  const void* X_in;
  void* X_out;
  void* Y;
  void* st;
  const void* K;
  void* rowsum;
  const double* dk;
  const void* tw;
  void* st2;      // ETD2RK / ETDRK4 stage state (same layout as st), else null
  void* fst;      // kept forcing spectra of the exponential Runge-Kutta stages, else null
  double* s1st;   // their k = 0 forcing sums ([n][2] ETD2RK, [n][4] ETDRK4), else null
};

struct MultiArgs {
  int ncls;
  int start[kMaxClasses + 1];  // first workgroup of each class; start[ncls] = grid size
  ClassArgs c[kMaxClasses];
  double beta, gamma_v, lambda0, gamma_w;
  LinCoef lc;
};

template <int N, int BS>
struct TileOf {
  static constexpr int TT = N / 8;
  static constexpr int R = BS / TT;  // row pairs (row pass) or columns (column pass)
  static constexpr bool ok = BS % TT == 0 && R >= 1;
};

// LDS bytes of one tile of size N; the launch allocates the largest over the
// size classes present (dynamic LDS), so that a context without the small
// grids, whose padded tiles need the most LDS, keeps a higher occupancy.
// A tile may take up to the 160 KB of LDS one gfx950 workgroup can address
// (FP64 transforms of 2048 points need about 70 KB); larger tiles give 0.
constexpr size_t kMaxTileLds = 163840;
template <class T, int BS, int N, int SCH = kSchedDefault>
constexpr size_t row_smem_n() {
  if constexpr (TileOf<N, BS>::ok) {
    constexpr size_t b = RowSmem<N, TileOf<N, BS>::R, T, SCH>::bytes;
    return b <= kMaxTileLds ? b : 0;
  } else {
    return 0;
  }
}
template <class T, int BS, bool GW, int N, int SCH = kSchedDefault>
constexpr size_t col_smem_n() {
  if constexpr (TileOf<N, BS>::ok) {
    constexpr size_t b = ColSmem<N, TileOf<N, BS>::R, T, GW, SCH>::bytes;
    return b <= kMaxTileLds ? b : 0;
  } else {
    return 0;
  }
}
template <class T, int BS, int SCH = kSchedDefault>
constexpr size_t row_smem_of(int N) {
  return N == 64 ? row_smem_n<T, BS, 64, SCH>() : N == 128 ? row_smem_n<T, BS, 128, SCH>()
       : N == 256 ? row_smem_n<T, BS, 256, SCH>() : N == 512 ? row_smem_n<T, BS, 512, SCH>()
       : N == 1024 ? row_smem_n<T, BS, 1024, SCH>() : N == 2048 ? row_smem_n<T, BS, 2048, SCH>() : 0;
}
template <class T, int BS, bool GW, int SCH = kSchedDefault>
constexpr size_t col_smem_of(int N) {
  return N == 64 ? col_smem_n<T, BS, GW, 64, SCH>() : N == 128 ? col_smem_n<T, BS, GW, 128, SCH>()
       : N == 256 ? col_smem_n<T, BS, GW, 256, SCH>() : N == 512 ? col_smem_n<T, BS, GW, 512, SCH>()
       : N == 1024 ? col_smem_n<T, BS, GW, 1024, SCH>() : N == 2048 ? col_smem_n<T, BS, GW, 2048, SCH>() : 0;
}

// Workgroups are handed to the eight XCDs round-robin (workgroup b runs on
// XCD b % 8).  Map them so that each XCD receives one contiguous range of
// tiles: neighbouring row tiles share cache lines of the interleaved
// mixed-domain arrays, and this keeps those lines in one XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int x = b & 7, j = b >> 3, q = G >> 3, r = G & 7;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + j;
}

__device__ __forceinline__ int class_of(const MultiArgs& a, int b) {
  int ci = 0;
#pragma unroll
  for (int q = 1; q < kMaxClasses; ++q)
    if (q < a.ncls && b >= a.start[q]) ci = q;
  return ci;
}

template <int N, class T, bool GW, int BS, int SCH = kSchedDefault>
__device__ __forceinline__ void row_go(const ClassArgs& d, const RowCoef<T>& c, int inst, int tile,
                                       unsigned char* smem) {
  if constexpr (row_smem_n<T, BS, N, SCH>() > 0)
    row_body<N, TileOf<N, BS>::R, T, GW, SCH>((const C2<T>*)d.X_in, (C2<T>*)d.Y, (const T*)d.K,
                                              (T*)d.rowsum, (const C2<T>*)d.tw, c, inst, tile, smem);
}

template <class T, bool GW, int BS, int SCH = kSchedDefault>
__global__ void __launch_bounds__(BS) row_multi(MultiArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int ci = class_of(a, b);
  const ClassArgs& d = a.c[ci];
  const int local = b - a.start[ci];
  const int inst = local / d.tiles;
  const int tile = local - inst * d.tiles;
  const RowCoef<T> c{(T)a.beta, (T)a.gamma_v, (T)a.lambda0, (T)a.gamma_w};
  switch (d.N) {
    case 64: row_go<64, T, GW, BS, SCH>(d, c, inst, tile, smem); break;
    case 128: row_go<128, T, GW, BS, SCH>(d, c, inst, tile, smem); break;
    case 256: row_go<256, T, GW, BS, SCH>(d, c, inst, tile, smem); break;
    case 512: row_go<512, T, GW, BS, SCH>(d, c, inst, tile, smem); break;
    case 1024: row_go<1024, T, GW, BS, SCH>(d, c, inst, tile, smem); break;
    default: break;
  }
}

template <int N, class T, class S, bool GW, int MODE, int BS, int SCH = kSchedDefault>
__device__ __forceinline__ void col_go(const ClassArgs& d, const LinCoef& lc, int inst, int tile,
                                       unsigned char* smem) {
  if constexpr (col_smem_n<T, BS, GW, N, SCH>() > 0) {
    LinCoef l = lc;
    l.dt_over_N = lc.dt / N;  // the unnormalised forward FFT carries N x the unitary DFT
    col_body<N, TileOf<N, BS>::R, T, S, GW, MODE, SCH>((const C2<T>*)d.Y, (C2<T>*)d.X_out, (C2<S>*)d.st,
                                                  (const T*)d.rowsum, d.dk, (const C2<T>*)d.tw, l,
                                                  inst, tile, smem, (C2<S>*)d.st2, (C2<T>*)d.fst, d.s1st);
  }
}

template <class T, class S, bool GW, int MODE, int BS, int SCH = kSchedDefault>
__global__ void __launch_bounds__(BS) col_multi(MultiArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int ci = class_of(a, b);
  const ClassArgs& d = a.c[ci];
  const int local = b - a.start[ci];
  const int inst = local / d.tiles;
  const int tile = local - inst * d.tiles;
  switch (d.N) {
    case 64: col_go<64, T, S, GW, MODE, BS, SCH>(d, a.lc, inst, tile, smem); break;
    case 128: col_go<128, T, S, GW, MODE, BS, SCH>(d, a.lc, inst, tile, smem); break;
    case 256: col_go<256, T, S, GW, MODE, BS, SCH>(d, a.lc, inst, tile, smem); break;
    case 512: col_go<512, T, S, GW, MODE, BS, SCH>(d, a.lc, inst, tile, smem); break;
    case 1024: col_go<1024, T, S, GW, MODE, BS, SCH>(d, a.lc, inst, tile, smem); break;
    default: break;
  }
}

// One size class per launch (args.c[0] only): the same tile bodies compiled
// for a single N, so that the register budget is that of this N alone and the
// tile decode is constant; the autotuner picks this or the multi-size launch.
// Grids of 2048 points are served only here (their tiles would raise the
// register budget of the multi-size kernels for every other size).
template <int N, class T, bool GW, int BS>
__global__ void __launch_bounds__(BS) row_one(MultiArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const ClassArgs& d = a.c[0];
  const int inst = b / d.tiles;
  const int tile = b - inst * d.tiles;
  const RowCoef<T> c{(T)a.beta, (T)a.gamma_v, (T)a.lambda0, (T)a.gamma_w};
  row_go<N, T, GW, BS>(d, c, inst, tile, smem);
}

template <int N, class T, class S, bool GW, int MODE, int BS>
__global__ void __launch_bounds__(BS) col_one(MultiArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const ClassArgs& d = a.c[0];
  const int inst = b / d.tiles;
  const int tile = b - inst * d.tiles;
  col_go<N, T, S, GW, MODE, BS>(d, a.lc, inst, tile, smem);
}

}  // namespace ttsh
