// Full-array transforms used by the set-up and read-out paths: one length-N
// Stockham transform per row (contiguous) or per column (stride N) of a batch
// of N x N complex arrays, unnormalised, in place.
#pragma once

#include "fft.hpp"

namespace ttsh {

// ---- full-array transforms (unnormalised), rows contiguous ----------------
template <int N>
struct FullFft {
  static constexpr int TT = N / kFftE;
  static constexpr int RPB = TT >= 64 ? 1 : 64 / TT;              // rows per block
  static constexpr int CPB = (256 / TT) < 1 ? 1 : ((256 / TT) > 16 ? 16 : 256 / TT);  // columns per block
};

// rows: a [batch*N rows][N]; one transform per row, thread t of a row reads
// the contiguous elements t + e*TT
template <int N, int DIR, class T>
__global__ void __launch_bounds__(FullFft<N>::RPB*(N / 8))
fft_rows(C2<T>* __restrict__ a, int nrows, const C2<T>* __restrict__ tw) {
  constexpr int TT = FullFft<N>::TT, RPB = FullFft<N>::RPB, NP = Padded<N>::value;
  __shared__ C2<T> lds[RPB * NP];
  const int t = threadIdx.x % TT, lane = threadIdx.x / TT;
  const int row = blockIdx.x * RPB + lane;
  const bool ok = row < nrows;
  C2<T> v[1][kFftE];
#pragma unroll
  for (int e = 0; e < kFftE; ++e) v[0][e] = ok ? a[(size_t)row * N + t + e * TT] : mk<T>(0, 0);
  fft<N, DIR, 1>(v, lds + lane * NP, t, tw);
  if (ok)
#pragma unroll
    for (int e = 0; e < kFftE; ++e) a[(size_t)row * N + t + e * TT] = v[0][e];
}

// columns: a [batch][N][N]; consecutive threads take consecutive columns
template <int N, int DIR, class T>
__global__ void __launch_bounds__(FullFft<N>::CPB*(N / 8))
fft_cols(C2<T>* __restrict__ a, int ncols, const C2<T>* __restrict__ tw) {
  constexpr int TT = FullFft<N>::TT, CPB = FullFft<N>::CPB, NP = Padded<N>::value;
  __shared__ C2<T> lds[CPB * NP];
  const int lane = threadIdx.x % CPB, t = threadIdx.x / CPB;
  const int gc = blockIdx.x * CPB + lane;  // global column over the batch
  const bool ok = gc < ncols;
  const size_t base = (size_t)(gc / N) * N * N + (gc % N);
  C2<T> v[1][kFftE];
#pragma unroll
  for (int e = 0; e < kFftE; ++e) v[0][e] = ok ? a[base + (size_t)(t + e * TT) * N] : mk<T>(0, 0);
  fft<N, DIR, 1>(v, lds + lane * NP, t, tw);
  if (ok)
#pragma unroll
    for (int e = 0; e < kFftE; ++e) a[base + (size_t)(t + e * TT) * N] = v[0][e];
}

}  // namespace ttsh
