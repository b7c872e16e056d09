// Workgroup-level Stockham FFT staged through LDS, for gfx950.
//
// One transform of length N (64..2048, a power of two) is carried by TT = N/8
// threads of a workgroup; thread t holds the 8 elements t + e*TT (e = 0..7)
// in registers.  Each stage of radix R (8, or a final 4 or 2) reads its
// butterfly inputs x[i + r*N/R] from exactly those registers, multiplies by
// the twiddles w^(r*k) (k = i mod P, P the product of the earlier radices),
// does the radix-R DFT and scatters the outputs to y[(i-k)R + k + rP]
// (Stockham autosort, decimation in time; Van Loan, Computational Frameworks
// for the FFT, ch. 1.7).  Because the input stride N/R is the same in every
// stage, the scatter is followed by a gather of t + e*TT, and in the last stage
// (P = N/R) the scatter target is t + e*TT itself, so the output lands in the
// registers that held the input, in natural order.  A transform therefore
// costs (#stages - 1) LDS round trips and needs no bit reversal.
//
// NF independent transforms that share the same threads are processed
// together.  At most TTSH_FFT_SLOTS of them occupy LDS at a time: with as many
// slots as transforms one barrier pair per stage serves all of them; with
// fewer, the transforms take turns in the slots (one more barrier per extra
// transform and stage), which shrinks the LDS footprint of a transform group
// and lets more waves stay resident on a CU.
//
// All threads of the workgroup must call these functions (they contain
// workgroup barriers, or wavefront-scope ordering for one-wavefront
// workgroups); threads that carry no useful data just transform zeros.
#pragma once

#include "common.hpp"

namespace ttsh {

constexpr int kFftE = 8;  // elements per thread

// Schedule of a transform, one int SCH = 2 PAD + SMALL_FIRST:
//   PAD          the LDS index gets one pad slot every 2^PAD entries (breaks
//                the strided scatter of the stages across banks);
//   SMALL_FIRST  for N not a power of 8, whether the radix left over after
//                the radix-8 stages (2 or 4) runs as the first stage or the
//                last one.
// The default (one slot per 16, small radix last) was the fastest of the
// hand-measured settings on gfx950; the autotuner also tries PAD = 3, 5 and
// the small radix first for the time-step kernels.  The schedule changes
// neither the result's layout nor, for the padding, its arithmetic.
constexpr int sched_code(int pad, bool small_first) { return 2 * pad + (small_first ? 1 : 0); }
constexpr int kSchedDefault = sched_code(4, false);
constexpr int sched_pad(int sch) { return sch >> 1; }
constexpr bool sched_small_first(int sch) { return (sch & 1) != 0; }

template <int SCH = kSchedDefault>
__host__ __device__ constexpr int lds_pad(int j) { return j + (j >> sched_pad(SCH)); }
template <int N, int SCH = kSchedDefault>
struct Padded {
  static constexpr int value = N + (N >> sched_pad(SCH));
};

// radix of the stage that follows stages whose radices multiply to P
template <int N, int SCH>
constexpr int stage_radix(int P) {
  int l2 = 0;
  while ((1 << l2) < N) ++l2;
  const int small = 1 << (l2 % 3);  // 1, 2 or 4
  if (sched_small_first(SCH) && small > 1) return P == 1 ? small : 8;
  const int rem = N / P;
  return rem % 8 == 0 ? 8 : (rem % 4 == 0 ? 4 : 2);
}

#ifndef TTSH_FFT_SLOTS
#define TTSH_FFT_SLOTS 2
#endif
static_assert(TTSH_FFT_SLOTS >= 2, "the slot rotation needs at least two slots");
// LDS regions of Padded<N> entries that NF transforms use during an exchange
__host__ __device__ constexpr int fft_slots(int nf) { return nf < TTSH_FFT_SLOTS ? nf : TTSH_FFT_SLOTS; }

// ---- radix-R DFTs, DIR = -1 forward (e^{-2 pi i nk/R}), +1 inverse ---------
template <int DIR, class T>
__device__ __forceinline__ void dft4(C2<T>& a0, C2<T>& a1, C2<T>& a2, C2<T>& a3) {
  const C2<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3;
  const C2<T> t3 = mul_i<DIR>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <int R, int DIR, class T>
struct Dft;

template <int DIR, class T>
struct Dft<2, DIR, T> {
  __device__ static __forceinline__ void run(C2<T> (&u)[2]) {
    const C2<T> d = u[0] - u[1];
    u[0] = u[0] + u[1];
    u[1] = d;
  }
};

template <int DIR, class T>
struct Dft<4, DIR, T> {
  __device__ static __forceinline__ void run(C2<T> (&u)[4]) { dft4<DIR>(u[0], u[1], u[2], u[3]); }
};

template <int DIR, class T>
struct Dft<8, DIR, T> {
  __device__ static __forceinline__ void run(C2<T> (&u)[8]) {
    // even / odd halves, then combine with W8^k = e^{DIR 2 pi i k / 8}
    C2<T> e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6];
    C2<T> o0 = u[1], o1 = u[3], o2 = u[5], o3 = u[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    const T c = (T)0.70710678118654752440084436210484903928;
    const T d = (T)DIR;
    const C2<T> w1 = mk(c * (o1.x - d * o1.y), c * (d * o1.x + o1.y));
    const C2<T> w2 = mul_i<DIR>(o2);
    const C2<T> w3 = mk(c * (-o3.x - d * o3.y), c * (d * o3.x - o3.y));
    u[0] = e0 + o0;
    u[4] = e0 - o0;
    u[1] = e1 + w1;
    u[5] = e1 - w1;
    u[2] = e2 + w2;
    u[6] = e2 - w2;
    u[3] = e3 + w3;
    u[7] = e3 - w3;
  }
};

// Orders the LDS accesses between the stages of a transform group.  With
// WAVE, the group's workgroup is a single wavefront: the LDS unit executes one
// wavefront's instructions in issue order, so a store is seen by every later
// load of the same wavefront without a barrier or a wait for the store to
// complete; a wavefront-scope fence (which emits no instruction) keeps the
// compiler from moving the loads above the stores.  Otherwise a workgroup
// barrier.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// ---- one Stockham stage, recursing into the next ---------------------------
// v[f][e] holds element t + e*TT of transform f.  `lds` points at this group's
// fft_slots(NF) regions of Padded<N> entries each.  `tw[j]` = e^{-2 pi i j / N}.
template <int N, int DIR, int NF, int P, class T, int SCH, bool WAVE>
struct FftStage {
  static constexpr int E = kFftE;
  static constexpr int TT = N / E;
  static constexpr int R = stage_radix<N, SCH>(P);
  static_assert(R == 2 || R == 4 || R == 8, "radix");
  static constexpr int NB = E / R;  // butterflies per thread in this stage
  static constexpr bool LAST = (P * R == N);
  static constexpr int NP = Padded<N, SCH>::value;

  // twiddle multiplication and radix-R DFT of the NB butterflies of transform
  // f; the outputs go back to registers (last stage) or to LDS region `slot`
  __device__ static __forceinline__ void butterflies(C2<T> (&v)[NF][E], int f, C2<T>* slot, int t,
                                                     const C2<T>* __restrict__ tw) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = t + b * TT;
      const int k = i & (P - 1);
      C2<T> u[R];
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[f][b + r * NB];
      if constexpr (P > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C2<T> w = tw[r * k * (N / (P * R))];
          if constexpr (DIR > 0) w.y = -w.y;
          u[r] = cmul(u[r], w);
        }
      }
      Dft<R, DIR, T>::run(u);
      if constexpr (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[f][b + r * NB] = u[r];
      } else {
        const int j0 = (i - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) slot[lds_pad<SCH>(j0 + r * P)] = u[r];
      }
    }
  }

  __device__ static __forceinline__ void gather(C2<T> (&v)[NF][E], int f, const C2<T>* slot, int t) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[f][e] = slot[lds_pad<SCH>(t + e * TT)];
  }

  __device__ static __forceinline__ void run(C2<T> (&v)[NF][E], C2<T>* lds, int t,
                                             const C2<T>* __restrict__ tw) {
    constexpr int NS = fft_slots(NF);
    if constexpr (LAST) {
#pragma unroll
      for (int f = 0; f < NF; ++f) butterflies(v, f, lds, t, tw);
    } else if constexpr (NS == NF) {
#pragma unroll
      for (int f = 0; f < NF; ++f) butterflies(v, f, lds + f * NP, t, tw);
      lds_sync<WAVE>();
#pragma unroll
      for (int f = 0; f < NF; ++f) gather(v, f, lds + f * NP, t);
      lds_sync<WAVE>();
      FftStage<N, DIR, NF, P * R, T, SCH, WAVE>::run(v, lds, t, tw);
    } else {
      // transform f uses slot f % NS; the barrier after writing f also orders
      // every read of f - NS (issued before it) ahead of the reuse of its slot
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        butterflies(v, f, lds + (f % NS) * NP, t, tw);
        lds_sync<WAVE>();
        gather(v, f, lds + (f % NS) * NP, t);
      }
      lds_sync<WAVE>();
      FftStage<N, DIR, NF, P * R, T, SCH, WAVE>::run(v, lds, t, tw);
    }
  }
};

// Unnormalised transform(s): out[m] = sum_n in[n] e^{DIR 2 pi i m n / N}.
// WAVE: the calling workgroup is one wavefront (see lds_sync).
template <int N, int DIR, int NF, int SCH = kSchedDefault, bool WAVE = false, class T>
__device__ __forceinline__ void fft(C2<T> (&v)[NF][kFftE], C2<T>* lds, int t,
                                    const C2<T>* __restrict__ tw) {
  static_assert(N >= 64 && (N & (N - 1)) == 0, "N must be a power of two >= 64");
  FftStage<N, DIR, NF, 1, T, SCH, WAVE>::run(v, lds, t, tw);
}

}  // namespace ttsh
