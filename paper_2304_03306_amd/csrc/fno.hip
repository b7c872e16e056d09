// Fourier-neural-operator surrogate on gfx950 (interface: include/fno.h).
//
// Every dense piece of the network goes through one strided, batched GEMM on
// the matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation): the pruned 2D DFTs as products with small DFT matrices (only
// m of W/2+1 k_x columns and 2m of H k_y rows are ever needed), the per-mode
// complex channel mixing as real block products [Re, Im] [[R_r, R_i],
// [-R_i, R_r]], the 1x1 convolutions, the projection and every weight
// gradient (split over chunks of the point axis, partial sums reduced in a
// fixed order).  A GEMM call may add a second product (A2 B2) and fuses bias,
// exact GELU, GELU' and the saving of pre-activations into its epilogue.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/fno.h"
#include "../../include/ttsh.h"
#include "common.hpp"
#include "launch.hpp"

namespace {

using bf16 = uint16_t;

// ---- BF16 <-> FP32 (round to nearest even) ---------------------------------------
__host__ __device__ inline bf16 f2bf(float f) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_bit_cast(bf16, (__bf16)f);  // v_cvt_pk_bf16_f32, round to nearest even
#else
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
#endif
}
typedef float float2v_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef unsigned uint2v_t __attribute__((ext_vector_type(2)));
// two values in one v_cvt_pk_bf16_f32 (round to nearest even), a in the low half
__device__ inline unsigned pack2(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(float2v_t{a, b}, bf16x2_t));
}
__host__ __device__ inline float bf2f(bf16 h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// erfc of a / sqrt(2) for a >= 0 by Abramowitz and Stegun, Handbook of
// Mathematical Functions, 7.1.28: erf(u) = 1 - (1 + a1 u + ... + a6 u^6)^-16,
// |error| <= 3e-7 (the coefficients below are a_i 2^{-i/2}, so that the
// polynomial takes a directly).  One reciprocal and no exponential; the
// activations it feeds are stored in BF16 (relative resolution 2^-8).
__device__ inline float erfc_half(float a) {
  constexpr double r = 0.70710678118654752440;
  constexpr float b1 = (float)(0.0705230784 * r), b2 = (float)(0.0422820123 * r * r),
                  b3 = (float)(0.0092705272 * r * r * r), b4 = (float)(0.0001520143 * r * r * r * r),
                  b5 = (float)(0.0002765672 * r * r * r * r * r), b6 = (float)(0.0000430638 * r * r * r * r * r * r);
  const float p = fmaf(a, fmaf(a, fmaf(a, fmaf(a, fmaf(a, fmaf(a, b6, b5), b4), b3), b2), b1), 1.0f);
  const float q = __builtin_amdgcn_rcpf(p), q2 = q * q, q4 = q2 * q2, q8 = q4 * q4;
  return q8 * q8;
}
// Phi(x) = (1 + erf(x / sqrt 2)) / 2, the standard normal distribution
__device__ inline float norm_cdf(float x) {
  const float h = 0.5f * erfc_half(fabsf(x));
  return x >= 0.f ? 1.0f - h : h;
}
// Phi(-a) = erfc(a / sqrt 2) / 2 for a >= 0, the same formula with the factor
// 1/2 taken into the polynomial: (2^{1/16} p)^-16 = p^-16 / 2, so the
// coefficients are 2^{1/16} times those of erfc_half
__device__ inline float half_erfc_half(float a) {
  constexpr double r = 0.70710678118654752440, s = 1.04427378242741384032;  // 2^(1/16)
  constexpr float c0 = (float)s, c1 = (float)(s * 0.0705230784 * r), c2 = (float)(s * 0.0422820123 * r * r),
                  c3 = (float)(s * 0.0092705272 * r * r * r), c4 = (float)(s * 0.0001520143 * r * r * r * r),
                  c5 = (float)(s * 0.0002765672 * r * r * r * r * r),
                  c6 = (float)(s * 0.0000430638 * r * r * r * r * r * r);
  const float p = fmaf(a, fmaf(a, fmaf(a, fmaf(a, fmaf(a, fmaf(a, c6, c5), c4), c3), c2), c1), c0);
  const float q = __builtin_amdgcn_rcpf(p), q2 = q * q, q4 = q2 * q2, q8 = q4 * q4;
  return q8 * q8;
}
// exact (erf) GELU x Phi(x) = max(x, 0) - |x| Phi(-|x|) (for x < 0, x Phi(x) =
// -|x| Phi(-|x|); for x >= 0, x (1 - Phi(-x))): one max and one fma around the
// tail probability; and its derivative Phi(x) + x phi(x)
__device__ inline float gelu(float x) {
  const float a = fabsf(x);
  return fmaf(-a, half_erfc_half(a), fmaxf(x, 0.f));
}
__device__ inline float gelu_grad(float x) {
  return norm_cdf(x) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

// ---- GEMM -------------------------------------------------------------------------------
struct Op {
  const bf16* p;
  long long s1, s2, r, c;  // batch strides (b1, b2), row stride, column stride
  int kvec;                // set by the launcher: runs of 4 along k are contiguous and 8-byte aligned
};

struct GemmArgs {
  int M, N, K, K2;
  int nb1, nb2;            // batch = b1 * nb2 + b2
  Op A, B, A2, B2;         // C = alpha A B + alpha2 A2 B2
  float alpha, alpha2;
  void* C;
  long long sC1, sC2, rC, cC;
  int c_bf16;              // C element type: 1 bf16, 0 float
  int accumulate;          // float C only: C += result
  const float* bias;       // per column, added before the activation
  int act;                 // 0 none, 1 GELU, 2 multiply by GELU'(pre_in)
  const bf16* pre_in;      // act 2: pre-activations (same strides as C)
  bf16* pre_out;           // act 1: store the pre-activation (same strides as C)
  const float* skip;       // float C only: C[i][j] += skip[i * skip_r + j] (after everything else)
  long long skip_r;
  int vecC;                // set by the launcher: rows of C hold aligned runs of 4 contiguous columns
  int staged;              // set by the launcher: -1 direct loads, else 2 FA + FB of gemm_part_lds
};

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef short short8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
__device__ inline short4_t pack4(float a, float b, float c, float d) {
  return __builtin_bit_cast(short4_t, uint2v_t{pack2(a, b), pack2(c, d)});
}
// The matrix-core products.  gfx950's v_mfma_f32_16x16x32_bf16 (mfma32)
// takes 32 along k per instruction, eight per lane: lane l holds row l%16 of
// the first operand and column l%16 of the second, both at the eight k slots
// of lane group l/16, and receives rows 4(l/16)..+3 of column l%16 of the
// 16 x 16 result.  Which k a slot carries is the caller's choice, as long as
// both operands agree: most callers give group g the run k = 8g..8g+7 (one
// 16-byte load per operand); where an operand is the result of an earlier
// product (four consecutive rows per lane), the two halves of a slot group
// are the two 16-row halves, k = 4g..4g+3 and 16+4g..16+4g+3 (cat8).  The
// 16-deep form (mfma16: k = 4(l/16)..+3) serves only contractions that are
// 16 deep.
__device__ inline float4_t mfma32(short8_t a, short8_t b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}
__device__ inline float4_t mfma16(short4_t a, short4_t b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline short8_t cat8(short4_t lo, short4_t hi) {
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ inline short4_t load_frag(const bf16* base, long long r, long long c, int row, int k0,
                                     int nrow, int K, int kvec) {
  if (kvec && row < nrow && k0 + 3 < K) return *(const short4_t*)(base + (long long)row * r + k0);
  short4_t v;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = k0 + q;
    v[q] = (row < nrow && k < K) ? (short)base[(long long)row * r + (long long)k * c] : (short)0;
  }
  return v;
}

// One wavefront computes one 32 x 32 tile of C as 2 x 2 MFMA 16 x 16 blocks,
// 32 along k per step (lane group g: k = k0 + 8g..+7, zero past K).  The
// product is formed transposed (C^T = B^T A^T: the B fragment goes first), so
// that lane l ends up with row l%16 of the block and four consecutive columns
// 4(l/16)..+3: one vector store per block when C's columns are contiguous.
__device__ inline void gemm_part(const Op& A, const Op& B, int K, int M, int N, int b1, int b2,
                                 int i0, int j0, int lane, float4_t (&acc)[2][2]) {
  const bf16* pa = A.p + b1 * A.s1 + b2 * A.s2;
  const bf16* pb = B.p + b1 * B.s1 + b2 * B.s2;
  const int rl = lane & 15, kq = (lane >> 4) * 8;
  for (int k0 = 0; k0 < K; k0 += 32) {
    short8_t a[2], b[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      a[s] = cat8(load_frag(pa, A.r, A.c, i0 + 16 * s + rl, k0 + kq, M, K, A.kvec),
                  load_frag(pa, A.r, A.c, i0 + 16 * s + rl, k0 + kq + 4, M, K, A.kvec));
      // B[k][j]: treat as rows j with stride B.c, columns k with stride B.r
      b[s] = cat8(load_frag(pb, B.c, B.r, j0 + 16 * s + rl, k0 + kq, N, K, B.kvec),
                  load_frag(pb, B.c, B.r, j0 + 16 * s + rl, k0 + kq + 4, N, K, B.kvec));
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[s][t] = mfma32(b[t], a[s], acc[s][t]);
  }
}

// The same product with both operands staged through the wavefront's own LDS
// in chunks of 32 along k, read from HBM with coalesced 16-byte loads along
// whichever dimension is contiguous: FA = 0 when A's rows run along k, 1 when
// its columns do (A given transposed); FB = 0 when B's rows run along n, 1
// when along k.  LDS holds A as [m][k] and B as [n][k] (k contiguous, what the
// MFMA fragments read 8 at a time), so the operands whose memory runs along
// the other dimension are transposed on their way in.  The launcher checks
// unit strides, multiples of 8 and 16-byte alignment.
constexpr int kKC = 32, kLDK = 40;  // k chunk, LDS row stride (bf16) with padding
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// stage a 32 x 32 block: rows `lo` (m or n, limit `nlo`) and k from k0 (limit
// K) of an operand whose element (row, k) sits at base + row * rs + k * ks;
// KRUN: the 16-byte runs go along k (ks == 1), else along rows (rs == 1)
template <bool KRUN>
__device__ inline void stage_block(const bf16* __restrict__ base, long long rs, long long ks, int lo, int nlo, int k0,
                                   int K, int lane, bf16* __restrict__ dst) {
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int a = pass * 16 + (lane >> 2), seg = (lane & 3) * 8;
    uint4 v = {0u, 0u, 0u, 0u};
    if constexpr (KRUN) {  // a = row, seg = k offset
      if (lo + a < nlo && k0 + seg < K) v = *(const uint4*)(base + (long long)(lo + a) * rs + k0 + seg);
      *(uint4*)(dst + a * kLDK + seg) = v;
    } else {  // a = k offset, seg = row offset
      if (k0 + a < K && lo + seg < nlo) v = *(const uint4*)(base + (long long)(k0 + a) * ks + lo + seg);
      const bf16* e = (const bf16*)&v;
#pragma unroll
      for (int q = 0; q < 8; ++q) dst[(seg + q) * kLDK + a] = e[q];
    }
  }
}
template <int FA, int FB>
__device__ inline void gemm_part_lds(const Op& A, const Op& B, int K, int M, int N, int b1, int b2, int i0, int j0,
                                     int lane, float4_t (&acc)[2][2], bf16* __restrict__ As,
                                     bf16* __restrict__ Bt) {
  const bf16* pa = A.p + b1 * A.s1 + b2 * A.s2;
  const bf16* pb = B.p + b1 * B.s1 + b2 * B.s2;
  const int rl = lane & 15, kq = (lane >> 4) * 8;
  for (int k0 = 0; k0 < K; k0 += kKC) {
    // A(i, k) at pa + i * A.r + k * A.c;  B(k, j) at pb + k * B.r + j * B.c
    stage_block<FA == 0>(pa, A.r, A.c, i0, M, k0, K, lane, As);
    stage_block<FB == 1>(pb, B.c, B.r, j0, N, k0, K, lane, Bt);
    wave_lds_sync();
    short8_t a[2], b[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      a[s] = *(const short8_t*)(As + (16 * s + rl) * kLDK + kq);
      b[s] = *(const short8_t*)(Bt + (16 * s + rl) * kLDK + kq);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[s][t] = mfma32(b[t], a[s], acc[s][t]);
    wave_lds_sync();  // the next chunk overwrites the staging buffers
  }
}

// Work items (batch, tile) are numbered batch-major and dealt four to a
// workgroup, one per wavefront, so that GEMMs with a single tile per batch
// still fill every wavefront.
// STAGED: -1 direct loads; else 2 * FA + FB of the LDS-staged form
template <int STAGED>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g, int tiles_n, int tiles) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long nbatch = (long long)g.nb1 * g.nb2;
  const long long item = (long long)blockIdx.x * 4 + wave;
  if (item >= nbatch * tiles) return;  // whole wavefront exits together
  const long long batch = item / tiles;
  const int tile = (int)(item % tiles);
  const int b1 = (int)(batch / g.nb2), b2 = (int)(batch % g.nb2);
  const int i0 = (tile / tiles_n) * 32, j0 = (tile % tiles_n) * 32;
  float4_t acc[2][2], acc2[2][2];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      acc[s][t] = float4_t{0.f, 0.f, 0.f, 0.f};
      acc2[s][t] = float4_t{0.f, 0.f, 0.f, 0.f};
    }
  if constexpr (STAGED >= 0) {
    constexpr int FA = STAGED >> 1, FB = STAGED & 1;
    __shared__ __align__(16) bf16 stage[4][2][32 * kLDK];
    gemm_part_lds<FA, FB>(g.A, g.B, g.K, g.M, g.N, b1, b2, i0, j0, lane, acc, stage[wave][0], stage[wave][1]);
    if (g.K2 > 0)
      gemm_part_lds<FA, FB>(g.A2, g.B2, g.K2, g.M, g.N, b1, b2, i0, j0, lane, acc2, stage[wave][0],
                            stage[wave][1]);
  } else {
    gemm_part(g.A, g.B, g.K, g.M, g.N, b1, b2, i0, j0, lane, acc);
    if (g.K2 > 0) gemm_part(g.A2, g.B2, g.K2, g.M, g.N, b1, b2, i0, j0, lane, acc2);
  }
  const long long cbase = b1 * g.sC1 + b2 * g.sC2;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int i = i0 + 16 * s + (lane & 15);
      const int jb = j0 + 16 * t + (lane >> 4) * 4;
      if (i >= g.M || jb >= g.N) continue;
      const long long ob = cbase + (long long)i * g.rC + (long long)jb * g.cC;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = jb + e;
        v[e] = 0.f;
        if (j >= g.N) continue;
        const long long off = ob + (long long)e * g.cC;
        float x = g.alpha * acc[s][t][e] + (g.K2 > 0 ? g.alpha2 * acc2[s][t][e] : 0.f);
        if (g.accumulate) x += ((float*)g.C)[off];
        if (g.bias) x += g.bias[j];
        if (g.act == 1) {
          if (g.pre_out) g.pre_out[off] = f2bf(x);
          x = gelu(x);
        } else if (g.act == 2) {
          x *= gelu_grad(bf2f(g.pre_in[off]));
        }
        if (g.skip) x += g.skip[(long long)i * g.skip_r + j];
        v[e] = x;
      }
      if (g.vecC && jb + 3 < g.N) {
        if (g.c_bf16) {
          uint2 o;
          o.x = pack2(v[0], v[1]);
          o.y = pack2(v[2], v[3]);
          *(uint2*)((bf16*)g.C + ob) = o;
        } else {
          *(float4*)((float*)g.C + ob) = make_float4(v[0], v[1], v[2], v[3]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (jb + e >= g.N) continue;
          const long long off = ob + (long long)e * g.cC;
          if (g.c_bf16)
            ((bf16*)g.C)[off] = f2bf(v[e]);
          else
            ((float*)g.C)[off] = v[e];
        }
      }
    }
}

hipError_t gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipErrorInvalidValue;
  const int tiles_n = (g.N + 31) / 32, tiles = ((g.M + 31) / 32) * tiles_n;
  const long long blocks = ((long long)g.nb1 * g.nb2 * tiles + 3) / 4;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (g.staged) {
    case 0: hipLaunchKernelGGL(gemm_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, s, g, tiles_n, tiles); break;
    case 1: hipLaunchKernelGGL(gemm_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s, g, tiles_n, tiles); break;
    case 2: hipLaunchKernelGGL(gemm_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, g, tiles_n, tiles); break;
    case 3: hipLaunchKernelGGL(gemm_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, s, g, tiles_n, tiles); break;
    default: hipLaunchKernelGGL(gemm_kernel<-1>, dim3((unsigned)blocks), dim3(256), 0, s, g, tiles_n, tiles);
  }
  return hipGetLastError();
}

// Form (0 or 1) in which an operand can be staged through LDS, -1 if none:
// its 16-byte runs go along `first` (the row dimension m of A / k of B: form
// 0 for A means runs along k) -- see gemm_part_lds.  `run` is the stride of
// the contiguous dimension (1), `other` the other stride; the contiguous
// dimension's extent must be a multiple of 8.
int stage_form(const Op& o, bool is_a, int M_or_N, int K) {
  if (((uintptr_t)o.p & 15) || o.s1 % 8 || o.s2 % 8) return -1;
  // A(i, k) = p[i r + k c]; B(k, j) = p[k r + j c]
  const long long kstride = is_a ? o.c : o.r, xstride = is_a ? o.r : o.c;
  if (kstride == 1 && xstride % 8 == 0 && K % 8 == 0) return is_a ? 0 : 1;  // runs along k
  if (xstride == 1 && kstride % 8 == 0 && M_or_N % 8 == 0) return is_a ? 1 : 0;  // runs along m / n
  return -1;
}
// staged form of a whole GEMM (both products share it), -1 if not stageable
int staged_form(const GemmArgs& g) {
  const int fa = stage_form(g.A, true, g.M, g.K), fb = stage_form(g.B, false, g.N, g.K);
  if (fa < 0 || fb < 0) return -1;
  if (g.K2 > 0 && (stage_form(g.A2, true, g.M, g.K2) != fa || stage_form(g.B2, false, g.N, g.K2) != fb)) return -1;
  return 2 * fa + fb;
}

Op op(const bf16* p, long long r, long long c, long long s1 = 0, long long s2 = 0) { return Op{p, s1, s2, r, c, 0}; }

// k runs of 4 are one aligned 8-byte load when the k stride is 1 and every
// other stride and the base keep 4-element alignment
int kvec_ok(const Op& o, bool a_side) {
  const long long ks = a_side ? o.c : o.r, rs = a_side ? o.r : o.c;
  return ks == 1 && rs % 4 == 0 && o.s1 % 4 == 0 && o.s2 % 4 == 0 && ((uintptr_t)o.p & 7) == 0;
}



// ---- element-wise kernels ------------------------------------------------------------------
// y[j][i] = x[i][j] for an n x n matrix
__global__ void k_transpose_bf16(const float* __restrict__ x, bf16* __restrict__ y, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) y[(i % n) * n + i / n] = f2bf(x[i]);
}
__global__ void k_to_bf16(const float* __restrict__ x, bf16* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// h0[p][c] = sum_k x[p][k] P_w[k][c] + P_b[c]  (cin is small: vector ALU)
__global__ void k_lift(const bf16* __restrict__ x, const bf16* __restrict__ Pw,
                       const float* __restrict__ Pb, bf16* __restrict__ h, long long npts, int cin, int C) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts * C) return;
  const long long p = i / C;
  const int c = (int)(i % C);
  float v = Pb[c];
  for (int k = 0; k < cin; ++k) v += bf2f(x[p * cin + k]) * bf2f(Pw[k * C + c]);
  h[i] = f2bf(v);
}

// the same with one thread per point and 8 channels (C % 8 == 0): 16-byte stores
__global__ void k_lift8(const bf16* __restrict__ x, const bf16* __restrict__ Pw, const float* __restrict__ Pb,
                        bf16* __restrict__ h, long long npts, int cin, int C) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int groups = C / 8;
  if (i >= npts * groups) return;
  const long long p = i / groups;
  const int c0 = (int)(i % groups) * 8;
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = Pb[c0 + e];
  for (int k = 0; k < cin; ++k) {
    const float xk = bf2f(x[p * cin + k]);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] += xk * bf2f(Pw[k * C + c0 + e]);
  }
  uint4 o;
  o.x = pack2(v[0], v[1]);
  o.y = pack2(v[2], v[3]);
  o.z = pack2(v[4], v[5]);
  o.w = pack2(v[6], v[7]);
  *(uint4*)(h + p * C + c0) = o;
}

// Inference projection fused in one pass, so that the hidden layer stays in
// registers: y[p][o] = sum_k GELU(u[p][k]) Q2[k][o] + Q2_b[o] (+ skip[p][o]),
// u = h Q1 + Q1_b.  Computed transposed on the matrix cores (u^T = Q1^T h^T,
// then y^T = Q2^T a^T) because the result layout of the first product (lane =
// point column, 4 consecutive hidden rows) is exactly the operand layout the
// second one needs.  A wavefront handles G groups of 16 points per iteration.
#ifndef FNO_PROJ_GROUPS
#define FNO_PROJ_GROUPS 4
#endif
constexpr int kProjGroups = FNO_PROJ_GROUPS;  // groups of 16 points per wavefront and iteration
template <int C, int HID, int G>
__global__ void __launch_bounds__(256) k_proj_fused(const bf16* __restrict__ h, const bf16* __restrict__ Q1,
                                                    const float* __restrict__ b1, const bf16* __restrict__ Q2,
                                                    const float* __restrict__ b2, int cout, float* __restrict__ y,
                                                    long long ys, const float* __restrict__ skip, long long skip_r,
                                                    long long npts) {
  // k slots: the first product runs over channels k = 32 kb + 8 g + e; the
  // second over the hidden pair (2 P, 2 P + 1) of 16-row blocks, slot (g, e)
  // carrying hidden row 32 P + 16 (e / 4) + 4 g + e % 4 (what two results of
  // the first product hold, cat8)
  static_assert(C % 32 == 0 && HID % 32 == 0, "k in steps of 32");
  constexpr int HB = HID / 16, KB = C / 32;
  const int lane = threadIdx.x & 63, l16 = lane & 15, g4 = lane >> 4, q4 = g4 * 4, q8 = g4 * 8;
  const long long wave = (long long)blockIdx.x * 4 + (threadIdx.x >> 6), nwave = (long long)gridDim.x * 4;
  short8_t qa[HB][KB], qb[HB / 2];
  float bias1[HB][4];
#pragma unroll
  for (int hb = 0; hb < HB; ++hb) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int e = 0; e < 8; ++e) qa[hb][kb][e] = (short)Q1[(32 * kb + q8 + e) * HID + 16 * hb + l16];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      bias1[hb][e] = b1[16 * hb + q4 + e];
      qb[hb / 2][4 * (hb & 1) + e] = l16 < cout ? (short)Q2[(16 * hb + q4 + e) * cout + l16] : (short)0;
    }
  }
  // G independent groups of 16 points per iteration, for instruction-level
  // parallelism between their MFMA and GELU chains
  for (long long t = wave * G; t * 16 < npts; t += nwave * G) {
    long long p[G];
    bool ok[G];
    short8_t hv[G][KB];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      p[g] = (t + g) * 16 + l16;
      ok[g] = p[g] < npts;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        hv[g][kb] = ok[g] ? *(const short8_t*)(h + p[g] * C + 32 * kb + q8) : short8_t{0, 0, 0, 0, 0, 0, 0, 0};
    }
    float4_t acc2[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc2[g] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int hp = 0; hp < HB / 2; ++hp) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        short4_t av[2];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int hb = 2 * hp + hh;
          float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) acc = mfma32(qa[hb][kb], hv[g][kb], acc);
          // the bias is added after the product, as the unfused path does
          av[hh] = pack4(gelu(acc[0] + bias1[hb][0]), gelu(acc[1] + bias1[hb][1]), gelu(acc[2] + bias1[hb][2]),
                         gelu(acc[3] + bias1[hb][3]));
        }
        acc2[g] = mfma32(qb[hp], cat8(av[0], av[1]), acc2[g]);
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int o = q4 + e;
        if (ok[g] && o < cout) {
          float v = acc2[g][e] + b2[o];
          if (skip) v += skip[p[g] * skip_r + o];
          y[p[g] * ys + o] = v;
        }
      }
  }
}

// Tail of one Fourier layer for C = 32 channels, 2m = 32 kept k_x rows and
// W = 128 points per image row, fused so that the new activation row is used
// while it is on chip.  A workgroup takes one image row (b, y) per iteration,
// its four wavefronts 32 points x each:
//   out[x][c] = act(sum_j Ax[x][j] T2[b][y][j][c] + sum_k h[b][y][x][k] Wl[k][c] + bias[c])
// stored to hn[b][y][x][c] (the pre-activation to z[b][y][x][c] when z is
// given), and with NEXT the next layer's truncated k_x transform of that row,
//   T1[b][j][y][c] = sum_x Dx[j][x] out_bf16[x][c],
// from the rounded values that were stored (the same operand the separate
// analysis GEMM reads back).  The four wavefronts' partial sums over their 32
// points are added in a fixed order.  The product is formed untransposed, so
// that lane l holds column c = l%16 and four consecutive points: exactly the
// operand layout of the Dx product; the stores go through LDS to 32-byte rows.
// With LIFT the row is instead the lifting layer's output: h is the input
// x[b][y][x][k] (cin <= 16 channels), Wl the lifting weights Pw[k][c] and bias
// Pb, out = Pb + sum_k x[k] Pw[k][c], one MFMA k step with k padded to 16.
// With DGRAD it is the backward of a layer: out = Ax1 T2 + dz Wl^T (Wl given
// transposed, no bias) is the gradient with respect to the previous layer's
// output, rounded to BF16 and multiplied by GELU'(zin) of that layer's stored
// pre-activation: the next gradient dz, stored to hn, whose k_x transform
// with DxG (passed as Dx) is formed as above.
constexpr int kMaxLiftCin = 16;
template <bool ACT, bool NEXT, bool LIFT, bool DGRAD = false, bool CSUM = false>
__global__ void __launch_bounds__(256, CSUM ? 4 : 1) k_layer_tail(const bf16* __restrict__ h, const bf16* __restrict__ T2,
                                                    const bf16* __restrict__ Ax, const bf16* __restrict__ Wl,
                                                    const float* __restrict__ bias, const bf16* __restrict__ Dx,
                                                    bf16* __restrict__ hn, bf16* __restrict__ z,
                                                    bf16* __restrict__ T1, int H, long long rows, int cin,
                                                    const bf16* __restrict__ zin = nullptr,
                                                    float* __restrict__ csum = nullptr) {
  constexpr int C = 32, J = 32, W = 128;
  __shared__ __align__(16) bf16 Ts[C * kLDK];      // T2 block transposed: [c][j]
  __shared__ __align__(16) bf16 Os[4][32 * kLDK];  // per wavefront output tile [x][c]
  __shared__ float Rs[NEXT ? 4 : 1][J][C + 1];     // partial k_x transforms [wave][j][c]
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, l16 = lane & 15, q4 = (lane >> 4) * 4;
  const int q8 = (lane >> 4) * 8;
  const int tid = threadIdx.x;
  // row-independent operands, held in registers.  k slots: j = q8..q8+7 for
  // Ax, channels q8..q8+7 for Wl; for Dx the points 32 w + {q4..q4+3,
  // 16+q4..16+q4+3}, the two result halves the k_x transform takes (cat8)
  short8_t a1[2], b2[2], a3[2];
  short4_t pw[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if constexpr (!LIFT) {
      a1[s] = *(const short8_t*)(Ax + (32 * w + 16 * s + l16) * J + q8);
#pragma unroll
      for (int e = 0; e < 8; ++e) b2[s][e] = (short)Wl[(q8 + e) * C + 16 * s + l16];
    }
    if constexpr (NEXT)
      a3[s] = cat8(*(const short4_t*)(Dx + (16 * s + l16) * W + 32 * w + q4),
                   *(const short4_t*)(Dx + (16 * s + l16) * W + 32 * w + 16 + q4));
  }
  float bc[2], cs[2] = {0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    bc[t] = (DGRAD || !bias) ? 0.f : bias[16 * t + l16];
    if constexpr (LIFT) {
#pragma unroll
      for (int e = 0; e < 4; ++e) pw[t][e] = q4 + e < cin ? (short)Wl[(q4 + e) * C + 16 * t + l16] : (short)0;
    }
  }

  // Without LIFT, the next row's activation fragments and T2 piece are loaded
  // at the top of each iteration (into a2n, t2n), so that their latency
  // overlaps the current row's work instead of starting each iteration.
  const int tj = tid >> 3, tc0 = (tid & 7) * 4;  // this thread's piece of T2[b][y]
  short8_t a2n[2];
  uint2 t2n = {0u, 0u};
  if constexpr (!LIFT) {
    const long long r0 = blockIdx.x;
    if (r0 < rows) {
      const bf16* hp = h + r0 * (W * C);
#pragma unroll
      for (int s = 0; s < 2; ++s) a2n[s] = *(const short8_t*)(hp + (32 * w + 16 * s + l16) * C + q8);
      t2n = *(const uint2*)(T2 + r0 * (J * C) + tj * C + tc0);
    }
  }
  for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
    float4_t acc[2][2];
    if constexpr (LIFT) {
      __syncthreads();  // the previous row's reads of Rs are done before it is rewritten
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16* xr = h + (row * W + 32 * w + 16 * s + l16) * cin;
        short4_t xa;
#pragma unroll
        for (int e = 0; e < 4; ++e) xa[e] = q4 + e < cin ? (short)xr[q4 + e] : (short)0;
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[s][t] = mfma16(xa, pw[t], float4_t{0.f, 0.f, 0.f, 0.f});
      }
    } else {
      short8_t a2[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) a2[s] = a2n[s];
      const uint2 v = t2n;
      const long long rn = row + gridDim.x;
      if (rn < rows) {
        const bf16* hp = h + rn * (W * C);
#pragma unroll
        for (int s = 0; s < 2; ++s) a2n[s] = *(const short8_t*)(hp + (32 * w + 16 * s + l16) * C + q8);
        t2n = *(const uint2*)(T2 + rn * (J * C) + tj * C + tc0);
      }
      {  // T2[b][y] (J x C) into LDS as [c][j]
        const bf16* e = (const bf16*)&v;
#pragma unroll
        for (int q = 0; q < 4; ++q) Ts[(tc0 + q) * kLDK + tj] = e[q];
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const short8_t b1 = *(const short8_t*)(Ts + (16 * t + l16) * kLDK + q8);
          acc[s][t] = mfma32(a1[s], b1, float4_t{0.f, 0.f, 0.f, 0.f});
          acc[s][t] = mfma32(a2[s], b2[t], acc[s][t]);
        }
    }
    // acc[s][t][e] = out[x = 32 w + 16 s + q4 + e][c = 16 t + l16]
    bf16* Ow = Os[w];
    bf16* hrow = hn + row * (W * C) + 32 * w * C;
    const int sr = lane >> 1, sh = (lane & 1) * 16;  // store: tile row, first channel
    if (z) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int e = 0; e < 4; ++e) Ow[(16 * s + q4 + e) * kLDK + 16 * t + l16] = f2bf(acc[s][t][e] + bc[t]);
      wave_lds_sync();
      bf16* zrow = z + row * (W * C) + 32 * w * C;
      *(uint4*)(zrow + sr * C + sh) = *(const uint4*)(Ow + sr * kLDK + sh);
      *(uint4*)(zrow + sr * C + sh + 8) = *(const uint4*)(Ow + sr * kLDK + sh + 8);
      wave_lds_sync();
    }
    if constexpr (DGRAD) {  // the wavefront's 32 x 32 tile of zin into Ow, 16-byte runs
      const bf16* zr = zin + row * (W * C) + 32 * w * C;
      *(uint4*)(Ow + sr * kLDK + sh) = *(const uint4*)(zr + sr * C + sh);
      *(uint4*)(Ow + sr * kLDK + sh + 8) = *(const uint4*)(zr + sr * C + sh + 8);
      wave_lds_sync();
    }
    short4_t b3[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float v = acc[s][t][e] + bc[t];
          if constexpr (ACT) v = gelu(v);
          if constexpr (DGRAD)
            v = bf2f(f2bf(v)) * gelu_grad(bf2f(Ow[(16 * s + q4 + e) * kLDK + 16 * t + l16]));
          b3[s][t][e] = (short)f2bf(v);
        }
    if constexpr (DGRAD) wave_lds_sync();  // zin read before the tile is overwritten
    if constexpr (CSUM) {  // this lane's channels 16 t + l16, the stored (rounded) values in point order
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int e = 0; e < 4; ++e) cs[t] += bf2f((bf16)b3[s][t][e]);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) Ow[(16 * s + q4 + e) * kLDK + 16 * t + l16] = (bf16)b3[s][t][e];
    wave_lds_sync();
    *(uint4*)(hrow + sr * C + sh) = *(const uint4*)(Ow + sr * kLDK + sh);
    *(uint4*)(hrow + sr * C + sh + 8) = *(const uint4*)(Ow + sr * kLDK + sh + 8);
    if constexpr (NEXT) {
      // partial transform over this wavefront's 32 points: p[r][t][e] = P[16 r + q4 + e][16 t + l16]
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const float4_t p = mfma32(a3[r], cat8(b3[0][t], b3[1][t]), float4_t{0.f, 0.f, 0.f, 0.f});
#pragma unroll
          for (int e = 0; e < 4; ++e) Rs[w][16 * r + q4 + e][16 * t + l16] = p[e];
        }
      __syncthreads();
      const int j = tid >> 3, c0 = (tid & 7) * 4;
      const long long b = row / H, y = row % H;
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = ((Rs[0][j][c0 + q] + Rs[1][j][c0 + q]) + Rs[2][j][c0 + q]) + Rs[3][j][c0 + q];
      uint2 o;
      o.x = pack2(v[0], v[1]);
      o.y = pack2(v[2], v[3]);
      *(uint2*)(T1 + ((b * J + j) * H + y) * C + c0) = o;
    } else {
      __syncthreads();  // Ts is overwritten by the next row
    }
    wave_lds_sync();  // Os is overwritten by the next row
  }
  if constexpr (CSUM) {
    // column sums of everything this workgroup stored: the four lane groups of a
    // wavefront, then the four wavefronts in order, into csum[blockIdx.x][C]
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      cs[t] += __shfl_xor(cs[t], 16);
      cs[t] += __shfl_xor(cs[t], 32);
    }
    __syncthreads();  // every wavefront is done with Rs
    float* cw = &Rs[0][0][0];
    if (lane < 16) {
      cw[w * C + l16] = cs[0];
      cw[w * C + 16 + l16] = cs[1];
    }
    __syncthreads();
    if (tid < C) csum[(long long)blockIdx.x * C + tid] = ((cw[tid] + cw[C + tid]) + cw[2 * C + tid]) + cw[3 * C + tid];
  }
}

// The last Fourier layer's tail fused with the projection (C = 32, 2m = 32,
// W = 128, hidden HID): per image row (b, y) and wavefront (32 points x),
//   out[x][c] = sum_j Ax[x][j] T2[b][y][j][c] + sum_k h[b][y][x][k] Wl[k][c] + bias[c]
// (the last layer has no activation) is rounded to BF16 into the wavefront's
// LDS tile -- the values the unfused path stores as h_L -- and stored to hn
// only when hn is given (the training backward reads h_L); then, for the two
// groups of 16 points, y[p][o] = sum_j GELU(u[p][j]) Q2[j][o] + b2[o] (+ skip)
// with u = out Q1 + b1, formed as k_proj_fused forms it (same products and
// order, so the two paths give the same bits).  The projection's GELUs bound
// the kernel; the tail's memory traffic runs beneath them and h_L makes no
// round trip through memory.
template <int HID>
__global__ void __launch_bounds__(256, 3) k_tail_proj(const bf16* __restrict__ h, const bf16* __restrict__ T2,
                                                   const bf16* __restrict__ Ax, const bf16* __restrict__ Wl,
                                                   const float* __restrict__ bias, bf16* __restrict__ hn,
                                                   const bf16* __restrict__ Q1, const float* __restrict__ b1,
                                                   const bf16* __restrict__ Q2, const float* __restrict__ b2,
                                                   int cout, float* __restrict__ y, long long ys,
                                                   const float* __restrict__ skip, long long skip_r, long long rows) {
  constexpr int C = 32, J = 32, W = 128, HB = HID / 16;
  static_assert(HID % 32 == 0, "hidden width in steps of 32");
  __shared__ __align__(16) bf16 Ts[C * kLDK];      // T2 block transposed: [c][j]
  __shared__ __align__(16) bf16 Os[4][32 * kLDK];  // per wavefront output tile [x][c]
  __shared__ __align__(16) float B1s[HID];          // the hidden layer's bias
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, l16 = lane & 15, q4 = (lane >> 4) * 4;
  const int q8 = (lane >> 4) * 8;
  const int tid = threadIdx.x;
  // the tail's operands (k slots as in k_layer_tail) and the projection's (as in k_proj_fused)
  short8_t ax[2], wl[2], qa[HB], qb[HB / 2];
  float bc[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    ax[s] = *(const short8_t*)(Ax + (32 * w + 16 * s + l16) * J + q8);
#pragma unroll
    for (int e = 0; e < 8; ++e) wl[s][e] = (short)Wl[(q8 + e) * C + 16 * s + l16];
    bc[s] = bias[16 * s + l16];
  }
#pragma unroll
  for (int hb = 0; hb < HB; ++hb) {
#pragma unroll
    for (int e = 0; e < 8; ++e) qa[hb][e] = (short)Q1[(q8 + e) * HID + 16 * hb + l16];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      qb[hb / 2][4 * (hb & 1) + e] = l16 < cout ? (short)Q2[(16 * hb + q4 + e) * cout + l16] : (short)0;
  }
  for (int i = tid; i < HID; i += 256) B1s[i] = b1[i];  // read after the first row's barrier
  const int tj = tid >> 3, tc0 = (tid & 7) * 4;  // this thread's piece of T2[b][y]
  short8_t a2n[2];
  uint2 t2n = {0u, 0u};
  if (blockIdx.x < rows) {
    const bf16* hp = h + (long long)blockIdx.x * (W * C);
#pragma unroll
    for (int s = 0; s < 2; ++s) a2n[s] = *(const short8_t*)(hp + (32 * w + 16 * s + l16) * C + q8);
    t2n = *(const uint2*)(T2 + (long long)blockIdx.x * (J * C) + tj * C + tc0);
  }
  bf16* Ow = Os[w];
  const int sr = lane >> 1, sh = (lane & 1) * 16;  // store: tile row, first channel
  for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
    short8_t a2[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) a2[s] = a2n[s];
    const uint2 v = t2n;
    const long long rn = row + gridDim.x;
    if (rn < rows) {  // the next row's operands, loaded while this row is worked on
      const bf16* hp = h + rn * (W * C);
#pragma unroll
      for (int s = 0; s < 2; ++s) a2n[s] = *(const short8_t*)(hp + (32 * w + 16 * s + l16) * C + q8);
      t2n = *(const uint2*)(T2 + rn * (J * C) + tj * C + tc0);
    }
    {  // T2[b][y] (J x C) into LDS as [c][j]
      const bf16* e = (const bf16*)&v;
#pragma unroll
      for (int q = 0; q < 4; ++q) Ts[(tc0 + q) * kLDK + tj] = e[q];
    }
    __syncthreads();
    // acc[s][t][e] = out[x = 32 w + 16 s + q4 + e][c = 16 t + l16]
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const short8_t b1v = *(const short8_t*)(Ts + (16 * t + l16) * kLDK + q8);
        float4_t acc = mfma32(ax[s], b1v, float4_t{0.f, 0.f, 0.f, 0.f});
        acc = mfma32(a2[s], wl[t], acc);
#pragma unroll
        for (int e = 0; e < 4; ++e) Ow[(16 * s + q4 + e) * kLDK + 16 * t + l16] = f2bf(acc[e] + bc[t]);
      }
    wave_lds_sync();
    if (hn) {
      bf16* hrow = hn + row * (W * C) + 32 * w * C;
      *(uint4*)(hrow + sr * C + sh) = *(const uint4*)(Ow + sr * kLDK + sh);
      *(uint4*)(hrow + sr * C + sh + 8) = *(const uint4*)(Ow + sr * kLDK + sh + 8);
    }
    short8_t hv[2];
#pragma unroll
    for (int gp = 0; gp < 2; ++gp) hv[gp] = *(const short8_t*)(Ow + (16 * gp + l16) * kLDK + q8);
    float4_t acc2[2] = {float4_t{0.f, 0.f, 0.f, 0.f}, float4_t{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int hp = 0; hp < HB / 2; ++hp) {
#pragma unroll
      for (int gp = 0; gp < 2; ++gp) {
        short4_t av[2];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int hb = 2 * hp + hh;
          const float4_t u = mfma32(qa[hb], hv[gp], float4_t{0.f, 0.f, 0.f, 0.f});
          const float4 bb = *(const float4*)(B1s + 16 * hb + q4);
          av[hh] = pack4(gelu(u[0] + bb.x), gelu(u[1] + bb.y), gelu(u[2] + bb.z), gelu(u[3] + bb.w));
        }
        acc2[gp] = mfma32(qb[hp], cat8(av[0], av[1]), acc2[gp]);
      }
    }
#pragma unroll
    for (int gp = 0; gp < 2; ++gp) {
      const long long p = row * W + 32 * w + 16 * gp + l16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int o = q4 + e;
        if (o < cout) {
          float r = acc2[gp][e] + b2[o];
          if (skip) r += skip[p * skip_r + o];
          y[p * ys + o] = r;
        }
      }
    }
    __syncthreads();  // Ts and the tiles are overwritten by the next row
  }
}

// The k_y step of the truncated transform for C = 32, 2m = 32 and H = 128,
// one (sample b, k_x) pair per workgroup iteration.  With the real and
// imaginary k_x rows R = T1[b][kx], I = T1[b][m + kx] (H x C each),
//   G[kx][q][b][c] = sum_y DyRe[q][y] R[y][c] + DyIm[q][y] I[y][c],  q < 4m,
// wavefront w computing rows q = 16w .. 16w + 15 over all of y from the two
// blocks staged in LDS as [c][y]; the product is formed transposed so that a
// lane stores four consecutive channels.
__global__ void __launch_bounds__(256) k_yanalysis(const bf16* __restrict__ T1, const bf16* __restrict__ DyRe,
                                                   const bf16* __restrict__ DyIm, bf16* __restrict__ G, int B,
                                                   long long items) {
  constexpr int C = 32, H = 128, m = 16, Q = 4 * m, LD = H + 8;
  __shared__ __align__(16) bf16 Rs[2][C * LD];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, l16 = lane & 15, q4 = (lane >> 4) * 4;
  const int q8 = (lane >> 4) * 8;
  const int tid = threadIdx.x;
  short8_t aR[H / 32], aI[H / 32];  // k slots: y = 32 kk + q8 .. + 7
#pragma unroll
  for (int kk = 0; kk < H / 32; ++kk) {
    aR[kk] = *(const short8_t*)(DyRe + (16 * w + l16) * H + 32 * kk + q8);
    aI[kk] = *(const short8_t*)(DyIm + (16 * w + l16) * H + 32 * kk + q8);
  }
  for (long long it = blockIdx.x; it < items; it += gridDim.x) {
    const int kx = (int)(it % m);
    const long long b = it / m;
    {  // 2 blocks x 32 groups of 4 rows x 4 runs of 8 channels: a thread reads one
       // 4 x 8 patch and writes each channel's 4 rows as one 8-byte run of [c][y]
      const int part = tid >> 7, y0 = ((tid >> 2) & 31) * 4, c0 = (tid & 3) * 8;
      const bf16* src = T1 + ((b * 2 * m + part * m + kx) * H + y0) * C + c0;
      uint4 v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = *(const uint4*)(src + r * C);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        short4_t col;
#pragma unroll
        for (int r = 0; r < 4; ++r) col[r] = (short)((const bf16*)&v[r])[q];
        *(short4_t*)(Rs[part] + (c0 + q) * LD + y0) = col;
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < H / 32; ++kk) {
        const short8_t bR = *(const short8_t*)(Rs[0] + (16 * t + l16) * LD + 32 * kk + q8);
        const short8_t bI = *(const short8_t*)(Rs[1] + (16 * t + l16) * LD + 32 * kk + q8);
        acc = mfma32(bR, aR[kk], acc);
        acc = mfma32(bI, aI[kk], acc);
      }
      // lane: row q = 16 w + l16, channels 16 t + q4 .. + 3
      *(short4_t*)(G + (((long long)kx * Q + 16 * w + l16) * B + b) * C + 16 * t + q4) =
          pack4(acc[0], acc[1], acc[2], acc[3]);
    }
    __syncthreads();  // Rs is overwritten by the next pair
  }
}

// The k_y synthesis for C = 32, 2m = 32 and H = 128, one (sample b, k_x) pair
// per workgroup iteration: from the mixed modes O[kx][ky][b] = (O_r, O_i),
//   T2[b][y][kx][c]     = sum_ky Ec[y][ky] O_r[ky][c] - Es[y][ky] O_i[ky][c]
//   T2[b][y][m + kx][c] = sum_ky Es[y][ky] O_r[ky][c] + Ec[y][ky] O_i[ky][c]
// wavefront w computing y = 32w .. 32w + 31, both parts, from O_r and O_i
// staged in LDS as [c][ky].
__global__ void __launch_bounds__(256) k_ysynth(const bf16* __restrict__ O, const bf16* __restrict__ Ec,
                                                const bf16* __restrict__ Es, const bf16* __restrict__ Esn,
                                                bf16* __restrict__ T2, int B, long long items) {
  constexpr int C = 32, H = 128, m = 16, K = 2 * m;
  __shared__ __align__(16) bf16 Os[2][C * kLDK];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, l16 = lane & 15, q4 = (lane >> 4) * 4;
  const int q8 = (lane >> 4) * 8;
  const int tid = threadIdx.x;
  short8_t ac[2], as[2], an[2];  // k slots: ky = q8 .. q8 + 7
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int off = (32 * w + 16 * s + l16) * K + q8;
    ac[s] = *(const short8_t*)(Ec + off);
    as[s] = *(const short8_t*)(Es + off);
    an[s] = *(const short8_t*)(Esn + off);
  }
  for (long long it = blockIdx.x; it < items; it += gridDim.x) {
    const int kx = (int)(it % m);
    const long long b = it / m;
    if (tid < 64) {  // 2 parts x 8 groups of 4 ky x 4 runs of 8 channels, one 4 x 8 patch per thread
      const int part = tid >> 5, ky0 = ((tid >> 2) & 7) * 4, c0 = (tid & 3) * 8;
      uint4 v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        v[r] = *(const uint4*)(O + (((long long)kx * K + ky0 + r) * B + b) * 2 * C + part * C + c0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        short4_t col;
#pragma unroll
        for (int r = 0; r < 4; ++r) col[r] = (short)((const bf16*)&v[r])[q];
        *(short4_t*)(Os[part] + (c0 + q) * kLDK + ky0) = col;
      }
    }
    __syncthreads();
    short8_t br[2], bi[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      br[t] = *(const short8_t*)(Os[0] + (16 * t + l16) * kLDK + q8);
      bi[t] = *(const short8_t*)(Os[1] + (16 * t + l16) * kLDK + q8);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        float4_t fr = {0.f, 0.f, 0.f, 0.f}, fi = {0.f, 0.f, 0.f, 0.f};
        fr = mfma32(br[t], ac[s], fr);
        fr = mfma32(bi[t], an[s], fr);
        fi = mfma32(br[t], as[s], fi);
        fi = mfma32(bi[t], ac[s], fi);
        // lane: y = 32 w + 16 s + l16, channels 16 t + q4 .. + 3
        bf16* row = T2 + ((b * H + 32 * w + 16 * s + l16) * K) * C + 16 * t + q4;
        *(short4_t*)(row + kx * C) = pack4(fr[0], fr[1], fr[2], fr[3]);
        *(short4_t*)(row + (m + kx) * C) = pack4(fi[0], fi[1], fi[2], fi[3]);
      }
    __syncthreads();  // Os is overwritten by the next pair
  }
}

// Per-mode channel mixing for C = 32 (2C = 64): for mode (kx, q) the rows b
// of [G_r, G_i] (B x 64, G[kx][q][b][c] and G[kx][2m + q][b][c]) times the
// 64 x 64 block V, out[kx][q][b][n] = sum_k [G_r, G_i][b][k] V[k][n], with V
// given transposed (Vt[n][k], rows along k): WbT for the forward product,
// Wb itself for the adjoint (V = Wb^T).  One workgroup per mode, its
// wavefronts taking the 32 x 32 output tiles in turn; every fragment is read
// straight from memory with 8-byte loads, and the product is formed
// transposed so that a lane stores four consecutive outputs.
__global__ void __launch_bounds__(256) k_mix(const bf16* __restrict__ G, const bf16* __restrict__ Vt,
                                             bf16* __restrict__ out, int B, int m) {
  constexpr int C = 32, C2 = 64;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, l16 = lane & 15, q4 = (lane >> 4) * 4;
  const int q8 = (lane >> 4) * 8;  // k slots: 32 kk + q8 .. + 7 (kk = 0: G_r, 1: G_i)
  const long long mode = blockIdx.x;  // kx * 2m + q
  const int kx = (int)(mode / (2 * m)), q = (int)(mode % (2 * m));
  const bf16* Gr = G + ((long long)kx * 4 * m + q) * B * C;
  const bf16* Gi = Gr + 2LL * m * B * C;
  const bf16* V = Vt + mode * C2 * C2;
  bf16* o = out + mode * B * C2;
  const int tiles = (B + 31) / 32 * 2;
  for (int tile = w; tile < tiles; tile += 4) {
    const int i0 = (tile >> 1) * 32, j0 = (tile & 1) * 32;
    short8_t a[2][2], v[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int row = i0 + 16 * s + l16;
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
        a[s][kk] = row < B ? *(const short8_t*)((kk == 0 ? Gr : Gi) + (long long)row * C + q8)
                           : short8_t{0, 0, 0, 0, 0, 0, 0, 0};
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) v[t][kk] = *(const short8_t*)(V + (j0 + 16 * t + l16) * C2 + 32 * kk + q8);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int row = i0 + 16 * s + l16;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) acc = mfma32(v[t][kk], a[s][kk], acc);
        if (row < B) *(short4_t*)(o + (long long)row * C2 + j0 + 16 * t + q4) = pack4(acc[0], acc[1], acc[2], acc[3]);
      }
    }
  }
}

// Backward of the projection y = GELU(u) Q2 + b2, u = h Q1 + b1, for C = 32
// and HID = 128, fused so that the hidden layer never reaches memory.  Per
// group of 16 points a wavefront recomputes u^T = Q1^T h^T on the matrix cores
// (the forward's operand layout: lane = point, four consecutive hidden rows),
// forms a = GELU(u) and du = (dy Q2^T) GELU'(u) in registers, writes
// dh = du Q1^T (du is already the second operand of that product), and adds
// the group to its running weight gradients dQ1^T = du^T h and dQ2 = a^T dy
// (operands transposed through the wavefront's LDS) and the bias gradients.
// Each wavefront finally writes its sums to slot `wave` of part, laid out as
// the gradient vector [dQ1 (C x HID) | db1 (HID) | dQ2 (HID x cout) | db2 (cout)],
// and the slots are reduced afterwards in a fixed order.
constexpr int kProjBackMaxCout = 4;
template <int C, int HID>
__global__ void __launch_bounds__(256, 2) k_proj_back(const bf16* __restrict__ h, const bf16* __restrict__ Q1,
                                                      const float* __restrict__ b1, const bf16* __restrict__ Q2,
                                                      const bf16* __restrict__ dy, int cout, bf16* __restrict__ dh,
                                                      float* __restrict__ part, long long npts) {
  static_assert(C == 32 && HID % 32 == 0, "k in steps of 32");
  constexpr int HB = HID / 16, KB = C / 16, LDJ = HID + 8, LDC = C + 8, MO = kProjBackMaxCout;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, l16 = lane & 15, q4 = (lane >> 4) * 4;
  const int q8 = (lane >> 4) * 8;  // k slots of the 32-deep products: q8 .. q8 + 7
  const long long wave = (long long)blockIdx.x * 4 + w, nwave = (long long)gridDim.x * 4;
  __shared__ float Q2s[HID][MO], B1s[HID];
  __shared__ __align__(16) bf16 Q1s[C * LDJ], Q1t[HID * LDC];  // Q1 [c][j] and Q1^T [j][c]
  __shared__ __align__(16) bf16 DU[4][16 * LDJ], AA[4][16 * LDJ], HS[4][16 * LDC], DY[4][16 * 16];
  for (int i = threadIdx.x; i < HID * MO; i += 256) {
    const int j = i / MO, o = i % MO;
    Q2s[j][o] = o < cout ? bf2f(Q2[j * cout + o]) : 0.f;
  }
  for (int i = threadIdx.x; i < HID; i += 256) B1s[i] = b1[i];
  for (int i = threadIdx.x; i < C * HID / 8; i += 256) {
    const int c = i / (HID / 8), j0 = (i % (HID / 8)) * 8;
    *(uint4*)(Q1s + c * LDJ + j0) = *(const uint4*)(Q1 + c * HID + j0);
  }
  for (int i = threadIdx.x; i < C * HID; i += 256) {
    const int c = i / HID, j = i % HID;
    Q1t[j * LDC + c] = Q1[i];
  }
  __syncthreads();
  float4_t g1[HB][KB], g2[HB];  // g1[jb][cb][e] = dQ1^T[16 jb + q4 + e][16 cb + l16]; g2[jb][e] = dQ2[16 jb + q4 + e][l16]
  float gb1[HB][4], gb2 = 0.f;  // gb1: this lane's point; gb2: output l16, points q4 .. q4 + 3
#pragma unroll
  for (int hb = 0; hb < HB; ++hb) {
    g2[hb] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) g1[hb][kb] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int e = 0; e < 4; ++e) gb1[hb][e] = 0.f;
  }
  bf16 *du_s = DU[w], *a_s = AA[w], *h_s = HS[w], *dy_s = DY[w];
  for (long long t = wave; t * 16 < npts; t += nwave) {
    const long long p = t * 16 + l16;
    const bool ok = p < npts;
    const short8_t hv = ok ? *(const short8_t*)(h + p * C + q8) : short8_t{0, 0, 0, 0, 0, 0, 0, 0};
    float dyv[MO];  // this lane's point
#pragma unroll
    for (int o = 0; o < MO; ++o) dyv[o] = (ok && o < cout) ? bf2f(dy[p * cout + o]) : 0.f;
#pragma unroll
    for (int e = 0; e < 4; ++e) dy_s[l16 * 16 + q4 + e] = (ok && q4 + e < cout) ? dy[p * cout + q4 + e] : (bf16)0;
    *(short8_t*)(h_s + l16 * LDC + q8) = hv;
#pragma unroll
    for (int hb = 0; hb < HB; ++hb) {
      const float4_t u = mfma32(*(const short8_t*)(Q1t + (16 * hb + l16) * LDC + q8), hv, float4_t{0.f, 0.f, 0.f, 0.f});
      float a4[4], d4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = 16 * hb + q4 + e;
        const float uv = u[e] + B1s[j];
        const float ph = norm_cdf(uv);
        float da = 0.f;
#pragma unroll
        for (int o = 0; o < MO; ++o) da += dyv[o] * Q2s[j][o];
        a4[e] = ok ? uv * ph : 0.f;
        d4[e] = ok ? da * (ph + uv * 0.39894228040143268f * __expf(-0.5f * uv * uv)) : 0.f;
      }
      const short4_t duf = pack4(d4[0], d4[1], d4[2], d4[3]);
      // rows = points, for dh below and the weight gradients
      *(short4_t*)(du_s + l16 * LDJ + 16 * hb + q4) = duf;
      *(short4_t*)(a_s + l16 * LDJ + 16 * hb + q4) = pack4(a4[0], a4[1], a4[2], a4[3]);
      // the bias gradient adds the stored (rounded) du, as the unfused path does
#pragma unroll
      for (int e = 0; e < 4; ++e) gb1[hb][e] += bf2f((bf16)duf[e]);
    }
    wave_lds_sync();
    // dh^T = Q1 du^T: lane = point, channels 16 cb + q4 .. + 3
#pragma unroll
    for (int cb = 0; cb < KB; ++cb) {
      float4_t d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int hp = 0; hp < HID / 32; ++hp)
        d = mfma32(*(const short8_t*)(Q1s + (16 * cb + l16) * LDJ + 32 * hp + q8),
                   *(const short8_t*)(du_s + l16 * LDJ + 32 * hp + q8), d);
      if (ok) *(short4_t*)(dh + p * C + 16 * cb + q4) = pack4(d[0], d[1], d[2], d[3]);
    }
    // weight gradients: contraction over the group's 16 points (16 deep)
    short4_t hT[KB], dyb;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int e = 0; e < 4; ++e) hT[kb][e] = (short)h_s[(q4 + e) * LDC + 16 * kb + l16];
#pragma unroll
    for (int e = 0; e < 4; ++e) dyb[e] = (short)dy_s[(q4 + e) * 16 + l16];
#pragma unroll
    for (int jb = 0; jb < HB; ++jb) {
      short4_t duT, aT;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        duT[e] = (short)du_s[(q4 + e) * LDJ + 16 * jb + l16];
        aT[e] = (short)a_s[(q4 + e) * LDJ + 16 * jb + l16];
      }
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) g1[jb][kb] = mfma16(duT, hT[kb], g1[jb][kb]);
      g2[jb] = mfma16(aT, dyb, g2[jb]);
    }
    // db2: this lane adds points q4 .. q4 + 3 of output l16 (the four lane groups are added at the end)
#pragma unroll
    for (int e = 0; e < 4; ++e) gb2 += bf2f((bf16)dyb[e]);
    wave_lds_sync();
  }
  // bias gradient db1: lanes with the same q4 hold different points
#pragma unroll
  for (int hb = 0; hb < HB; ++hb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float v = gb1[hb][e];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      gb1[hb][e] = v;
    }
  gb2 += __shfl_xor(gb2, 16);
  gb2 += __shfl_xor(gb2, 32);
  float* slot = part + wave * (long long)(C * HID + HID + HID * cout + cout);
#pragma unroll
  for (int jb = 0; jb < HB; ++jb) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int e = 0; e < 4; ++e) slot[(16 * kb + l16) * HID + 16 * jb + q4 + e] = g1[jb][kb][e];
    if (l16 == 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) slot[C * HID + 16 * jb + q4 + e] = gb1[jb][e];
    }
    if (l16 < cout) {
#pragma unroll
      for (int e = 0; e < 4; ++e) slot[C * HID + HID + (16 * jb + q4 + e) * cout + l16] = g2[jb][e];
    }
  }
  if (q4 == 0 && l16 < cout) slot[C * HID + HID + HID * cout + l16] = gb2;
}

// dz = dh * GELU'(z), eight elements per thread with 16-byte accesses (n % 8 == 0)
__global__ void k_gelu_back(const bf16* __restrict__ dh, const bf16* __restrict__ z, bf16* __restrict__ dz,
                            long long n) {
  const long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * 8;
  if (i >= n) return;
  const uint4 a = *(const uint4*)(dh + i), b = *(const uint4*)(z + i);
  const bf16* pa = (const bf16*)&a;
  const bf16* pb = (const bf16*)&b;
  bf16 o[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) o[q] = f2bf(bf2f(pa[q]) * gelu_grad(bf2f(pb[q])));
  *(uint4*)(dz + i) = *(const uint4*)o;
}

__global__ void k_gather(float* __restrict__ dst, long long dch, const float* __restrict__ src, long long sch,
                         int nch, long long npix, const long long* __restrict__ idx, long long tot) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tot) return;
  const long long s = i / (npix * nch), r = i % (npix * nch);
  const long long p = r / nch;
  const int ch = (int)(r % nch);
  dst[(s * npix + p) * dch + ch] = src[(idx[s] * npix + p) * sch + ch];
}

// k_gather with a symmetry of the square grid per sample: sample s takes the
// element g = sym[s] of the dihedral group D4 (r = g & 3 quarter turns
// counterclockwise, then with g & 4 the reflection y -> -y), about the grid
// centre (n/2, n/2) on the n x n periodic grid.  The destination node x' takes
// the source node M_g^-1 x' and the vector formed by channels 0 and 1 is
// multiplied by M_g; the other channels are copied.
__global__ void k_gather_d4(float* __restrict__ dst, long long dch, const float* __restrict__ src, long long sch,
                            int nch, int n, const long long* __restrict__ idx, const int* __restrict__ sym,
                            long long tot) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tot) return;
  const long long npix = (long long)n * n;
  const long long s = i / npix, p = i % npix;
  const int y = (int)(p / n), x = (int)(p % n), h = n / 2;
  const int g = sym[s], r = g & 3;
  // source position: reflect the destination position if asked, then turn
  // it back r quarter turns ((a, b) -> (b, -a) each)
  int a = x - h, b = y - h;
  if (g & 4) b = -b;
  for (int q = 0; q < r; ++q) {
    const int t = a;
    a = b;
    b = -t;
  }
  const int xs = (a + h + n) % n, ys = (b + h + n) % n;
  const float* sp = src + (idx[s] * npix + (long long)ys * n + xs) * sch;
  float* dp = dst + (s * npix + p) * dch;
  // the vector: r quarter turns ((u, v) -> (-v, u) each), then the reflection
  float u = sp[0], v = nch > 1 ? sp[1] : 0.f;
  for (int q = 0; q < r; ++q) {
    const float t = u;
    u = -v;
    v = t;
  }
  if (g & 4) v = -v;
  dp[0] = u;
  if (nch > 1) dp[1] = v;
  for (int c = 2; c < nch; ++c) dp[c] = sp[c];
}

// per-sample sums of (y - t)^2 and t^2 (FP64), one block of 1024 threads per
// sample, a thread per pixel (all its channels).  With ref non-null the second
// sum is of (t - ref)^2, ref holding the same channels at pixel stride ref_s
// (the denominator of an increment loss).
__global__ void __launch_bounds__(1024) k_loss_sums(const float* __restrict__ y, const float* __restrict__ t,
                                                    long long per, const float* __restrict__ ref, long long ref_s,
                                                    int nch, double* __restrict__ out) {
  const long long base = (long long)blockIdx.x * per;
  const long long npix = per / nch, pix0 = (long long)blockIdx.x * npix;
  double a = 0.0, b = 0.0;
  for (long long j = threadIdx.x; j < npix; j += blockDim.x) {
    const long long e = base + j * nch;
    for (int ch = 0; ch < nch; ++ch) {
      const double d = (double)y[e + ch] - (double)t[e + ch];
      a += d * d;
      double tv = (double)t[e + ch];
      if (ref) tv -= (double)ref[(pix0 + j) * ref_s + ch];
      b += tv * tv;
    }
  }
  __shared__ double red[16][2];
  a = ttsh::wave_sum_from(a, 1);
  b = ttsh::wave_sum_from(b, 1);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = a;
    red[threadIdx.x >> 6][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      sa += red[w][0];
      sb += red[w][1];
    }
    out[2 * blockIdx.x] = sa;
    out[2 * blockIdx.x + 1] = sb;
  }
}

// x[p][c] += amp * u, u uniform in [-1, 1) from SplitMix64 (Steele, Lea and
// Flood 2014) of seed + element index: a counter-based stream, the same for
// any launch shape.
__device__ inline unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_perturb(float* __restrict__ x, long long stride, int nch, long long tot, float amp,
                          unsigned long long seed) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tot) return;
  const unsigned long long r = splitmix64(seed * 0x100000001B3ull + (unsigned long long)i);
  const float u = (float)(r >> 40) * (1.0f / 8388608.0f) - 1.0f;  // 24 bits -> [-1, 1)
  x[(i / nch) * stride + i % nch] += amp * u;
}

// per-sample sums of (y - t)^2 and t^2 over strided channels-last fields
__global__ void __launch_bounds__(256) k_err_sums(const float* __restrict__ y, long long ys,
                                                  const float* __restrict__ t, long long ts, int nch,
                                                  long long npix, double* __restrict__ out) {
  const long long base = (long long)blockIdx.x * npix;
  double a = 0.0, b = 0.0;
  for (long long i = threadIdx.x; i < npix * nch; i += blockDim.x) {
    const long long p = base + i / nch;
    const int ch = (int)(i % nch);
    const double tv = t[p * ts + ch];
    const double d = (double)y[p * ys + ch] - tv;
    a += d * d;
    b += tv * tv;
  }
  __shared__ double red[4][2];
  a = ttsh::wave_sum_from(a, 1);
  b = ttsh::wave_sum_from(b, 1);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = a;
    red[threadIdx.x >> 6][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    out[2 * blockIdx.x + 1] = red[0][1] + red[1][1] + red[2][1] + red[3][1];
  }
}

// dl/dy = (y - t) / (||y - t|| ||t|| B)
__global__ void k_loss_grad(const float* __restrict__ y, const float* __restrict__ t,
                            const double* __restrict__ sums, long long per, int B, bf16* __restrict__ dy) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per * B) return;
  const long long s = i / per;
  const double num = sqrt(sums[2 * s]), den = sqrt(sums[2 * s + 1]);
  dy[i] = f2bf((float)(((double)y[i] - (double)t[i]) / (num * den * B)));
}

// column sums of a [rows][ncol] bf16 matrix: partials per chunk of rows
__global__ void k_colsum_part(const bf16* __restrict__ a, long long rows, int ncol, long long chunk,
                              float* __restrict__ part) {
  const int j = threadIdx.x % ncol;  // blockDim = ncol * lanes
  const int lanes = blockDim.x / ncol;
  const int l = threadIdx.x / ncol;
  const long long r0 = (long long)blockIdx.x * chunk, r1 = min(rows, r0 + chunk);
  float v = 0.f;
  for (long long r = r0 + l; r < r1; r += lanes) v += bf2f(a[r * ncol + j]);
  __shared__ float red[1024];
  red[threadIdx.x] = v;
  __syncthreads();
  if (l == 0) {
    float s = 0.f;
    for (int q = 0; q < lanes; ++q) s += red[q * ncol + j];
    part[(long long)blockIdx.x * ncol + j] = s;
  }
}

// the same for ncol = 8 * 2^k <= 256: a thread adds 8 adjacent columns with
// 16-byte loads; rows are dealt round robin to the 256 / (ncol / 8) row lanes,
// whose sums are then added in lane order
__global__ void __launch_bounds__(256) k_colsum_part8(const bf16* __restrict__ a, long long rows, int ncol,
                                                      long long chunk, float* __restrict__ part) {
  const int tpr = ncol / 8, rpi = 256 / tpr;
  const int g = threadIdx.x % tpr, r = threadIdx.x / tpr;
  const long long r0 = (long long)blockIdx.x * chunk, r1 = min(rows, r0 + chunk);
  float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (long long row = r0 + r; row < r1; row += rpi) {
    const uint4 u = *(const uint4*)(a + row * ncol + 8 * g);
    const bf16* e = (const bf16*)&u;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] += bf2f(e[q]);
  }
  __shared__ float red[256 * 8];
#pragma unroll
  for (int q = 0; q < 8; ++q) red[r * ncol + 8 * g + q] = v[q];
  __syncthreads();
  if (threadIdx.x < ncol) {
    float s = 0.f;
    for (int q = 0; q < rpi; ++q) s += red[q * ncol + threadIdx.x];
    part[(long long)blockIdx.x * ncol + threadIdx.x] = s;
  }
}

// Weight gradient of the lifting layer for CIN <= 4 inputs and 32 outputs:
// workgroup b sums x[p][k] dh[p][c] over the points of chunk b into
// part[b][k][c] (k_reduce_parts then adds the chunks).  Thread t takes the
// eight columns 8 (t % 4) .. 8 (t % 4) + 7 of every 64th point (one 16-byte
// load of dh per point), and the 64 point lanes are added in order.  The
// input channels are too few for the matrix-core tiles.
template <int CIN>
__global__ void __launch_bounds__(256) k_lift_wgrad_part(const bf16* __restrict__ x, const bf16* __restrict__ dh,
                                                         long long P, long long chunk, float* __restrict__ part) {
  constexpr int C = 32, LANES = 64;
  const int cg = threadIdx.x & 3, lp = threadIdx.x >> 2;
  const long long p0 = (long long)blockIdx.x * chunk;
  const long long p1 = p0 + chunk < P ? p0 + chunk : P;
  float acc[CIN][8];
#pragma unroll
  for (int k = 0; k < CIN; ++k)
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[k][e] = 0.f;
  for (long long p = p0 + lp; p < p1; p += LANES) {
    const uint4 raw = *(const uint4*)(dh + p * C + 8 * cg);
    const unsigned w[4] = {raw.x, raw.y, raw.z, raw.w};
    float g[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      g[2 * e] = __uint_as_float(w[e] << 16);
      g[2 * e + 1] = __uint_as_float(w[e] & 0xffff0000u);
    }
#pragma unroll
    for (int k = 0; k < CIN; ++k) {
      const float xv = bf2f(x[p * CIN + k]);
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[k][e] += xv * g[e];
    }
  }
  __shared__ float red[LANES][CIN * C];
#pragma unroll
  for (int k = 0; k < CIN; ++k)
#pragma unroll
    for (int e = 0; e < 8; ++e) red[lp][k * C + 8 * cg + e] = acc[k][e];
  __syncthreads();
  for (int o = threadIdx.x; o < CIN * C; o += blockDim.x) {
    float t = 0.f;
    for (int q = 0; q < LANES; ++q) t += red[q][o];
    part[(long long)blockIdx.x * CIN * C + o] = t;
  }
}

// out[j] = sum_c part[c][j] in a fixed order: 16 interleaved partial sums per
// column (c = g, g + 16, ...), then added for g = 0..15; 16 columns per block
__global__ void __launch_bounds__(256) k_reduce_parts(const float* __restrict__ part, int nparts, long long n,
                                                      float* __restrict__ out) {
  const int jj = threadIdx.x & 15, g = threadIdx.x >> 4;
  const long long j = (long long)blockIdx.x * 16 + jj;
  float s = 0.f;
  if (j < n)
    for (int c = g; c < nparts; c += 16) s += part[(long long)c * n + j];
  __shared__ float red[16][16];
  red[g][jj] = s;
  __syncthreads();
  if (g == 0 && j < n) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][jj];
    out[j] = t;
  }
}

// The same sums in two passes that keep every CU busy: kRedChunk consecutive
// partial vectors added in part order (one thread per element, consecutive
// threads on consecutive elements, so each part row is read coalesced), then
// the chunk sums added in chunk order.  The order is fixed, so the result is
// the same run to run.
constexpr int kRedChunk = 32;
__global__ void __launch_bounds__(256) k_reduce_chunks(const float* __restrict__ part, int nparts, long long n,
                                                       float* __restrict__ sums) {
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const int c0 = (int)blockIdx.y * kRedChunk, c1 = min(nparts, c0 + kRedChunk);
  float s = 0.f;
#pragma unroll 8
  for (int c = c0; c < c1; ++c) s += part[(long long)c * n + j];
  sums[(long long)blockIdx.y * n + j] = s;
}
__global__ void __launch_bounds__(256) k_reduce_sums(const float* __restrict__ sums, int nchunks, long long n,
                                                     float* __restrict__ out) {
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  float s = 0.f;
#pragma unroll 8
  for (int c = 0; c < nchunks; ++c) s += sums[(long long)c * n + j];
  out[j] = s;
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Wb[kx][q] = [[R_r, R_i], [-R_i, R_r]] (2C x 2C, bf16) from the master R
// (and its per-mode transpose WbT[kx][q][j][i] = Wb[kx][q][i][j])
__global__ void k_build_wb(const float* __restrict__ Rr, const float* __restrict__ Ri, bf16* __restrict__ Wb,
                           bf16* __restrict__ WbT, int m, int C) {
  const long long n = (long long)2 * m * m * 4 * C * C;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int C2 = 2 * C;
  const int j = (int)(idx % C2), i = (int)((idx / C2) % C2);
  const long long mode = idx / ((long long)C2 * C2);  // = kx * 2m + q
  const int q = (int)(mode % (2 * m)), kx = (int)(mode / (2 * m));
  const long long src = (((long long)q * m + kx) * C + (i % C)) * C + (j % C);
  float v;
  if (i < C) v = (j < C) ? Rr[src] : Ri[src];
  else v = (j < C) ? -Ri[src] : Rr[src];
  Wb[idx] = f2bf(v);
  WbT[(mode * C2 + j) * C2 + i] = f2bf(v);
}

unsigned nb(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// =============================================================================================
// context
// =============================================================================================
namespace {
thread_local std::string g_fno_err;
int ffail(int code, const std::string& msg);
}  // namespace

struct fno_ctx {
  int C, m, L, cin, cout, hid, H, W, maxB;
  hipStream_t s = nullptr;
  int64_t nparam = 0;
  // parameter offsets in the flat vector
  int64_t oPw, oPb, oR[16], oW[16], ob[16], oQ1, oQ1b, oQ2, oQ2b;
  float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  int adam_t = 0;
  // bf16 compute copies
  bf16 *Pw = nullptr, *Wl[16] = {}, *WlT[16] = {}, *Wb[16] = {}, *WbT[16] = {}, *Q1 = nullptr, *Q2 = nullptr;
  // DFT matrices (bf16)
  bf16 *Dx, *DxG, *DyRe, *DyIm, *Ec, *Es, *Esn, *Ax, *Ax1;
  // activations
  bf16 *xb, *h[17], *z[16], *G[16], *T1, *T2, *O, *u, *a, *dy;
  float* y = nullptr;  // last training output (pointer to caller buffer is not kept)
  // backward scratch
  bf16 *dh0, *dh1, *dz, *gG, *gF, *du, *xt;
  float *part = nullptr;
  size_t part_n = 0;
  float* red2 = nullptr;  // chunk sums of the two-pass reduction of part
  size_t red2_n = 0;
  double* lsum = nullptr;
  long long* gidx = nullptr;  // sample indices of fno_gather [max_batch]
  int* gsym = nullptr;        // symmetry elements of fno_gather_d4 [max_batch]
  int staged_gemm = 1;        // GEMMs whose operands allow it stage them through LDS
  int specialized = 1;        // kernels for C = 32, 2m = 32 and W = 128 (layer tail) / H = 128 (k_y steps)
  bool proj_train_fused = false;  // the last training forward left no hidden layer (fused backward)
  // stage capture (FNO_OPT_CAPTURE, for stage-level tests): per layer, the
  // intermediates that later layers overwrite, copied as they are produced
  bool capture = false;
  bool tail_proj = true;  // FNO_OPT_TAIL_PROJ
  bf16 *capT1[16] = {}, *capO[16] = {}, *capT2[16] = {};                       // forward
  bf16 *capDZ[16] = {}, *capBT1[16] = {}, *capGG[16] = {}, *capGF[16] = {}, *capBT2[16] = {}, *capDH[16] = {};
  bf16* capDHL = nullptr;                                                      // dl/dh_L from the projection
  std::vector<void*> allocs;
  std::vector<std::pair<const char*, size_t>> extents;  // (start, bytes) of every buffer
};

namespace {
int ffail(int code, const std::string& msg) {
  g_fno_err = msg;
  return ttsh::record_error(code, msg.c_str());
}

#define FCHK(expr)                                                                           \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return ffail(TTSH_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int alloc(fno_ctx* c, T** p, size_t n) {
  if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) return ffail(TTSH_ENOMEM, "fno allocation failed");
  c->allocs.push_back((void*)*p);
  c->extents.push_back({(const char*)*p, n * sizeof(T)});
  return TTSH_OK;
}

// Host-side bounds proof for a GEMM launch: the whole index range of every
// operand must fall inside one buffer of the context (or a caller buffer
// registered for the call).  Strides are non-negative by construction.
bool inside(const fno_ctx* c, const void* p, long long max_off, size_t elem,
            const std::pair<const char*, size_t>* extra, int nextra = 1) {
  if (!p) return true;
  const char* a = (const char*)p;
  const char* e = a + (size_t)(max_off + 1) * elem;
  auto fits = [&](const std::pair<const char*, size_t>& x) { return a >= x.first && e <= x.first + x.second; };
  for (int q = 0; extra && q < nextra; ++q)
    if (fits(extra[q])) return true;
  for (auto& x : c->extents)
    if (fits(x)) return true;
  return false;
}

long long span(const Op& o, int nb1, int nb2, int rows, int cols) {
  return (long long)(nb1 - 1) * o.s1 + (long long)(nb2 - 1) * o.s2 + (long long)(rows - 1) * o.r +
         (long long)(cols - 1) * o.c;
}

int upload_bf16(fno_ctx* c, bf16** dst, const std::vector<double>& v) {
  std::vector<bf16> h(v.size());
  for (size_t i = 0; i < v.size(); ++i) h[i] = f2bf((float)v[i]);
  int rc = alloc(c, dst, v.size());
  if (rc) return rc;
  FCHK(hipMemcpy(*dst, h.data(), h.size() * sizeof(bf16), hipMemcpyHostToDevice));
  return TTSH_OK;
}

// DFT matrices of the pruned transforms (FP64 on the host, rounded to bf16)
int make_dft(fno_ctx* c) {
  const int m = c->m, H = c->H, W = c->W;
  const double tp = 2.0 * M_PI, HW = (double)H * W;
  auto kyq = [&](int q) { return q < m ? q : q - 2 * m; };
  std::vector<double> Dx(2 * m * W), DxG(2 * m * W), DyRe(4 * m * H), DyIm(4 * m * H);
  std::vector<double> Ec(H * 2 * m), Es(H * 2 * m), Esn(H * 2 * m), Ax(W * 2 * m), Ax1(W * 2 * m);
  for (int kx = 0; kx < m; ++kx)
    for (int x = 0; x < W; ++x) {
      const double th = tp * kx * x / W, w = (kx == 0 ? 1.0 : 2.0) / HW;
      Dx[kx * W + x] = cos(th);
      Dx[(m + kx) * W + x] = -sin(th);
      DxG[kx * W + x] = w * cos(th);
      DxG[(m + kx) * W + x] = -w * sin(th);
      Ax[x * 2 * m + kx] = w * cos(th);
      Ax[x * 2 * m + m + kx] = -w * sin(th);
      Ax1[x * 2 * m + kx] = cos(th);
      Ax1[x * 2 * m + m + kx] = -sin(th);
    }
  for (int q = 0; q < 2 * m; ++q)
    for (int y = 0; y < H; ++y) {
      const double th = tp * kyq(q) * y / H;
      DyRe[q * H + y] = cos(th);
      DyRe[(2 * m + q) * H + y] = -sin(th);
      DyIm[q * H + y] = sin(th);
      DyIm[(2 * m + q) * H + y] = cos(th);
      Ec[y * 2 * m + q] = cos(th);
      Es[y * 2 * m + q] = sin(th);
      Esn[y * 2 * m + q] = -sin(th);
    }
  int rc;
  if ((rc = upload_bf16(c, &c->Dx, Dx)) || (rc = upload_bf16(c, &c->DxG, DxG)) ||
      (rc = upload_bf16(c, &c->DyRe, DyRe)) || (rc = upload_bf16(c, &c->DyIm, DyIm)) ||
      (rc = upload_bf16(c, &c->Ec, Ec)) || (rc = upload_bf16(c, &c->Es, Es)) ||
      (rc = upload_bf16(c, &c->Esn, Esn)) || (rc = upload_bf16(c, &c->Ax, Ax)) ||
      (rc = upload_bf16(c, &c->Ax1, Ax1)))
    return rc;
  return TTSH_OK;
}

// bf16 compute copies of the master parameters
int refresh_weights(fno_ctx* c) {
  const int C = c->C, m = c->m;
  hipLaunchKernelGGL(k_to_bf16, dim3(nb((long long)c->cin * C)), dim3(256), 0, c->s, c->theta + c->oPw, c->Pw,
                     (long long)c->cin * C);
  for (int l = 0; l < c->L; ++l) {
    hipLaunchKernelGGL(k_to_bf16, dim3(nb((long long)C * C)), dim3(256), 0, c->s, c->theta + c->oW[l], c->Wl[l],
                       (long long)C * C);
    hipLaunchKernelGGL(k_transpose_bf16, dim3(nb((long long)C * C)), dim3(256), 0, c->s, c->theta + c->oW[l],
                       c->WlT[l], C);
    const long long nwb = (long long)2 * m * m * 4 * C * C;
    const long long nR = (long long)2 * m * m * C * C;
    hipLaunchKernelGGL(k_build_wb, dim3(nb(nwb)), dim3(256), 0, c->s, c->theta + c->oR[l], c->theta + c->oR[l] + nR,
                       c->Wb[l], c->WbT[l], m, C);
  }
  hipLaunchKernelGGL(k_to_bf16, dim3(nb((long long)C * c->hid)), dim3(256), 0, c->s, c->theta + c->oQ1, c->Q1,
                     (long long)C * c->hid);
  hipLaunchKernelGGL(k_to_bf16, dim3(nb((long long)c->hid * c->cout)), dim3(256), 0, c->s, c->theta + c->oQ2, c->Q2,
                     (long long)c->hid * c->cout);
  FCHK(hipGetLastError());
  return TTSH_OK;
}

// Launch after proving every operand in bounds.
int cgemm(fno_ctx* c, const GemmArgs& g, const std::pair<const char*, size_t>* extra = nullptr, int nextra = 1) {
  const Op ops[4] = {g.A, g.B, g.A2, g.B2};
  const int rows[4] = {g.M, g.K, g.M, g.K2}, cols[4] = {g.K, g.N, g.K2, g.N};
  for (int q = 0; q < 4; ++q) {
    if (q >= 2 && g.K2 <= 0) break;
    const Op& o = ops[q];
    if (o.s1 < 0 || o.s2 < 0 || o.r < 0 || o.c < 0) return ffail(TTSH_EINVAL, "negative GEMM stride");
    if (!inside(c, o.p, span(o, g.nb1, g.nb2, rows[q], cols[q]), sizeof(bf16), extra, nextra))
      return ffail(TTSH_EINVAL, "GEMM operand out of bounds (internal layout error)");
  }
  const long long cmax = (long long)(g.nb1 - 1) * g.sC1 + (long long)(g.nb2 - 1) * g.sC2 +
                         (long long)(g.M - 1) * g.rC + (long long)(g.N - 1) * g.cC;
  if (!inside(c, g.C, cmax, g.c_bf16 ? 2 : 4, extra, nextra) || !inside(c, g.pre_in, cmax, 2, extra, nextra) ||
      !inside(c, g.pre_out, cmax, 2, extra, nextra) || !inside(c, g.bias, g.N - 1, 4, extra, nextra))
    return ffail(TTSH_EINVAL, "GEMM output out of bounds (internal layout error)");
  if (g.skip && (g.c_bf16 || g.skip_r < 0 ||
                 !inside(c, g.skip, (long long)(g.M - 1) * g.skip_r + g.N - 1, 4, extra, nextra)))
    return ffail(TTSH_EINVAL, "GEMM residual input out of bounds (internal layout error)");
  GemmArgs gv = g;
  gv.A.kvec = kvec_ok(g.A, true);
  gv.B.kvec = kvec_ok(g.B, false);
  gv.A2.kvec = g.K2 > 0 && kvec_ok(g.A2, true);
  gv.B2.kvec = g.K2 > 0 && kvec_ok(g.B2, false);
  {
    const size_t al = g.c_bf16 ? 8 : 16;
    gv.vecC = g.cC == 1 && g.rC % 4 == 0 && g.sC1 % 4 == 0 && g.sC2 % 4 == 0 && ((uintptr_t)g.C % al) == 0;
  }
  gv.staged = c->staged_gemm ? staged_form(g) : -1;
  const hipError_t e = gemm(gv, c->s);
  if (e != hipSuccess) return ffail(TTSH_EHIP, std::string("GEMM launch: ") + hipGetErrorString(e));
  return TTSH_OK;
}

GemmArgs ga() {
  GemmArgs g{};
  g.staged = -1;
  g.nb1 = g.nb2 = 1;
  g.alpha = 1.f;
  g.alpha2 = 1.f;
  return g;
}

// ---- spectral pieces shared by forward and backward ------------------------------------
// Forward truncated rfft2 of src [B][H][W][C] into the mode layout
// dst [m][4m][B][C] (rows 0..2m-1 real parts, 2m..4m-1 imaginary parts);
// Dxm is the k_x matrix (Dx, or DxG for the backward weights).
// (the k_x step alone: T1 [B][2m][H][C] = Dxm (2m x W) . src[b][y] (W x C))
int spectral_analysis_x(fno_ctx* c, const bf16* src, const bf16* Dxm, int B) {
  const int C = c->C, m = c->m, H = c->H, W = c->W;
  const long long HWC = (long long)H * W * C, HC = (long long)H * C;
  GemmArgs g = ga();
  g.M = 2 * m; g.N = C; g.K = W;
  g.nb1 = B; g.nb2 = H;
  g.A = op(Dxm, W, 1);
  g.B = op(src, C, 1, HWC, (long long)W * C);
  g.C = c->T1; g.c_bf16 = 1;
  g.sC1 = 2LL * m * HC; g.sC2 = C; g.rC = HC; g.cC = 1;
  return cgemm(c, g);
}
bool y_specialized(const fno_ctx* c) { return c->specialized && c->C == 32 && c->m == 16 && c->H == 128; }

// (the k_y step alone, from T1)
int spectral_analysis_y(fno_ctx* c, bf16* dst, int B) {
  const int C = c->C, m = c->m, H = c->H;
  const long long HC = (long long)H * C;
  if (y_specialized(c)) {
    const std::pair<const char*, size_t>* none = nullptr;
    const long long items = (long long)B * m;
    if (!inside(c, c->T1, items * 2 * H * C - 1, 2, none, 0) || !inside(c, dst, items * 4 * m * C - 1, 2, none, 0) ||
        !inside(c, c->DyRe, 4LL * m * H - 1, 2, none, 0) || !inside(c, c->DyIm, 4LL * m * H - 1, 2, none, 0))
      return ffail(TTSH_EINVAL, "k_y analysis operand out of bounds (internal layout error)");
    hipLaunchKernelGGL(k_yanalysis, dim3((unsigned)std::min<long long>(items, 1024)), dim3(256), 0, c->s, c->T1,
                       c->DyRe, c->DyIm, dst, B, items);
    FCHK(hipGetLastError());
    return TTSH_OK;
  }
  // dst[kx] (4m x C per b) = DyRe . T1_re + DyIm . T1_im
  GemmArgs h = ga();
  h.M = 4 * m; h.N = C; h.K = H; h.K2 = H;
  h.nb1 = B; h.nb2 = m;
  h.A = op(c->DyRe, H, 1);
  h.B = op(c->T1, C, 1, 2LL * m * HC, HC);
  h.A2 = op(c->DyIm, H, 1);
  h.B2 = op(c->T1 + (long long)m * HC, C, 1, 2LL * m * HC, HC);
  h.C = dst; h.c_bf16 = 1;
  h.sC1 = C; h.sC2 = 4LL * m * B * C; h.rC = (long long)B * C; h.cC = 1;
  return cgemm(c, h);
}
int spectral_analysis(fno_ctx* c, const bf16* src, const bf16* Dxm, bf16* dst, int B) {
  int rc;
  if ((rc = spectral_analysis_x(c, src, Dxm, B))) return rc;
  return spectral_analysis_y(c, dst, B);
}

bool tail_fusable(const fno_ctx* c) { return c->specialized && c->C == 32 && c->m == 16 && c->W == 128; }

// out[0:n] = sum over the nparts vectors part[c][0:n] in a fixed order: two
// passes (k_reduce_chunks, k_reduce_sums) when the chunk sums fit their
// buffer, else the one-pass k_reduce_parts
int reduce_parts(fno_ctx* c, const float* part, long long nparts, long long n, float* out) {
  const long long nch = (nparts + kRedChunk - 1) / kRedChunk;
  if (nparts > kRedChunk && nch <= 65535 && (size_t)(nch * n) <= c->red2_n) {
    hipLaunchKernelGGL(k_reduce_chunks, dim3(nb(n), (unsigned)nch), dim3(256), 0, c->s, part, (int)nparts, n,
                       c->red2);
    hipLaunchKernelGGL(k_reduce_sums, dim3(nb(n)), dim3(256), 0, c->s, c->red2, (int)nch, n, out);
  } else {
    hipLaunchKernelGGL(k_reduce_parts, dim3(nb(n, 16)), dim3(256), 0, c->s, part, (int)nparts, n, out);
  }
  FCHK(hipGetLastError());
  return TTSH_OK;
}

// Backward tail of layer l: dh_l = Ax1 T2 + dz W_l^T into `out`; for l > 0
// multiplied by GELU'(z[l-1]) (the next gradient dz) with its k_x transform
// (DxG) into T1.  With bias_grad, the column sums of what it stores (the bias
// gradient of layer l - 1, or of the lift for l = 0) go there: per-workgroup
// partial sums, then reduce_parts.
int layer_tail_back(fno_ctx* c, int l, int B, const bf16* dz, bf16* out, float* bias_grad) {
  const long long rows = (long long)B * c->H, P = rows * c->W;
  const std::pair<const char*, size_t>* none = nullptr;
  const bf16* zin = l > 0 ? c->z[l - 1] : nullptr;
  if (!inside(c, dz, P * 32 - 1, 2, none, 0) || !inside(c, out, P * 32 - 1, 2, none, 0) ||
      !inside(c, c->T2, rows * 32 * 32 - 1, 2, none, 0) || !inside(c, c->T1, rows * 32 * 32 - 1, 2, none, 0) ||
      !inside(c, zin, P * 32 - 1, 2, none, 0) || !inside(c, c->Ax1, 128 * 32 - 1, 2, none, 0) ||
      !inside(c, c->DxG, 32 * 128 - 1, 2, none, 0) || !inside(c, c->WlT[l], 32 * 32 - 1, 2, none, 0))
    return ffail(TTSH_EINVAL, "layer tail (backward) operand out of bounds (internal layout error)");
  const unsigned blocks = (unsigned)std::min<long long>(rows, 1280);
  if (bias_grad && (size_t)blocks * 32 > c->part_n) return ffail(TTSH_ENOMEM, "fno partials buffer too small");
  if (l > 0 && bias_grad)
    hipLaunchKernelGGL((k_layer_tail<false, true, false, true, true>), dim3(blocks), dim3(256), 0, c->s, dz, c->T2,
                       c->Ax1, c->WlT[l], nullptr, c->DxG, out, nullptr, c->T1, c->H, rows, 0, zin, c->part);
  else if (l > 0)
    hipLaunchKernelGGL((k_layer_tail<false, true, false, true>), dim3(blocks), dim3(256), 0, c->s, dz, c->T2,
                       c->Ax1, c->WlT[l], nullptr, c->DxG, out, nullptr, c->T1, c->H, rows, 0, zin, nullptr);
  else if (bias_grad)
    hipLaunchKernelGGL((k_layer_tail<false, false, false, false, true>), dim3(blocks), dim3(256), 0, c->s, dz,
                       c->T2, c->Ax1, c->WlT[l], nullptr, c->DxG, out, nullptr, c->T1, c->H, rows, 0, nullptr, c->part);
  else
    hipLaunchKernelGGL((k_layer_tail<false, false, false, false>), dim3(blocks), dim3(256), 0, c->s, dz, c->T2,
                       c->Ax1, c->WlT[l], nullptr, c->DxG, out, nullptr, c->T1, c->H, rows, 0, nullptr, nullptr);
  FCHK(hipGetLastError());
  if (bias_grad) return reduce_parts(c, c->part, blocks, 32, bias_grad);
  return TTSH_OK;
}

// The lifting layer fused with the first layer's k_x transform: h[0] and T1
// from the BF16 input xb.
int lift_tail(fno_ctx* c, int B) {
  const long long rows = (long long)B * c->H, P = rows * c->W;
  const std::pair<const char*, size_t>* none = nullptr;
  if (!inside(c, c->xb, P * c->cin - 1, 2, none, 0) || !inside(c, c->h[0], P * 32 - 1, 2, none, 0) ||
      !inside(c, c->T1, rows * 32 * 32 - 1, 2, none, 0) || !inside(c, c->Pw, (long long)c->cin * 32 - 1, 2, none, 0) ||
      !inside(c, c->Dx, 32 * 128 - 1, 2, none, 0))
    return ffail(TTSH_EINVAL, "lift operand out of bounds (internal layout error)");
  const unsigned blocks = (unsigned)std::min<long long>(rows, 1280);
  hipLaunchKernelGGL((k_layer_tail<false, true, true>), dim3(blocks), dim3(256), 0, c->s, c->xb, nullptr, nullptr,
                     c->Pw, c->theta + c->oPb, c->Dx, c->h[0], nullptr, c->T1, c->H, rows, c->cin);
  FCHK(hipGetLastError());
  return TTSH_OK;
}

// One launch of k_layer_tail for layer l (act and next: not the last layer).
// Every operand is a context buffer sized for the maximum batch.
int layer_tail(fno_ctx* c, int l, int B, bool train) {
  const bool last = l == c->L - 1;
  const long long rows = (long long)B * c->H, P = rows * c->W;
  const std::pair<const char*, size_t>* none = nullptr;
  const bf16* zp = (train && !last) ? c->z[l] : nullptr;
  if (!inside(c, c->h[l], P * 32 - 1, 2, none, 0) || !inside(c, c->h[l + 1], P * 32 - 1, 2, none, 0) ||
      !inside(c, c->T2, rows * 32 * 32 - 1, 2, none, 0) || !inside(c, c->T1, rows * 32 * 32 - 1, 2, none, 0) ||
      !inside(c, zp, P * 32 - 1, 2, none, 0) || !inside(c, c->Ax, 128 * 32 - 1, 2, none, 0) ||
      !inside(c, c->Dx, 32 * 128 - 1, 2, none, 0) || !inside(c, c->Wl[l], 32 * 32 - 1, 2, none, 0))
    return ffail(TTSH_EINVAL, "layer tail operand out of bounds (internal layout error)");
  const unsigned blocks = (unsigned)std::min<long long>(rows, 1280);
  const float* bias = c->theta + c->ob[l];
  bf16* z = train && !last ? c->z[l] : nullptr;
  if (last)
    hipLaunchKernelGGL((k_layer_tail<false, false, false>), dim3(blocks), dim3(256), 0, c->s, c->h[l], c->T2, c->Ax,
                       c->Wl[l], bias, c->Dx, c->h[l + 1], z, c->T1, c->H, rows, 0);
  else
    hipLaunchKernelGGL((k_layer_tail<true, true, false>), dim3(blocks), dim3(256), 0, c->s, c->h[l], c->T2, c->Ax,
                       c->Wl[l], bias, c->Dx, c->h[l + 1], z, c->T1, c->H, rows, 0);
  FCHK(hipGetLastError());
  return TTSH_OK;
}

// The last layer's tail fused with the projection into y (pixel stride ys,
// skip: the residual input or null).  h_L is written only where something
// reads it: the training backward, or the stage capture.
int last_tail_proj(fno_ctx* c, int B, bool train, float* y, long long ys, const float* skip) {
  const int l = c->L - 1;
  const long long rows = (long long)B * c->H, P = rows * c->W;
  const std::pair<const char*, size_t>* none = nullptr;
  bf16* hn = (train || c->capture) ? c->h[l + 1] : nullptr;
  if (!inside(c, c->h[l], P * 32 - 1, 2, none, 0) || !inside(c, hn, P * 32 - 1, 2, none, 0) ||
      !inside(c, c->T2, rows * 32 * 32 - 1, 2, none, 0) || !inside(c, c->Ax, 128 * 32 - 1, 2, none, 0) ||
      !inside(c, c->Wl[l], 32 * 32 - 1, 2, none, 0) || !inside(c, c->Q1, 32LL * 128 - 1, 2, none, 0) ||
      !inside(c, c->Q2, 128LL * c->cout - 1, 2, none, 0))
    return ffail(TTSH_EINVAL, "tail projection operand out of bounds (internal layout error)");
  const unsigned blocks = (unsigned)std::min<long long>(rows, 1280);
  hipLaunchKernelGGL((k_tail_proj<128>), dim3(blocks), dim3(256), 0, c->s, c->h[l], c->T2, c->Ax, c->Wl[l],
                     c->theta + c->ob[l], hn, c->Q1, c->theta + c->oQ1b, c->Q2, c->theta + c->oQ2b, c->cout, y, ys,
                     skip, (long long)c->cin, rows);
  FCHK(hipGetLastError());
  return TTSH_OK;
}

// Inverse along y of the mode array src [m][2m][B][2C] (real, imaginary halves
// of each channel block) into T2 [B][H][2m][C] (k_x real at kx, imaginary at m+kx).
int spectral_synth_y(fno_ctx* c, const bf16* src, int B) {
  int rc;
  const int C = c->C, m = c->m, H = c->H;
  const long long modeS = (long long)B * 2 * C;  // stride between k_y rows
  if (y_specialized(c)) {
    const std::pair<const char*, size_t>* none = nullptr;
    const long long items = (long long)B * m;
    if (!inside(c, src, 2LL * m * m * modeS - 1, 2, none, 0) || !inside(c, c->T2, (long long)B * H * 2 * m * C - 1, 2, none, 0) ||
        !inside(c, c->Ec, (long long)H * 2 * m - 1, 2, none, 0) || !inside(c, c->Es, (long long)H * 2 * m - 1, 2, none, 0) ||
        !inside(c, c->Esn, (long long)H * 2 * m - 1, 2, none, 0))
      return ffail(TTSH_EINVAL, "k_y synthesis operand out of bounds (internal layout error)");
    hipLaunchKernelGGL(k_ysynth, dim3((unsigned)std::min<long long>(items, 1024)), dim3(256), 0, c->s, src, c->Ec,
                       c->Es, c->Esn, c->T2, B, items);
    FCHK(hipGetLastError());
    return TTSH_OK;
  }
  for (int part = 0; part < 2; ++part) {
    // part 0: Fr = Ec . O_r + (-Es) . O_i ;  part 1: Fi = Es . O_r + Ec . O_i
    GemmArgs g = ga();
    g.M = H; g.N = C; g.K = 2 * m; g.K2 = 2 * m;
    g.nb1 = B; g.nb2 = m;
    g.A = op(part == 0 ? c->Ec : c->Es, 2 * m, 1);
    g.B = op(src, modeS, 1, 2LL * C, 2LL * m * modeS);
    g.A2 = op(part == 0 ? c->Esn : c->Ec, 2 * m, 1);
    g.B2 = op(src + C, modeS, 1, 2LL * C, 2LL * m * modeS);
    g.C = c->T2 + (part ? (long long)m * C : 0); g.c_bf16 = 1;
    g.sC1 = (long long)H * 2 * m * C; g.sC2 = C; g.rC = 2LL * m * C; g.cC = 1;
    if ((rc = cgemm(c, g))) return rc;
  }
  return TTSH_OK;
}

// Mode mixing: out[kx][q][b][0:2C] = [G_r, G_i][b] . Wb (forward) or Wb^T (adjoint)
int spectral_mix(fno_ctx* c, const bf16* G, const bf16* Wb, const bf16* WbT, bool transpose, bf16* out, int B) {
  int rc;
  const int C = c->C, m = c->m;
  const long long C2 = 2LL * C;
  if (c->specialized && C == 32) {
    const std::pair<const char*, size_t>* none = nullptr;
    const bf16* Vt = transpose ? Wb : WbT;
    const long long modes = 2LL * m * m;
    if (!inside(c, G, modes * 2 * B * C - 1, 2, none, 0) || !inside(c, Vt, modes * C2 * C2 - 1, 2, none, 0) ||
        !inside(c, out, modes * B * C2 - 1, 2, none, 0))
      return ffail(TTSH_EINVAL, "mode mixing operand out of bounds (internal layout error)");
    hipLaunchKernelGGL(k_mix, dim3((unsigned)modes), dim3(256), 0, c->s, G, Vt, out, B, m);
    FCHK(hipGetLastError());
    return TTSH_OK;
  }
  GemmArgs g = ga();
  g.M = B; g.N = 2 * C; g.K = C; g.K2 = C;
  g.nb1 = m; g.nb2 = 2 * m;
  g.A = op(G, C, 1, 4LL * m * B * C, (long long)B * C);
  g.A2 = op(G + 2LL * m * B * C, C, 1, 4LL * m * B * C, (long long)B * C);
  const long long wS1 = 2LL * m * C2 * C2, wS2 = C2 * C2;
  if (!transpose) {
    g.B = op(Wb, C2, 1, wS1, wS2);
    g.B2 = op(Wb + C * C2, C2, 1, wS1, wS2);
  } else {  // B[k][j] = Wb[j][k]
    g.B = op(Wb, 1, C2, wS1, wS2);
    g.B2 = op(Wb + C, 1, C2, wS1, wS2);
  }
  g.C = out; g.c_bf16 = 1;
  g.sC1 = 2LL * m * B * C2; g.sC2 = B * C2; g.rC = C2; g.cC = 1;
  if ((rc = cgemm(c, g))) return rc;
  return TTSH_OK;
}

long long pts(const fno_ctx* c, int B) { return (long long)B * c->H * c->W; }


// element counts of the captured buffers at the maximum batch
long long cap_len_T(const fno_ctx* c) { return (long long)c->maxB * 2 * c->m * c->H * c->C; }  // T1, T2
long long cap_len_O(const fno_ctx* c) { return (long long)c->m * 2 * c->m * c->maxB * 2 * c->C; }  // O, gF, gG
long long cap_len_P(const fno_ctx* c) { return pts(c, c->maxB) * c->C; }  // dz, dh

// copy n elements of src into a capture slot when capturing (stream-ordered)
int cap_copy(fno_ctx* c, bf16* dst, const bf16* src, long long n) {
  if (!c->capture || !dst) return TTSH_OK;
  FCHK(hipMemcpyAsync(dst, src, (size_t)n * sizeof(bf16), hipMemcpyDeviceToDevice, c->s));
  return TTSH_OK;
}

// points per partial product of a weight gradient: short enough that the
// partial products (one wavefront per 32 x 32 tile each) fill the chip
constexpr long long kWgradChunk = 1024;

// split-K weight gradient: out (M x N, float, += into grad) = A^T-like product
// over the point axis.  A[i][p] at A + i*rA + p*cA, B[p][j] at B + p*rB + j*cB.
int wgrad(fno_ctx* c, int M, int N, long long P, const bf16* A, long long rA, long long cA, const bf16* Bm,
          long long rB, long long cB, float* out) {
  int rc;
  const long long chunk = kWgradChunk;
  const long long nchunk = (P + chunk - 1) / chunk;
  if ((size_t)(nchunk * M * N) > c->part_n) return ffail(TTSH_ENOMEM, "fno partials buffer too small");
  GemmArgs g = ga();
  g.M = M; g.N = N; g.K = (int)chunk;
  g.nb1 = (int)nchunk; g.nb2 = 1;
  g.A = op(A, rA, cA, chunk * cA, 0);
  g.B = op(Bm, rB, cB, chunk * rB, 0);
  g.C = c->part; g.c_bf16 = 0;
  g.sC1 = (long long)M * N; g.rC = N; g.cC = 1;
  // the last chunk may be short: handled by passing K per call below
  if (P % chunk == 0) {
    if ((rc = cgemm(c, g))) return rc;
  } else {
    g.nb1 = (int)(nchunk - 1);
    if (g.nb1 > 0) if ((rc = cgemm(c, g))) return rc;
    GemmArgs t = g;
    t.nb1 = 1;
    t.K = (int)(P - (nchunk - 1) * chunk);
    t.A.p = A + (nchunk - 1) * chunk * cA;
    t.B.p = Bm + (nchunk - 1) * chunk * rB;
    t.C = c->part + (nchunk - 1) * M * N;
    if ((rc = cgemm(c, t))) return rc;
  }
  return reduce_parts(c, c->part, nchunk, (long long)M * N, out);
}

int colsum(fno_ctx* c, const bf16* a, long long rows, int ncol, float* out) {
  const bool vec = ncol % 8 == 0 && ncol <= 256 && ((ncol / 8) & (ncol / 8 - 1)) == 0 && ((uintptr_t)a & 15) == 0;
  const long long chunk = vec ? 2048 : 8192;
  const long long nchunk = (rows + chunk - 1) / chunk;
  if ((size_t)(nchunk * ncol) > c->part_n) return ffail(TTSH_ENOMEM, "fno partials buffer too small");
  if (vec) {
    hipLaunchKernelGGL(k_colsum_part8, dim3((unsigned)nchunk), dim3(256), 0, c->s, a, rows, ncol, chunk, c->part);
  } else {
    const int lanes = std::max(1, std::min(1024 / ncol, 64));
    hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)nchunk), dim3(lanes * ncol), 0, c->s, a, rows, ncol, chunk,
                       c->part);
  }
  FCHK(hipGetLastError());
  return reduce_parts(c, c->part, nchunk, (long long)ncol, out);
}

void free_fno(fno_ctx* c) {
  if (!c) return;
  for (void* p : c->allocs) hipFree(p);
  delete c;
}

}  // namespace

extern "C" {

int fno_create(fno_ctx** out, int width, int modes, int layers, int cin, int cout, int hidden, int H, int W,
               int max_batch, uint64_t seed, void* stream) {
  if (!out) return ffail(TTSH_EINVAL, "null output");
  *out = nullptr;
  if (width < 1 || width > 256 || modes < 1 || layers < 1 || layers > 16 || cin < 1 || cin > 16 || cout < 1 ||
      cout > 16 || hidden < 1 || hidden > 1024 || H < 16 || W < 16 || H % 16 || W % 16 || 2 * modes > H ||
      modes > W / 2 || max_batch < 1 || (long long)max_batch * H * W > (1LL << 31) / 256)
    return ffail(TTSH_EINVAL, "fno_create: invalid sizes");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return ffail(TTSH_EHIP, "no HIP device available");
  fno_ctx* c = new fno_ctx();
  c->C = width; c->m = modes; c->L = layers; c->cin = cin; c->cout = cout; c->hid = hidden;
  c->H = H; c->W = W; c->maxB = max_batch; c->s = (hipStream_t)stream;
  const long long C = width, m = modes;
  int64_t o = 0;
  c->oPw = o; o += cin * C;
  c->oPb = o; o += C;
  for (int l = 0; l < layers; ++l) {
    c->oR[l] = o; o += 2 * (2 * m * m * C * C);
    c->oW[l] = o; o += C * C;
    c->ob[l] = o; o += C;
  }
  c->oQ1 = o; o += C * hidden;
  c->oQ1b = o; o += hidden;
  c->oQ2 = o; o += (long long)hidden * cout;
  c->oQ2b = o; o += cout;
  c->nparam = o;
  auto bail = [&](int rc) { free_fno(c); return rc; };
  int rc;
  const long long P = (long long)max_batch * H * W;
  const long long modesz = (long long)m * 4 * m * max_batch * C;
  if ((rc = alloc(c, &c->theta, o)) || (rc = alloc(c, &c->grad, o)) || (rc = alloc(c, &c->m1, o)) ||
      (rc = alloc(c, &c->m2, o)) || (rc = alloc(c, &c->Pw, (size_t)(cin * C))) ||
      (rc = alloc(c, &c->Q1, (size_t)(C * hidden))) || (rc = alloc(c, &c->Q2, (size_t)(hidden * cout))) ||
      (rc = alloc(c, &c->xb, (size_t)(P * cin))) || (rc = alloc(c, &c->T1, (size_t)(max_batch * 2 * m * H * C))) ||
      (rc = alloc(c, &c->T2, (size_t)(max_batch * 2 * m * H * C))) || (rc = alloc(c, &c->O, (size_t)modesz)) ||
      (rc = alloc(c, &c->u, (size_t)(P * hidden))) || (rc = alloc(c, &c->a, (size_t)(P * hidden))) ||
      (rc = alloc(c, &c->dy, (size_t)(P * cout))) || (rc = alloc(c, &c->dh0, (size_t)(P * C))) ||
      (rc = alloc(c, &c->dh1, (size_t)(P * C))) || (rc = alloc(c, &c->dz, (size_t)(P * C))) ||
      (rc = alloc(c, &c->gG, (size_t)modesz)) || (rc = alloc(c, &c->gF, (size_t)modesz)) ||
      (rc = alloc(c, &c->du, (size_t)(P * hidden))) || (rc = alloc(c, &c->lsum, (size_t)(2 * max_batch))) ||
      (rc = alloc(c, &c->gidx, (size_t)max_batch)) || (rc = alloc(c, &c->gsym, (size_t)max_batch)))
    return bail(rc);
  for (int l = 0; l <= layers; ++l)
    if ((rc = alloc(c, &c->h[l], (size_t)(P * C)))) return bail(rc);
  for (int l = 0; l < layers; ++l)
    if ((rc = alloc(c, &c->z[l], (size_t)(P * C))) || (rc = alloc(c, &c->G[l], (size_t)modesz)) ||
        (rc = alloc(c, &c->Wl[l], (size_t)(C * C))) || (rc = alloc(c, &c->WlT[l], (size_t)(C * C))) ||
        (rc = alloc(c, &c->Wb[l], (size_t)(2 * m * m * 4 * C * C))) ||
        (rc = alloc(c, &c->WbT[l], (size_t)(2 * m * m * 4 * C * C))))
      return bail(rc);
  // partial sums of the split-K reductions: (points / kWgradChunk) x the largest gradient block
  const long long maxblk = std::max<long long>({C * C, C * hidden, (long long)hidden * cout, cin * C});
  c->part_n = (size_t)((P + kWgradChunk - 1) / kWgradChunk + 1) * (size_t)std::max<long long>(maxblk, 1024);
  // (and 2048 wavefront slots of the fused projection backward: two workgroups per CU)
  c->part_n = std::max<size_t>(c->part_n, (size_t)2048 * (size_t)(C * hidden + hidden + (long long)hidden * cout + cout));
  if ((rc = alloc(c, &c->part, c->part_n))) return bail(rc);
  c->red2_n = c->part_n / kRedChunk + 65536;
  if ((rc = alloc(c, &c->red2, c->red2_n))) return bail(rc);
  if ((rc = make_dft(c))) return bail(rc);
  // seeded initial parameters (same distributions as the oracle's)
  std::vector<float> th(o, 0.f);
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::uniform_real_distribution<double> ud(0.0, 1.0);
  for (long long i = 0; i < cin * C; ++i) th[c->oPw + i] = (float)(nd(gen) / sqrt((double)cin));
  for (int l = 0; l < layers; ++l) {
    for (long long i = 0; i < 2 * (2 * m * m * C * C); ++i) th[c->oR[l] + i] = (float)(ud(gen) / (double)(C * C));
    for (long long i = 0; i < C * C; ++i) th[c->oW[l] + i] = (float)(nd(gen) / sqrt((double)C));
  }
  for (long long i = 0; i < C * hidden; ++i) th[c->oQ1 + i] = (float)(nd(gen) / sqrt((double)C));
  for (long long i = 0; i < (long long)hidden * cout; ++i) th[c->oQ2 + i] = (float)(nd(gen) / sqrt((double)hidden));
  if (hipMemcpy(c->theta, th.data(), o * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(c->m1, 0, o * 4) != hipSuccess || hipMemset(c->m2, 0, o * 4) != hipSuccess ||
      hipMemset(c->grad, 0, o * 4) != hipSuccess)
    return bail(ffail(TTSH_EHIP, "parameter upload failed"));
  if ((rc = refresh_weights(c))) return bail(rc);
  if (hipStreamSynchronize(c->s) != hipSuccess) return bail(ffail(TTSH_EHIP, "sync failed"));
  *out = c;
  return TTSH_OK;
}

void fno_destroy(fno_ctx* c) {
  if (!c) return;
  hipStreamSynchronize(c->s);
  free_fno(c);
}

int64_t fno_num_params(fno_ctx* c) { return c ? c->nparam : (int64_t)ffail(TTSH_EINVAL, "null context"); }

int fno_set_params(fno_ctx* c, const float* p) {
  if (!c || !p) return ffail(TTSH_EINVAL, "null argument");
  FCHK(hipMemcpy(c->theta, p, c->nparam * 4, hipMemcpyHostToDevice));
  c->adam_t = 0;
  FCHK(hipMemset(c->m1, 0, c->nparam * 4));
  FCHK(hipMemset(c->m2, 0, c->nparam * 4));
  int rc = refresh_weights(c);
  if (rc) return rc;
  FCHK(hipStreamSynchronize(c->s));
  return TTSH_OK;
}

int fno_get_params(fno_ctx* c, float* p) {
  if (!c || !p) return ffail(TTSH_EINVAL, "null argument");
  FCHK(hipStreamSynchronize(c->s));
  FCHK(hipMemcpy(p, c->theta, c->nparam * 4, hipMemcpyDeviceToHost));
  return TTSH_OK;
}

int fno_get_grads(fno_ctx* c, float* p) {
  if (!c || !p) return ffail(TTSH_EINVAL, "null argument");
  FCHK(hipStreamSynchronize(c->s));
  FCHK(hipMemcpy(p, c->grad, c->nparam * 4, hipMemcpyDeviceToHost));
  return TTSH_OK;
}

int fno_set_option(fno_ctx* c, int option, int value) {
  if (!c) return ffail(TTSH_EINVAL, "null context");
  if (option == FNO_OPT_STAGED_GEMM) c->staged_gemm = value != 0;
  else if (option == FNO_OPT_SPECIALIZED) c->specialized = value != 0;
  else if (option == FNO_OPT_TAIL_PROJ) c->tail_proj = value != 0;
  else if (option == FNO_OPT_CAPTURE) {
    if (value && !c->capT1[0]) {  // buffers are allocated once, on first use
      int rc;
      const long long nT = cap_len_T(c), nO = cap_len_O(c), nP = cap_len_P(c);
      for (int l = 0; l < c->L; ++l)
        if ((rc = alloc(c, &c->capT1[l], nT)) || (rc = alloc(c, &c->capO[l], nO)) || (rc = alloc(c, &c->capT2[l], nT)) ||
            (rc = alloc(c, &c->capDZ[l], nP)) || (rc = alloc(c, &c->capBT1[l], nT)) ||
            (rc = alloc(c, &c->capGG[l], nO)) || (rc = alloc(c, &c->capGF[l], nO)) ||
            (rc = alloc(c, &c->capBT2[l], nT)) || (rc = alloc(c, &c->capDH[l], nP)))
          return rc;
      if ((rc = alloc(c, &c->capDHL, nP))) return rc;
    }
    c->capture = value != 0;
  } else {
    return ffail(TTSH_EINVAL, "unknown option");
  }
  return TTSH_OK;
}

int fno_capture(fno_ctx* c, int what, int layer, float* out, int64_t n) {
  if (!c || !out) return ffail(TTSH_EINVAL, "null argument");
  if (!c->capT1[0]) return ffail(TTSH_EINVAL, "capture was never enabled");
  const bool per_layer = what != FNO_CAP_XB && what != FNO_CAP_DHL && what != FNO_CAP_H && what != FNO_CAP_DY;
  if (what == FNO_CAP_H ? (layer < 0 || layer > c->L) : (per_layer && (layer < 0 || layer >= c->L)))
    return ffail(TTSH_EINVAL, "layer out of range");
  const bf16* src = nullptr;
  long long len = 0;
  const long long nT = cap_len_T(c), nO = cap_len_O(c), nP = cap_len_P(c);
  switch (what) {
    case FNO_CAP_XB: src = c->xb; len = pts(c, c->maxB) * c->cin; break;
    case FNO_CAP_H: src = c->h[layer]; len = nP; break;
    case FNO_CAP_Z: src = c->z[layer]; len = layer < c->L - 1 ? nP : 0; break;
    case FNO_CAP_T1: src = c->capT1[layer]; len = nT; break;
    case FNO_CAP_G: src = c->G[layer]; len = (long long)c->m * 4 * c->m * c->maxB * c->C; break;
    case FNO_CAP_O: src = c->capO[layer]; len = nO; break;
    case FNO_CAP_T2: src = c->capT2[layer]; len = nT; break;
    case FNO_CAP_DZ: src = c->capDZ[layer]; len = nP; break;
    case FNO_CAP_BT1: src = c->capBT1[layer]; len = nT; break;
    case FNO_CAP_GG: src = c->capGG[layer]; len = nO; break;
    case FNO_CAP_GF: src = c->capGF[layer]; len = nO; break;
    case FNO_CAP_BT2: src = c->capBT2[layer]; len = nT; break;
    case FNO_CAP_DH: src = c->capDH[layer]; len = nP; break;
    case FNO_CAP_DHL: src = c->capDHL; len = nP; break;
    case FNO_CAP_DY: src = c->dy; len = pts(c, c->maxB) * c->cout; break;
    default: return ffail(TTSH_EINVAL, "unknown capture item");
  }
  if (!src || len == 0) return ffail(TTSH_EINVAL, "nothing captured for this item");
  if (n < 1 || n > len) return ffail(TTSH_EINVAL, "element count out of range");
  std::vector<bf16> h((size_t)n);
  FCHK(hipStreamSynchronize(c->s));
  FCHK(hipMemcpy(h.data(), src, (size_t)n * sizeof(bf16), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i) out[i] = bf2f(h[(size_t)i]);
  return TTSH_OK;
}

int fno_forward(fno_ctx* c, const float* x, float* y, int B, int train) {
  return c ? fno_forward_ex(c, x, y, c->cout, 0, B, train) : ffail(TTSH_EINVAL, "null context");
}

int fno_forward_ex(fno_ctx* c, const float* x, float* y, int64_t ys, int residual, int B, int train) {
  if (!c || !x || !y) return ffail(TTSH_EINVAL, "null argument");
  if (ys < c->cout) return ffail(TTSH_EINVAL, "output pixel stride smaller than cout");
  if (B < 1 || B > c->maxB) return ffail(TTSH_EINVAL, "batch out of range");
  if (residual && c->cout > c->cin) return ffail(TTSH_EINVAL, "residual output needs cout <= cin");
  const int C = c->C, m = c->m, H = c->H, W = c->W;
  const long long P = pts(c, B);
  {
    // an output that overlaps the input must be the input's own first channels
    const char *x0 = (const char*)x, *x1 = x0 + P * c->cin * sizeof(float);
    const char *y0 = (const char*)y, *y1 = y0 + ((P - 1) * ys + c->cout) * sizeof(float);
    if (y0 < x1 && x0 < y1 && !(y0 == x0 && ys == c->cin))
      return ffail(TTSH_EINVAL, "output overlaps the input other than as its first channels");
  }
  hipLaunchKernelGGL(k_to_bf16, dim3(nb(P * c->cin)), dim3(256), 0, c->s, x, c->xb, P * c->cin);
  const bool fuse = tail_fusable(c);
  const bool fuse_lift = fuse && c->cin <= kMaxLiftCin;
  int rc;
  if (fuse_lift) {
    if ((rc = lift_tail(c, B))) return rc;
  } else if (C % 8 == 0)
    hipLaunchKernelGGL(k_lift8, dim3(nb(P * (C / 8))), dim3(256), 0, c->s, c->xb, c->Pw, c->theta + c->oPb,
                       c->h[0], P, c->cin, C);
  else
    hipLaunchKernelGGL(k_lift, dim3(nb(P * C)), dim3(256), 0, c->s, c->xb, c->Pw, c->theta + c->oPb, c->h[0], P,
                       c->cin, C);
  FCHK(hipGetLastError());
  // the fused projection: always for inference; in training too with the
  // specialized kernels, whose fused backward recomputes the hidden layer
  const bool proj_fused = C == 32 && c->hid == 128 && c->cout <= 16 &&
                          (!train || (c->specialized && c->cout <= kProjBackMaxCout));
  c->proj_train_fused = train && proj_fused;
  for (int l = 0; l < c->L; ++l) {
    const bool last = l == c->L - 1;
    // with the fused tail (and lift), the previous step already left T1 (the k_x step of h_l)
    if (l == 0 ? !fuse_lift : !fuse)
      if ((rc = spectral_analysis_x(c, c->h[l], c->Dx, B))) return rc;
    if ((rc = cap_copy(c, c->capT1[l], c->T1, (long long)B * 2 * m * H * C))) return rc;
    if ((rc = spectral_analysis_y(c, c->G[l], B))) return rc;
    if ((rc = spectral_mix(c, c->G[l], c->Wb[l], c->WbT[l], false, c->O, B))) return rc;
    if ((rc = cap_copy(c, c->capO[l], c->O, (long long)m * 2 * m * B * 2 * C))) return rc;
    if ((rc = spectral_synth_y(c, c->O, B))) return rc;
    if ((rc = cap_copy(c, c->capT2[l], c->T2, (long long)B * H * 2 * m * C))) return rc;
    if (fuse) {
      if (last && proj_fused && c->tail_proj)
        return last_tail_proj(c, B, train != 0, y, (long long)ys, residual ? x : nullptr);
      if ((rc = layer_tail(c, l, B, train != 0))) return rc;
      continue;
    }
    // h_{l+1} = act(Ax . T2[b][y] + h_l[b][y] . W_l + b_l)
    GemmArgs g = ga();
    g.M = W; g.N = C; g.K = 2 * m; g.K2 = C;
    g.nb1 = B; g.nb2 = H;
    g.A = op(c->Ax, 2 * m, 1);
    g.B = op(c->T2, C, 1, (long long)H * 2 * m * C, 2LL * m * C);
    g.A2 = op(c->h[l], C, 1, (long long)H * W * C, (long long)W * C);
    g.B2 = op(c->Wl[l], C, 1);
    g.C = c->h[l + 1]; g.c_bf16 = 1;
    g.sC1 = (long long)H * W * C; g.sC2 = (long long)W * C; g.rC = C; g.cC = 1;
    g.bias = c->theta + c->ob[l];
    if (!last) {
      g.act = 1;
      if (train) g.pre_out = c->z[l];  // pre-activations are kept for the backward pass only
    }
    if ((rc = cgemm(c, g))) return rc;
  }
  if (proj_fused) {
    // h_L is [P][C] (inside h[L]), y and skip were range-checked above
    const long long tiles = (P + 15) / 16;
    const long long blocks = std::min<long long>((tiles + 4 * kProjGroups - 1) / (4 * kProjGroups), 8192);
    hipLaunchKernelGGL((k_proj_fused<32, 128, kProjGroups>), dim3((unsigned)blocks), dim3(256), 0, c->s, c->h[c->L], c->Q1,
                       c->theta + c->oQ1b, c->Q2, c->theta + c->oQ2b, c->cout, y, (long long)ys,
                       residual ? x : nullptr, (long long)c->cin, P);
    FCHK(hipGetLastError());
    return TTSH_OK;
  }
  // projection: a = GELU(h_L Q1 + Q1_b) (pre-activation u kept), y = a Q2 + Q2_b
  GemmArgs g = ga();
  g.M = (int)P; g.N = c->hid; g.K = C;
  g.A = op(c->h[c->L], C, 1);
  g.B = op(c->Q1, c->hid, 1);
  g.C = c->a; g.c_bf16 = 1; g.rC = c->hid; g.cC = 1;
  g.bias = c->theta + c->oQ1b; g.act = 1; g.pre_out = c->u;
  if ((rc = cgemm(c, g))) return rc;
  GemmArgs q = ga();
  q.M = (int)P; q.N = c->cout; q.K = c->hid;
  q.A = op(c->a, c->hid, 1);
  q.B = op(c->Q2, c->cout, 1);
  q.C = y; q.c_bf16 = 0; q.rC = ys; q.cC = 1;
  q.bias = c->theta + c->oQ2b;
  if (residual) {
    q.skip = x;
    q.skip_r = c->cin;
  }
  const std::pair<const char*, size_t> ext[2] = {
      {(const char*)y, (size_t)((P - 1) * ys + c->cout) * sizeof(float)},
      {(const char*)x, (size_t)(P * c->cin) * sizeof(float)}};
  if ((rc = cgemm(c, q, ext, 2))) return rc;
  return TTSH_OK;
}

int fno_loss(fno_ctx* c, const float* y, const float* t, int B, double* loss) {
  return fno_loss_ex(c, y, t, nullptr, 0, B, loss);
}

int fno_loss_ex(fno_ctx* c, const float* y, const float* t, const float* ref, int64_t ref_stride, int B,
                double* loss) {
  if (!c || !y || !t || !loss) return ffail(TTSH_EINVAL, "null argument");
  if (B < 1 || B > c->maxB) return ffail(TTSH_EINVAL, "batch out of range");
  if (ref && ref_stride < c->cout) return ffail(TTSH_EINVAL, "reference pixel stride smaller than cout");
  const long long per = (long long)c->H * c->W * c->cout;
  hipLaunchKernelGGL(k_loss_sums, dim3(B), dim3(1024), 0, c->s, y, t, per, ref, (long long)ref_stride, c->cout,
                     c->lsum);
  hipLaunchKernelGGL(k_loss_grad, dim3(nb(per * B)), dim3(256), 0, c->s, y, t, c->lsum, per, B, c->dy);
  FCHK(hipGetLastError());
  std::vector<double> h(2 * B);
  FCHK(hipMemcpyAsync(h.data(), c->lsum, 2 * B * sizeof(double), hipMemcpyDeviceToHost, c->s));
  FCHK(hipStreamSynchronize(c->s));
  double acc = 0.0;
  for (int s = 0; s < B; ++s) acc += sqrt(h[2 * s]) / sqrt(h[2 * s + 1]);
  *loss = acc / B;
  return TTSH_OK;
}

int fno_backward(fno_ctx* c, int B) {
  if (!c) return ffail(TTSH_EINVAL, "null context");
  if (B < 1 || B > c->maxB) return ffail(TTSH_EINVAL, "batch out of range");
  const int C = c->C, m = c->m, H = c->H, W = c->W, hid = c->hid, co = c->cout;
  const long long P = pts(c, B);
  int rc;
  // projection
  if (c->proj_train_fused) {
    // one slot of partial gradients per wavefront, [dQ1 | db1 | dQ2 | db2] as in the parameter vector
    const long long S = (long long)C * hid + hid + (long long)hid * co + co;
    const long long groups = (P + 15) / 16;
    const long long blocks = std::max<long long>(1, std::min<long long>({(groups + 3) / 4, 512, (long long)c->part_n / (4 * S)}));
    const std::pair<const char*, size_t>* none = nullptr;
    if ((long long)c->part_n < 4 * S || !inside(c, c->h[c->L], P * C - 1, 2, none, 0) ||
        !inside(c, c->dy, P * co - 1, 2, none, 0) || !inside(c, c->dh0, P * C - 1, 2, none, 0))
      return ffail(TTSH_EINVAL, "projection backward operand out of bounds (internal layout error)");
    hipLaunchKernelGGL((k_proj_back<32, 128>), dim3((unsigned)blocks), dim3(256), 0, c->s, c->h[c->L], c->Q1,
                       c->theta + c->oQ1b, c->Q2, c->dy, co, c->dh0, c->part, P);
    FCHK(hipGetLastError());
    if ((rc = reduce_parts(c, c->part, blocks * 4, S, c->grad + c->oQ1))) return rc;
  } else {
  if ((rc = wgrad(c, hid, co, P, c->a, 1, hid, c->dy, co, 1, c->grad + c->oQ2))) return rc;
  if ((rc = colsum(c, c->dy, P, co, c->grad + c->oQ2b))) return rc;
  GemmArgs g = ga();  // du = (dy Q2^T) * GELU'(u)
  g.M = (int)P; g.N = hid; g.K = co;
  g.A = op(c->dy, co, 1);
  g.B = op(c->Q2, 1, co);
  g.C = c->du; g.c_bf16 = 1; g.rC = hid; g.cC = 1;
  g.act = 2; g.pre_in = c->u;
  if ((rc = cgemm(c, g))) return rc;
  if ((rc = wgrad(c, C, hid, P, c->h[c->L], 1, C, c->du, hid, 1, c->grad + c->oQ1))) return rc;
  if ((rc = colsum(c, c->du, P, hid, c->grad + c->oQ1b))) return rc;
  GemmArgs d = ga();  // dh_L = du Q1^T
  d.M = (int)P; d.N = C; d.K = hid;
  d.A = op(c->du, hid, 1);
  d.B = op(c->Q1, 1, hid);
  d.C = c->dh0; d.c_bf16 = 1; d.rC = C; d.cC = 1;
  if ((rc = cgemm(c, d))) return rc;
  }
  if ((rc = cap_copy(c, c->capDHL, c->dh0, P * C))) return rc;
  // with the specialized kernels each layer's backward tail leaves the next
  // gradient already multiplied by GELU' (in dh) and its k_x transform (in T1)
  const bool fuse_b = tail_fusable(c);
  bf16* dh = c->dh0;
  bf16* dh_next = c->dh1;
  for (int l = c->L - 1; l >= 0; --l) {
    const bf16* dz = dh;
    if (l < c->L - 1 && !fuse_b) {
      // P * C is a multiple of 8: P = batch H W with H, W multiples of 16
      hipLaunchKernelGGL(k_gelu_back, dim3(nb((P * C + 7) / 8)), dim3(256), 0, c->s, dh, c->z[l], c->dz, P * C);
      FCHK(hipGetLastError());
      dz = c->dz;
      // the gradient layer l + 1 hands down, in the fused tail's form dl/dz_l
      if ((rc = cap_copy(c, c->capDH[l + 1], dz, P * C))) return rc;
    }
    if ((rc = cap_copy(c, c->capDZ[l], dz, P * C))) return rc;
    if ((rc = wgrad(c, C, C, P, c->h[l], 1, C, dz, C, 1, c->grad + c->oW[l]))) return rc;
    // (with the fused backward tails, layer l + 1's tail summed dz already)
    if (!(fuse_b && l < c->L - 1))
      if ((rc = colsum(c, dz, P, C, c->grad + c->ob[l]))) return rc;
    // g_G = (w/(HW)) trunc rfft2(dz)
    if (!fuse_b || l == c->L - 1)
      if ((rc = spectral_analysis_x(c, dz, c->DxG, B))) return rc;
    if ((rc = cap_copy(c, c->capBT1[l], c->T1, (long long)B * 2 * m * H * C))) return rc;
    if ((rc = spectral_analysis_y(c, c->gG, B))) return rc;
    if ((rc = cap_copy(c, c->capGG[l], c->gG, (long long)m * 4 * m * B * C))) return rc;
    // dR per mode (kx, q): dR_r = F_r^T gG_r + F_i^T gG_i ; dR_i = F_r^T gG_i - F_i^T gG_r
    const long long nR = 2LL * m * m * C * C;
    for (int part = 0; part < 2; ++part) {
      GemmArgs r = ga();
      r.M = C; r.N = C; r.K = B; r.K2 = B;
      r.nb1 = m; r.nb2 = 2 * m;
      const long long s1 = 4LL * m * B * C, s2 = (long long)B * C, im = 2LL * m * B * C;
      r.A = op(c->G[l], 1, C, s1, s2);                 // F_r^T
      r.A2 = op(c->G[l] + im, 1, C, s1, s2);           // F_i^T
      if (part == 0) {
        r.B = op(c->gG, C, 1, s1, s2);
        r.B2 = op(c->gG + im, C, 1, s1, s2);
      } else {
        r.B = op(c->gG + im, C, 1, s1, s2);
        r.B2 = op(c->gG, C, 1, s1, s2);
        r.alpha2 = -1.f;
      }
      r.C = c->grad + c->oR[l] + part * nR; r.c_bf16 = 0;
      r.sC1 = (long long)C * C; r.sC2 = (long long)m * C * C; r.rC = C; r.cC = 1;
      if ((rc = cgemm(c, r))) return rc;
    }
    // g_F = g_G Wb^T  (into gF, mode layout [m][2m][B][2C])
    if ((rc = spectral_mix(c, c->gG, c->Wb[l], c->WbT[l], true, c->gF, B))) return rc;
    if ((rc = cap_copy(c, c->capGF[l], c->gF, (long long)m * 2 * m * B * 2 * C))) return rc;
    if ((rc = spectral_synth_y(c, c->gF, B))) return rc;
    if ((rc = cap_copy(c, c->capBT2[l], c->T2, (long long)B * H * 2 * m * C))) return rc;
    if (fuse_b) {
      if ((rc = layer_tail_back(c, l, B, dz, dh_next, c->grad + (l > 0 ? c->ob[l - 1] : c->oPb)))) return rc;
      if ((rc = cap_copy(c, c->capDH[l], dh_next, P * C))) return rc;
      std::swap(dh, dh_next);
      continue;
    }
    // dh_l = Ax1 . T2 + dz W_l^T
    GemmArgs e = ga();
    e.M = W; e.N = C; e.K = 2 * m; e.K2 = C;
    e.nb1 = B; e.nb2 = H;
    e.A = op(c->Ax1, 2 * m, 1);
    e.B = op(c->T2, C, 1, (long long)H * 2 * m * C, 2LL * m * C);
    e.A2 = op(dz, C, 1, (long long)H * W * C, (long long)W * C);
    e.B2 = op(c->Wl[l], 1, C);
    e.C = dh_next; e.c_bf16 = 1;
    e.sC1 = (long long)H * W * C; e.sC2 = (long long)W * C; e.rC = C; e.cC = 1;
    if ((rc = cgemm(c, e))) return rc;
    if (l == 0 && (rc = cap_copy(c, c->capDH[0], dh_next, P * C))) return rc;
    std::swap(dh, dh_next);
  }
  // lift
  if (C == 32 && c->cin >= 1 && c->cin <= 4 && ((uintptr_t)dh & 15) == 0) {
    const long long nchunk = (P + kWgradChunk - 1) / kWgradChunk;
    if ((size_t)(nchunk * c->cin * C) > c->part_n) return ffail(TTSH_ENOMEM, "fno partials buffer too small");
    const dim3 g((unsigned)nchunk), t(256);
    const bf16* xb = c->xb;
    switch (c->cin) {
      case 1: hipLaunchKernelGGL(k_lift_wgrad_part<1>, g, t, 0, c->s, xb, (const bf16*)dh, P, kWgradChunk, c->part); break;
      case 2: hipLaunchKernelGGL(k_lift_wgrad_part<2>, g, t, 0, c->s, xb, (const bf16*)dh, P, kWgradChunk, c->part); break;
      case 3: hipLaunchKernelGGL(k_lift_wgrad_part<3>, g, t, 0, c->s, xb, (const bf16*)dh, P, kWgradChunk, c->part); break;
      default: hipLaunchKernelGGL(k_lift_wgrad_part<4>, g, t, 0, c->s, xb, (const bf16*)dh, P, kWgradChunk, c->part); break;
    }
    FCHK(hipGetLastError());
    if ((rc = reduce_parts(c, c->part, nchunk, (long long)c->cin * C, c->grad + c->oPw))) return rc;
  } else if ((rc = wgrad(c, c->cin, C, P, c->xb, 1, c->cin, dh, C, 1, c->grad + c->oPw))) {
    return rc;
  }
  if (!fuse_b)  // else layer 0's backward tail summed dh already
    if ((rc = colsum(c, dh, P, C, c->grad + c->oPb))) return rc;
  return TTSH_OK;
}

int fno_adam_step(fno_ctx* c, float lr, float b1, float b2, float eps) {
  if (!c) return ffail(TTSH_EINVAL, "null context");
  if (!(lr >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return ffail(TTSH_EINVAL, "invalid Adam coefficients");
  c->adam_t += 1;
  const float c1 = 1.f - powf(b1, (float)c->adam_t), c2 = 1.f - powf(b2, (float)c->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(nb(c->nparam)), dim3(256), 0, c->s, c->theta, c->grad, c->m1, c->m2,
                     (long long)c->nparam, lr, b1, b2, eps, c1, c2);
  FCHK(hipGetLastError());
  return refresh_weights(c);
}

int fno_gather(fno_ctx* c, float* dst, int64_t dch, const float* src, int64_t sch, int nch, int64_t npix,
               const int64_t* idx, int n) {
  if (!c || !dst || !src || !idx) return ffail(TTSH_EINVAL, "null argument");
  if (n < 1 || n > c->maxB) return ffail(TTSH_EINVAL, "sample count out of range");
  if (nch < 1 || npix < 1 || dch < nch || sch < nch) return ffail(TTSH_EINVAL, "invalid sizes");
  for (int s = 0; s < n; ++s)
    if (idx[s] < 0) return ffail(TTSH_EINVAL, "negative sample index");
  static_assert(sizeof(long long) == sizeof(int64_t), "index width");
  FCHK(hipMemcpyAsync(c->gidx, idx, sizeof(int64_t) * n, hipMemcpyHostToDevice, c->s));
  const long long tot = (long long)n * npix * nch;
  hipLaunchKernelGGL(k_gather, dim3(nb(tot)), dim3(256), 0, c->s, dst, (long long)dch, src, (long long)sch, nch,
                     (long long)npix, c->gidx, tot);
  FCHK(hipGetLastError());
  FCHK(hipStreamSynchronize(c->s));  // idx is read from pageable host memory
  return TTSH_OK;
}

int fno_gather_d4(fno_ctx* c, float* dst, int64_t dch, const float* src, int64_t sch, int nch, int n_side,
                  const int64_t* idx, const int* sym, int n) {
  if (!c || !dst || !src || !idx || !sym) return ffail(TTSH_EINVAL, "null argument");
  if (n < 1 || n > c->maxB) return ffail(TTSH_EINVAL, "sample count out of range");
  if (nch < 1 || dch < nch || sch < nch || n_side < 2 || n_side % 2) return ffail(TTSH_EINVAL, "invalid sizes");
  for (int s = 0; s < n; ++s) {
    if (idx[s] < 0) return ffail(TTSH_EINVAL, "negative sample index");
    if (sym[s] < 0 || sym[s] > 7) return ffail(TTSH_EINVAL, "symmetry element must be in 0..7");
  }
  FCHK(hipMemcpyAsync(c->gidx, idx, sizeof(int64_t) * n, hipMemcpyHostToDevice, c->s));
  FCHK(hipMemcpyAsync(c->gsym, sym, sizeof(int) * n, hipMemcpyHostToDevice, c->s));
  const long long tot = (long long)n * n_side * n_side;
  hipLaunchKernelGGL(k_gather_d4, dim3(nb(tot)), dim3(256), 0, c->s, dst, (long long)dch, src, (long long)sch, nch,
                     n_side, c->gidx, c->gsym, tot);
  FCHK(hipGetLastError());
  FCHK(hipStreamSynchronize(c->s));  // idx and sym are read from pageable host memory
  return TTSH_OK;
}

int fno_perturb(fno_ctx* c, float* x, int64_t pix_stride, int nch, int64_t npix, float amp, uint64_t seed) {
  if (!c || !x) return ffail(TTSH_EINVAL, "null argument");
  if (nch < 1 || npix < 1 || pix_stride < nch) return ffail(TTSH_EINVAL, "invalid sizes");
  if (!(amp >= 0.f)) return ffail(TTSH_EINVAL, "amplitude must be >= 0");
  const long long tot = (long long)npix * nch;
  hipLaunchKernelGGL(k_perturb, dim3(nb(tot)), dim3(256), 0, c->s, x, (long long)pix_stride, nch, tot, amp,
                     (unsigned long long)seed);
  FCHK(hipGetLastError());
  return TTSH_OK;
}

int fno_sample_errors(const float* y, int64_t ys, const float* t, int64_t ts, int nch, int64_t npix, int B,
                      double* out) {
  if (!y || !t || !out) return ffail(TTSH_EINVAL, "null argument");
  if (B < 1 || nch < 1 || npix < 1 || ys < nch || ts < nch) return ffail(TTSH_EINVAL, "invalid sizes");
  double* d = nullptr;
  FCHK(hipMalloc((void**)&d, 2 * B * sizeof(double)));
  hipLaunchKernelGGL(k_err_sums, dim3(B), dim3(256), 0, 0, y, (long long)ys, t, (long long)ts, nch,
                     (long long)npix, d);
  std::vector<double> h(2 * B);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(h.data(), d, 2 * B * sizeof(double), hipMemcpyDeviceToHost);
  hipFree(d);
  if (e != hipSuccess) return ffail(TTSH_EHIP, std::string("error sums: ") + hipGetErrorString(e));
  for (int s = 0; s < B; ++s) out[s] = sqrt(h[2 * s]) / sqrt(h[2 * s + 1]);
  return TTSH_OK;
}

int fno_gemm_bf16(int batch, int M, int N, int K, float alpha, const uint16_t* A, int64_t sA, int64_t rA,
                  int64_t cA, const uint16_t* B, int64_t sB, int64_t rB, int64_t cB, float* C, int64_t sC,
                  int64_t rC, int64_t cC) {
  if (!A || !B || !C) return ffail(TTSH_EINVAL, "null pointer");
  if (batch < 1 || M < 1 || N < 1 || K < 1) return ffail(TTSH_EINVAL, "sizes must be >= 1");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return ffail(TTSH_EHIP, "no HIP device available");
  GemmArgs g = ga();
  g.M = M; g.N = N; g.K = K;
  g.nb1 = batch;
  g.alpha = alpha;
  g.A = op(A, rA, cA, sA, 0);
  g.B = op(B, rB, cB, sB, 0);
  g.C = C; g.c_bf16 = 0; g.sC1 = sC; g.rC = rC; g.cC = cC;
  // the path the network's GEMMs take for these strides
  g.staged = staged_form(g);
  FCHK(gemm(g, 0));
  FCHK(hipDeviceSynchronize());
  return TTSH_OK;
}

}  // extern "C"
