// Set-up and read-out kernels (host runtime translation unit only): state
// packing with projection, masks (tanh wall and Algorithm 2), state
// layout conversion, resampling between grid sizes, FP64 norms.
// None of these runs inside the time loop.
#pragma once

#include "common.hpp"
#include "fft.hpp"
#include "step.hpp"
#include "fft_full.hpp"

namespace ttsh {

// ---- simple element-wise helpers -------------------------------------------
__global__ void k_pack_xy(const double* __restrict__ v, C2<double>* __restrict__ z, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = mk(v[i], v[n + i]);
}
__global__ void k_unpack_xy(const C2<double>* __restrict__ z, double* __restrict__ v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    v[i] = z[i].x;
    v[n + i] = z[i].y;
  }
}
__global__ void k_unpack_xy_strided(const C2<double>* __restrict__ z, float* __restrict__ v, int n,
                                    long long stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    v[(long long)i * stride] = (float)z[i].x;
    v[(long long)i * stride + 1] = (float)z[i].y;
  }
}
__global__ void k_pack_xy_strided(const float* __restrict__ v, long long stride, C2<double>* __restrict__ z,
                                  int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = mk((double)v[(long long)i * stride], (double)v[(long long)i * stride + 1]);
}

__global__ void k_real_part(const C2<double>* __restrict__ z, double* __restrict__ v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = z[i].x;
}
__global__ void k_scale_c(C2<double>* __restrict__ z, double s, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = cscale(z[i], s);
}
template <class D, class S>
__global__ void k_convert(const S* __restrict__ in, D* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (D)in[i];
}
__global__ void k_binary_to_c(const uint8_t* __restrict__ b, C2<double>* __restrict__ z, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = mk(b[i] ? 1.0 : 0.0, 0.0);
}

// integer mode number of FFT index i on an N grid
__device__ __forceinline__ int mode_of(int i, int N) { return i < N / 2 ? i : i - N; }

// Algorithm 2 cutoff: zero m^2 > (N/8)^2, scale the survivors by s
__global__ void k_lowpass(C2<double>* __restrict__ z, int N, int cut2, double s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * N) return;
  const int my = mode_of(i / N, N), mx = mode_of(i % N, N);
  z[i] = (mx * mx + my * my > cut2) ? mk(0.0, 0.0) : cscale(z[i], s);
}

// K = (Re z)^2 into the run precision
template <class T>
__global__ void k_square_real(const C2<double>* __restrict__ z, T* __restrict__ K, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) K[i] = (T)(z[i].x * z[i].x);
}

// tanh wall, product over circles; evaluated in FP64
struct Circles {
  int n;
  double cx[8], cy[8], R[8];
};
template <class T>
__global__ void k_mask_tanh(T* __restrict__ K, int N, double dx, Circles c, double xi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * N) return;
  const double x = ((i % N) - N / 2) * dx, y = ((i / N) - N / 2) * dx;
  double k = 1.0;
  for (int q = 0; q < c.n; ++q) {
    const double r = sqrt((x - c.cx[q]) * (x - c.cx[q]) + (y - c.cy[q]) * (y - c.cy[q]));
    k *= 0.5 * (1.0 + tanh((r - c.R[q]) / xi));
  }
  K[i] = (T)k;
}

// ---- counter-based noise (Philox-4x32-10) -------------------------------------
// Philox-4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): each round takes the 64-bit products of
// counter words 0 and 2 with two fixed multipliers and forms
// (hi(p1) ^ c1 ^ k0, lo(p1), hi(p0) ^ c3 ^ k1, lo(p0)); the key is advanced by
// two Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Continuation noise of one destination instance into Z = n_x + i n_y, [N][N]:
// node (i, j) takes counter (i N + j, inst, 0, 0); word c gives component c as
// amp (2 u - 1), u = (word >> 8) 2^-24, in FP64.
__global__ void k_philox_noise(C2<double>* __restrict__ Z, int N, uint32_t inst, uint32_t k0, uint32_t k1,
                               double amp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * N) return;
  uint32_t c[4] = {(uint32_t)i, inst, 0u, 0u};
  philox4x32_10(c, k0, k1);
  const double ux = (double)(c[0] >> 8) * 0x1p-24;
  const double uy = (double)(c[1] >> 8) * 0x1p-24;
  Z[i] = mk(amp * (2.0 * ux - 1.0), amp * (2.0 * uy - 1.0));
}

// ---- state packing -----------------------------------------------------------
// From Z = unnormalised 2D FFT of (v_x + i v_y): separate the two real fields,
// scale to the unitary DFT, cut at m^2 > M^2, project (k != 0), optionally add
// a compact FP64 spectrum `add` (same layout as the state), store the state.
// Z may be null (no field: the state becomes `add`, or zero).
// Thread per stored (component-pair) position.
template <class S>
__global__ void k_pack_state(const C2<double>* __restrict__ Z, const C2<double>* __restrict__ add,
                             C2<S>* __restrict__ st, int N) {
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MP * SP) return;
  const int mx = i / SP, pos = i % SP;
  C2<double> ox = mk(0.0, 0.0), oy = mk(0.0, 0.0);
  if (pos <= 2 * M) {
    const int my = pos <= M ? pos : pos - (2 * M + 1);
    if (mx * mx + my * my <= M * M && Z) {
      const C2<double> zp = Z[(size_t)((my + N) % N) * N + mx];
      const C2<double> zm = Z[(size_t)((N - my) % N) * N + (N - mx) % N];
      const double s = 1.0 / N;
      ox = cscale(mk(zp.x + zm.x, zp.y - zm.y), 0.5 * s);   // (Z(k) + Z(-k)^*)/2
      oy = cscale(mk(zp.y + zm.y, -(zp.x - zm.x)), 0.5 * s);  // -i (Z(k) - Z(-k)^*)/2
      const int m2 = mx * mx + my * my;
      if (m2 > 0) {
        const double inv = 1.0 / m2;
        const C2<double> d = cscale(mk(mx * ox.x + my * oy.x, mx * ox.y + my * oy.y), inv);
        ox = ox - cscale(d, (double)mx);
        oy = oy - cscale(d, (double)my);
      }
    }
    if (mx * mx + my * my <= M * M && add) {
      ox = ox + add[(0 * MP + mx) * SP + pos];
      oy = oy + add[(1 * MP + mx) * SP + pos];
    }
  }
  st[(0 * MP + mx) * SP + pos] = cvt<S>(ox);
  st[(1 * MP + mx) * SP + pos] = cvt<S>(oy);
}

// Full spectrum of (v_x + i v_y)/N (or omega/N) from the state, ready for the
// unnormalised inverse transform.  what = 0: velocity, 1: vorticity.
template <class S>
__global__ void k_state_to_full(const C2<S>* __restrict__ st, C2<double>* __restrict__ Z, int N,
                                double dk, int what) {
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * N) return;
  int my = mode_of(i / N, N), mx = mode_of(i % N, N);
  C2<double> out = mk(0.0, 0.0);
  if (mx * mx + my * my <= M * M) {
    const bool neg = mx < 0;
    const int ax = neg ? -mx : mx, ay = neg ? -my : my;
    const int pos = ay >= 0 ? ay : ay + 2 * M + 1;
    C2<double> a = cvt<double>(st[(0 * MP + ax) * SP + pos]);
    C2<double> b = cvt<double>(st[(1 * MP + ax) * SP + pos]);
    if (neg) {
      a = conj(a);
      b = conj(b);
    }
    if (what == 0) {
      out = mk(a.x - b.y, a.y + b.x);  // a + i b
    } else {
      const C2<double> c = cscale(b, (double)mx) - cscale(a, (double)my);
      out = mk(-c.y * dk, c.x * dk);    // i dk (m_x v_y - m_y v_x)
    }
    out = cscale(out, 1.0 / N);
  }
  Z[i] = out;
}

template <class S>
__global__ void k_convert_c(const C2<double>* __restrict__ in, C2<S>* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cvt<S>(in[i]);
}

// Batched full spectra Z of (v_x + i v_y) (unnormalised, [batch][N][N]) ->
// Z' of the projected field: components separated, cut at m^2 > (N/4)^2,
// Leray-projected (m != 0), recombined and scaled by 1/N^2 so that the
// unnormalised inverse transform returns the field.
__global__ void k_project_full(const C2<double>* __restrict__ Z, C2<double>* __restrict__ out, int N, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = i / (N * N), r = i % (N * N);
  const int my = mode_of(r / N, N), mx = mode_of(r % N, N);
  const int M = N / 4, m2 = mx * mx + my * my;
  C2<double> o = mk(0.0, 0.0);
  if (m2 <= M * M) {
    const C2<double>* Zb = Z + (size_t)b * N * N;
    const C2<double> zp = Zb[r];
    const C2<double> zm = Zb[(size_t)((N - my) % N) * N + (N - mx) % N];
    C2<double> ox = cscale(mk(zp.x + zm.x, zp.y - zm.y), 0.5);
    C2<double> oy = cscale(mk(zp.y + zm.y, -(zp.x - zm.x)), 0.5);
    if (m2 > 0) {
      const C2<double> d = cscale(mk(mx * ox.x + my * oy.x, mx * ox.y + my * oy.y), 1.0 / m2);
      ox = ox - cscale(d, (double)mx);
      oy = oy - cscale(d, (double)my);
    }
    o = cscale(mk(ox.x - oy.y, ox.y + oy.x), 1.0 / ((double)N * N));
  }
  out[i] = o;
}

// Per field of a batch of projected spectra (as written by k_project_full):
// out[2b] = sum_x |v|^2, out[2b+1] = sum_x |w|^2 with w the vorticity in
// integer-mode units (i (m_x v_y - m_y v_x) per mode).  Block per field.
__global__ void __launch_bounds__(256) k_full_norms(const C2<double>* __restrict__ Zs, int N,
                                                    double* __restrict__ out) {
  const C2<double>* Z = Zs + (size_t)blockIdx.x * N * N;
  const double s = (double)N * N;  // undo the 1/N^2 of the stored spectrum
  double e = 0.0, w = 0.0;
  for (int r = threadIdx.x; r < N * N; r += blockDim.x) {
    const int my = mode_of(r / N, N), mx = mode_of(r % N, N);
    const C2<double> zp = cscale(Z[r], s);
    const C2<double> zm = cscale(Z[(size_t)((N - my) % N) * N + (N - mx) % N], s);
    const C2<double> ox = cscale(mk(zp.x + zm.x, zp.y - zm.y), 0.5);
    const C2<double> oy = cscale(mk(zp.y + zm.y, -(zp.x - zm.x)), 0.5);
    e += zp.x * zp.x + zp.y * zp.y;
    const C2<double> c = cscale(oy, (double)mx) - cscale(ox, (double)my);
    w += c.x * c.x + c.y * c.y;
  }
  e = wave_sum_from(e, 1);
  w = wave_sum_from(w, 1);
  __shared__ double red[4][2];
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = e;
    red[threadIdx.x >> 6][1] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double inv = 1.0 / ((double)N * N);  // Parseval for the unnormalised transform
    out[2 * blockIdx.x] = (red[0][0] + red[1][0] + red[2][0] + red[3][0]) * inv;
    out[2 * blockIdx.x + 1] = (red[0][1] + red[1][1] + red[2][1] + red[3][1]) * inv;
  }
}

// internal state [2][M+1][2M+2]  <->  interface layout [2][2M+1][M+1] (FP64)
template <class S>
__global__ void k_state_to_abi(const C2<S>* __restrict__ st, C2<double>* __restrict__ o, int N) {
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * (2 * M + 1) * MP) return;
  const int c = i / ((2 * M + 1) * MP), r = (i / MP) % (2 * M + 1), mx = i % MP;
  const int my = r - M;
  const int pos = my >= 0 ? my : my + 2 * M + 1;
  o[i] = cvt<double>(st[(c * MP + mx) * SP + pos]);
}
template <class S>
__global__ void k_abi_to_state(const C2<double>* __restrict__ in, C2<S>* __restrict__ st, int N) {
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * MP * SP) return;
  const int c = i / (MP * SP), mx = (i / SP) % MP, pos = i % SP;
  C2<double> v = mk(0.0, 0.0);
  if (pos <= 2 * M) {
    const int my = pos <= M ? pos : pos - (2 * M + 1);
    if (mx * mx + my * my <= M * M) v = in[((size_t)c * (2 * M + 1) + (my + M)) * MP + mx];
  }
  st[i] = cvt<S>(v);
}

// dst (compact FP64, dst layout) <- src state scaled by Nd/Ns, by integer mode
// index; modes beyond either grid's radius are zero.
template <class S>
__global__ void k_resample(const C2<S>* __restrict__ src, int Ns, C2<double>* __restrict__ dst,
                           int Nd) {
  const int Md = Nd / 4, MPd = Md + 1, SPd = 2 * Md + 2;
  const int Ms = Ns / 4, MPs = Ms + 1, SPs = 2 * Ms + 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * MPd * SPd) return;
  const int c = i / (MPd * SPd), mx = (i / SPd) % MPd, pos = i % SPd;
  C2<double> v = mk(0.0, 0.0);
  if (pos <= 2 * Md) {
    const int my = pos <= Md ? pos : pos - (2 * Md + 1);
    const int m2 = mx * mx + my * my;
    if (m2 <= Md * Md && m2 <= Ms * Ms) {
      const int ps = my >= 0 ? my : my + 2 * Ms + 1;
      v = cscale(cvt<double>(src[((size_t)c * MPs + mx) * SPs + ps]), (double)Nd / (double)Ns);
    }
  }
  dst[i] = v;
}

// ---- order parameters on the real-space fields ------------------------------
// Vortex order parameter about (cx, cy) of the velocity in Z (real part v_x,
// imaginary part v_y, node (i, j) at x = (j - N/2) dx, y = (i - N/2) dx):
// sums of |e_theta . v| and |v| in FP64 in a fixed order.
//
// The reductions over the N^2 nodes here run in order_blocks(N) workgroups of
// 1024 threads, each writing one partial result; a one-thread kernel combines
// the partials in workgroup order, so that results do not vary between runs.
inline int order_blocks(int N) {
  const int b = N * N / 4096;
  return b < 1 ? 1 : (b > 256 ? 256 : b);  // at most kOrderMaxBlocks
}
__global__ void __launch_bounds__(1024) k_order_psi(const C2<double>* __restrict__ Z, int N, double dx, double cx,
                                                    double cy, double* __restrict__ part) {
  double num = 0.0, den = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N * N; i += gridDim.x * blockDim.x) {
    const double x = ((i % N) - N / 2) * dx - cx, y = ((i / N) - N / 2) * dx - cy;
    const double r = sqrt(x * x + y * y);
    const C2<double> v = Z[i];
    if (r > 0.0) num += fabs((-y * v.x + x * v.y) / r);
    den += sqrt(v.x * v.x + v.y * v.y);
  }
  num = wave_sum_from(num, 1);
  den = wave_sum_from(den, 1);
  __shared__ double red[16][2];
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = num;
    red[threadIdx.x >> 6][1] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a += red[w][0];
      b += red[w][1];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}
// The combining kernels run one workgroup of 256 threads: the partials
// (at most 256 per quantity) are staged in LDS in parallel, then one thread
// takes them in workgroup order.
constexpr int kOrderMaxBlocks = 256;
__global__ void __launch_bounds__(256) k_order_psi_final(const double* __restrict__ part, int nb,
                                                         double* __restrict__ out) {
  __shared__ double ps[2 * kOrderMaxBlocks];
  for (int q = threadIdx.x; q < 2 * nb; q += blockDim.x) ps[q] = part[q];
  __syncthreads();
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int q = 0; q < nb; ++q) {
    a += ps[2 * q];
    b += ps[2 * q + 1];
  }
  const double two_pi = 2.0 / M_PI;
  out[0] = (a / b - two_pi) / (1.0 - two_pi);
}

// Topological defects of the direction field of v = (Re Z, Im Z).  A node is
// inside when K < kmax and has a direction when |v|^2 > vmin^2.  Per grid cell
// (corners (i, j), (i, j+1), (i+1, j+1), (i+1, j), periodic, counter-
// clockwise) with all four corners inside with a direction, and per inside
// node without a direction whose eight neighbours are inside with one (a
// defect sitting on the node), the winding number of v around the cell or the
// ring, counted in quarter turns: each vector's quadrant comes from exact sign
// tests, a step to the next or previous quadrant is +-1, to the opposite one
// +-2 with the sign of the cross product of the two vectors; the sum around
// the loop is 4n.  out[0] = sum of n > 0 (vortex centres), out[1] = sum of |n|
// over n < 0 (saddles).  Integer sums (independent of order), one partial per
// workgroup combined by k_vortex_final.
__device__ __forceinline__ int quadrant(double x, double y) {
  if (x > 0.0 && y >= 0.0) return 0;
  if (x <= 0.0 && y > 0.0) return 1;
  if (x < 0.0 && y <= 0.0) return 2;
  return 3;
}
template <int P>
__device__ __forceinline__ int winding_quarters(const C2<double> (&w)[P]) {
  int turns = 0;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const C2<double> a = w[q], b = w[(q + 1) % P];
    const int d = (quadrant(b.x, b.y) - quadrant(a.x, a.y) + 4) & 3;
    if (d == 1) turns += 1;
    else if (d == 3) turns -= 1;
    else if (d == 2) turns += (a.x * b.y - a.y * b.x) >= 0.0 ? 2 : -2;
  }
  return turns;
}
template <class T>
__global__ void __launch_bounds__(1024) k_vortex_count(const C2<double>* __restrict__ Z, const T* __restrict__ K,
                                                       int N, double kmax, double vmin, int* __restrict__ part) {
  int pos = 0, neg = 0;
  const double v2 = vmin * vmin;
  auto inside = [&](int id) { return (double)K[id] < kmax; };
  auto fast = [&](const C2<double>& z) { return z.x * z.x + z.y * z.y > v2 && (z.x != 0.0 || z.y != 0.0); };
  const int m = N - 1;  // N is a power of two: (i + d) & m wraps
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N * N; c += gridDim.x * blockDim.x) {
    const int i = c / N, j = c % N;
    {  // the cell with lower-left corner (i, j)
      const int id[4] = {i * N + j, i * N + ((j + 1) & m), ((i + 1) & m) * N + ((j + 1) & m), ((i + 1) & m) * N + j};
      C2<double> w[4];
      bool ok = true;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        w[q] = Z[id[q]];
        ok = ok && inside(id[q]) && fast(w[q]);
      }
      if (ok) {
        const int n = winding_quarters(w) / 4;
        if (n > 0) pos += n;
        if (n < 0) neg -= n;
      }
    }
    if (inside(c) && !fast(Z[c])) {  // a defect on node (i, j): the ring of its neighbours
      const int di[8] = {-1, -1, -1, 0, 1, 1, 1, 0}, dj[8] = {-1, 0, 1, 1, 1, 0, -1, -1};
      C2<double> w[8];
      bool ok = true;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int id = ((i + di[q]) & m) * N + ((j + dj[q]) & m);
        w[q] = Z[id];
        ok = ok && inside(id) && fast(w[q]);
      }
      if (ok) {
        const int n = winding_quarters(w) / 4;
        if (n > 0) pos += n;
        if (n < 0) neg -= n;
      }
    }
  }
  __shared__ int red[16][2];
  for (int o = 32; o > 0; o >>= 1) {
    pos += __shfl_xor(pos, o);
    neg += __shfl_xor(neg, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = pos;
    red[threadIdx.x >> 6][1] = neg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, b = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a += red[w][0];
      b += red[w][1];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}
__global__ void __launch_bounds__(256) k_vortex_final(const int* __restrict__ part, int nb, int* __restrict__ out) {
  __shared__ int ps[2 * kOrderMaxBlocks];
  for (int q = threadIdx.x; q < 2 * nb; q += blockDim.x) ps[q] = part[q];
  __syncthreads();
  if (threadIdx.x != 0) return;
  int a = 0, b = 0;
  for (int q = 0; q < nb; ++q) {
    a += ps[2 * q];
    b += ps[2 * q + 1];
  }
  out[0] = a;
  out[1] = b;
}

// Two-chamber order parameter from the vorticity in the real part of Z: the
// nodes of largest |omega| in the left and right regions (ties to the lower
// index), |w_l + w_r| / (|w_l| + |w_r|).  Regions: with D > 0 the nodes within
// D/2 of (cx - D/2, cy) left of x = cx and within D/2 of (cx + D/2, cy) at or
// right of it; with D <= 0 the two half-planes.  An empty region gives NaN.
// The disk test rounds every product and sum separately (no fused
// multiply-add), so that a node on a disk's rim falls on the same side as in
// a plain evaluation of the same expression.
__global__ void __launch_bounds__(1024) k_order_psi2(const C2<double>* __restrict__ Z, int N, double dx, double cx,
                                                     double cy, double D, double* __restrict__ part) {
  const double r2 = __dmul_rn(0.5 * D, 0.5 * D);
  const double cl = __dsub_rn(cx, 0.5 * D), cr = __dadd_rn(cx, 0.5 * D);
  double best[2] = {-1.0, -1.0};
  int at[2] = {0, 0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N * N; i += gridDim.x * blockDim.x) {
    const double x = __dmul_rn((double)((i % N) - N / 2), dx);
    const int side = x < cx ? 0 : 1;
    if (D > 0.0) {
      const double y = __dmul_rn((double)((i / N) - N / 2), dx);
      const double ex = __dsub_rn(x, side ? cr : cl), ey = __dsub_rn(y, cy);
      if (__dadd_rn(__dmul_rn(ex, ex), __dmul_rn(ey, ey)) > r2) continue;
    }
    const double a = fabs(Z[i].x);
    if (a > best[side]) {  // i grows per thread: the first of equal values is kept
      best[side] = a;
      at[side] = i;
    }
  }
  __shared__ double bv[2][1024];
  __shared__ int bi[2][1024];
  for (int q = 0; q < 2; ++q) {
    bv[q][threadIdx.x] = best[q];
    bi[q][threadIdx.x] = at[q];
  }
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      for (int q = 0; q < 2; ++q) {
        const double v2 = bv[q][threadIdx.x + o];
        const int i2 = bi[q][threadIdx.x + o];
        if (v2 > bv[q][threadIdx.x] || (v2 == bv[q][threadIdx.x] && i2 < bi[q][threadIdx.x])) {
          bv[q][threadIdx.x] = v2;
          bi[q][threadIdx.x] = i2;
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {  // (best |w|, its node) per side; node indices < 2^53 are exact
    part[4 * blockIdx.x] = bv[0][0];
    part[4 * blockIdx.x + 1] = (double)bi[0][0];
    part[4 * blockIdx.x + 2] = bv[1][0];
    part[4 * blockIdx.x + 3] = (double)bi[1][0];
  }
}
// larger |w| wins, equal values go to the lower node: the same choice in any
// order, so the partials are combined by a tree in LDS
__global__ void __launch_bounds__(256) k_order_psi2_final(const C2<double>* __restrict__ Z,
                                                          const double* __restrict__ part, int nb,
                                                          double* __restrict__ out) {
  __shared__ double bv[2][kOrderMaxBlocks];
  __shared__ long long bi[2][kOrderMaxBlocks];
  const int t = threadIdx.x;
  for (int sd = 0; sd < 2; ++sd) {
    bv[sd][t] = t < nb ? part[4 * t + 2 * sd] : -1.0;
    bi[sd][t] = t < nb ? (long long)part[4 * t + 2 * sd + 1] : 0;
  }
  __syncthreads();
  for (int o = kOrderMaxBlocks / 2; o > 0; o >>= 1) {
    if (t < o)
      for (int sd = 0; sd < 2; ++sd) {
        const double v = bv[sd][t + o];
        const long long i = bi[sd][t + o];
        if (v > bv[sd][t] || (v == bv[sd][t] && v >= 0.0 && i < bi[sd][t])) {
          bv[sd][t] = v;
          bi[sd][t] = i;
        }
      }
    __syncthreads();
  }
  if (t == 0) {
    const double wl = Z[bi[0][0]].x, wr = Z[bi[1][0]].x;
    out[1] = (bv[0][0] < 0.0 || bv[1][0] < 0.0) ? __builtin_nan("") : fabs(wl + wr) / (fabs(wl) + fabs(wr));
  }
}

// ---- Lyapunov re-orthonormalisation -------------------------------------------
// Benettin's method (circle section: exponents of the transition): the
// deviations d_v = (X_v - X_0)/eps of p perturbed states from the base state
// are orthonormalised in order by modified Gram-Schmidt under the real-space
// inner product (Parseval: weight 1 on the m_x = 0 column, 2 on m_x > 0, the
// padding position excluded); logs[v] = log |d_v - projections| (the diagonal
// of R in D = Q R) and X_v = X_0 + eps q_v, rounded to the stored precision.
constexpr int kMaxLyap = 16;  // perturbed copies per call

__device__ __forceinline__ double block_sum_1024(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    red[16] = t;
  }
  __syncthreads();
  const double r = red[16];
  __syncthreads();  // red is reused by the next sum
  return r;
}

// The passes run over many workgroups of 1024 threads (thread g owns entry g
// of every vector, so updates need no synchronisation); each pass ends with a
// per-workgroup partial of the next inner product, and the next pass's
// workgroups each add all the partials in workgroup order, so every
// workgroup uses the same coefficient and results do not vary between runs.
// Launches per perturbed state v: one k_lyap_init, v times k_lyap_axpy, one
// k_lyap_scale.
__device__ __forceinline__ double lyap_weight(int i, int MPSP, int SP, int M, bool& pad) {
  const int r = i % MPSP;
  pad = r % SP > 2 * M;
  return r / SP == 0 ? 1.0 : 2.0;
}
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int nb) {
  double t = 0.0;
  for (int q = 0; q < nb; ++q) t += part[q];
  return t;
}

// q_v = (X_v - X_0)/eps; partial of <qd, q_v> (qd = null: of <q_v, q_v>)
template <class S>
__global__ void __launch_bounds__(1024) k_lyap_init(const C2<S>* __restrict__ base, const C2<S>* __restrict__ X,
                                                    int N, double eps, C2<double>* __restrict__ qv,
                                                    const C2<double>* __restrict__ qd, double* __restrict__ part) {
  __shared__ double red[17];
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2, n = 2 * MP * SP;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    bool pad;
    const double w = lyap_weight(i, MP * SP, SP, M, pad);
    const C2<double> x = cvt<double>(X[i]), b = cvt<double>(base[i]);
    const C2<double> d = pad ? mk(0.0, 0.0) : mk((x.x - b.x) / eps, (x.y - b.y) / eps);
    qv[i] = d;
    const C2<double> o = qd ? qd[i] : d;
    acc = w * (o.x * d.x + o.y * d.y);
  }
  const double t = block_sum_1024(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// q_v -= r q_u with r = sum of part_in; partial of <qd, q_v> (qd = null: <q_v, q_v>)
__global__ void __launch_bounds__(1024) k_lyap_axpy(C2<double>* __restrict__ qv, const C2<double>* __restrict__ qu,
                                                    const double* __restrict__ part_in, int nb, int N,
                                                    const C2<double>* __restrict__ qd, double* __restrict__ part) {
  __shared__ double red[17];
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2, n = 2 * MP * SP;
  const double r = sum_parts(part_in, nb);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    bool pad;
    const double w = lyap_weight(i, MP * SP, SP, M, pad);
    const C2<double> a = qv[i], u = qu[i];
    const C2<double> d = mk(a.x - r * u.x, a.y - r * u.y);
    qv[i] = d;
    const C2<double> o = qd ? qd[i] : d;
    acc = w * (o.x * d.x + o.y * d.y);
  }
  const double t = block_sum_1024(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// rr = sqrt(sum of part_in); q_v /= rr; X_v = X_0 + eps q_v; logv = log rr
template <class S>
__global__ void __launch_bounds__(1024) k_lyap_scale(const C2<S>* __restrict__ base, C2<S>* __restrict__ X,
                                                     C2<double>* __restrict__ qv, const double* __restrict__ part_in,
                                                     int nb, int N, double eps, double* __restrict__ logv) {
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2, n = 2 * MP * SP;
  const double rr = sqrt(sum_parts(part_in, nb));
  const double inv = 1.0 / rr;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    bool pad;
    (void)lyap_weight(i, MP * SP, SP, M, pad);
    const C2<double> q = mk(qv[i].x * inv, qv[i].y * inv);
    qv[i] = q;
    if (!pad) {
      const C2<double> b = cvt<double>(base[i]);
      X[i] = cvt<S>(mk(b.x + eps * q.x, b.y + eps * q.y));
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *logv = log(rr);
}

// ---- temporal power spectral density of the vorticity ----------------------------
// Circle section, eq. (PSD): S(f) = (1/N^2) sum_x |sum_t w(x, t) e^{-2 pi i f t}|^2.
// By Parseval over x (unitary DFT) the sum over nodes is the sum over all modes
// k of |W(k, f)|^2 with W(k, f) = sum_t w_hat(k, t) e^{-2 pi i f t}, so the
// accumulators live on the compact spectrum.  Only m_x >= 0 is stored; the
// mirror mode -k of a column m_x > 0 has W(-k, f) = conj(W(k, -f)), so each
// stored mode keeps two accumulators, at +f and at -f (the second is not used
// on the m_x = 0 column, which holds both signs of m_y itself).
// acc: [nf][2][M+1][2M+2] complex FP64, index 0 of the second axis for +f.
constexpr int kMaxPsdFreqs = 4096;

template <class S>
__global__ void __launch_bounds__(256) k_psd_acc(const C2<S>* __restrict__ st, int N, double dk,
                                                 const double* __restrict__ freqs, int nf, double t,
                                                 C2<double>* __restrict__ acc) {
  __shared__ double pc[256], ps[256];
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2, nm = MP * SP;
  const int f0 = blockIdx.y * 256;
  const int nfb = min(256, nf - f0);
  if ((int)threadIdx.x < nfb) {
    double sn, cs;
    sincospi(2.0 * freqs[f0 + threadIdx.x] * t, &sn, &cs);  // e^{-2 pi i f t} = cs - i sn
    pc[threadIdx.x] = cs;
    ps[threadIdx.x] = sn;
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nm) return;
  const int mx = i / SP, pos = i % SP;
  if (pos > 2 * M) return;
  const int my = pos <= M ? pos : pos - (2 * M + 1);
  const C2<double> vx = cvt<double>(st[i]), vy = cvt<double>(st[nm + i]);
  const double kx = dk * mx, ky = dk * my;
  // w_hat = i (k_x v_y - k_y v_x)
  const double dxr = kx * vy.x - ky * vx.x, dxi = kx * vy.y - ky * vx.y;
  const double wr = -dxi, wi = dxr;
  for (int q = 0; q < nfb; ++q) {
    const double c = pc[q], sn = ps[q];
    C2<double>* a = acc + ((size_t)(f0 + q) * 2) * nm + i;
    // w_hat (c - i sn) at +f, w_hat (c + i sn) at -f
    const C2<double> p0 = a[0], p1 = a[nm];
    a[0] = mk(p0.x + wr * c + wi * sn, p0.y + wi * c - wr * sn);
    a[nm] = mk(p1.x + wr * c - wi * sn, p1.y + wi * c + wr * sn);
  }
}

__global__ void __launch_bounds__(1024) k_psd_finish(const C2<double>* __restrict__ acc, int N,
                                                     double* __restrict__ S) {
  __shared__ double red[17];
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2, nm = MP * SP;
  const C2<double>* a = acc + (size_t)blockIdx.x * 2 * nm;
  double part = 0.0;
  for (int i = threadIdx.x; i < nm; i += blockDim.x) {
    const int mx = i / SP, pos = i % SP;
    if (pos > 2 * M) continue;
    part += a[i].x * a[i].x + a[i].y * a[i].y;
    if (mx > 0) part += a[nm + i].x * a[nm + i].x + a[nm + i].y * a[nm + i].y;
  }
  const double tot = block_sum_1024(part, red);
  if (threadIdx.x == 0) S[blockIdx.x] = tot / ((double)N * (double)N);
}

// ---- FP64 norms on the compact state -----------------------------------------
// Over kNormBlocks workgroups of 256 threads, each writing one partial
// [5] (sum of |v|^2 with the Parseval weights, max |k . v_hat|, non-finite
// flag, and, from workgroup 0, the k = 0 entries); k_norms_final combines the
// partials in workgroup order, so results do not vary between runs:
// out[0] = sum_x |v|^2 (Parseval, unitary), out[1..2] = <v_x>, <v_y>,
// out[3] = max |k . v_hat|, out[4] = 1 if any entry is non-finite.
constexpr int kNormBlocks = 64;
template <class S>
__global__ void __launch_bounds__(256) k_norms(const C2<S>* __restrict__ st, int N, double dk,
                                               double* __restrict__ part) {
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2;
  double e = 0.0, dv = 0.0, bad = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MP * SP; i += gridDim.x * blockDim.x) {
    const int mx = i / SP, pos = i % SP;
    if (pos > 2 * M) continue;
    const int my = pos <= M ? pos : pos - (2 * M + 1);
    const C2<double> a = cvt<double>(st[i]);
    const C2<double> b = cvt<double>(st[MP * SP + i]);
    const double w = mx == 0 ? 1.0 : 2.0;
    const double s = a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y;
    if (!isfinite(s)) bad = 1.0;
    e += w * s;
    const C2<double> d = mk(mx * a.x + my * b.x, mx * a.y + my * b.y);
    dv = fmax(dv, dk * sqrt(d.x * d.x + d.y * d.y));
  }
  __shared__ double red[4][3];
  for (int o = 1; o < 64; o <<= 1) {
    e += __shfl_xor(e, o, 64);
    dv = fmax(dv, __shfl_xor(dv, o, 64));
    bad = fmax(bad, __shfl_xor(bad, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = e;
    red[threadIdx.x >> 6][1] = dv;
    red[threadIdx.x >> 6][2] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double E0 = 0.0, D0 = 0.0, B0 = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      E0 += red[w][0];
      D0 = fmax(D0, red[w][1]);
      B0 = fmax(B0, red[w][2]);
    }
    double* o = part + 5 * blockIdx.x;
    o[0] = E0;
    o[1] = D0;
    o[2] = B0;
    if (blockIdx.x == 0) {
      o[3] = cvt<double>(st[0]).x / N;
      o[4] = cvt<double>(st[MP * SP]).x / N;
    }
  }
}

__global__ void k_norms_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double E0 = 0.0, D0 = 0.0, B0 = 0.0;
  for (int b = 0; b < nb; ++b) {
    E0 += part[5 * b];
    D0 = fmax(D0, part[5 * b + 1]);
    B0 = fmax(B0, part[5 * b + 2]);
  }
  out[0] = E0;
  out[1] = part[3];
  out[2] = part[4];
  out[3] = D0;
  out[4] = B0;
}

// ---- non-finite guard over every instance of a size class --------------------
// flags[i] = 1 if instance i of the class holds a NaN or Inf among its stored
// modes (workgroup (x, i) scans part of instance i; every writer stores the
// same value, so no atomics are needed).  The flags are cleared by k_fill_int.
template <class S>
__global__ void __launch_bounds__(256) k_guard(const C2<S>* __restrict__ st, int N, int* __restrict__ flags) {
  const int M = N / 4, MP = M + 1, SP = 2 * M + 2;
  const size_t per = (size_t)2 * MP * SP;
  const C2<S>* s = st + (size_t)blockIdx.y * per;
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (size_t)gridDim.x * blockDim.x) {
    const C2<S> v = s[i];
    bad |= !isfinite((double)v.x) || !isfinite((double)v.y);
  }
  if (bad) flags[blockIdx.y] = 1;
}

__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace ttsh
