// The two fused kernels of one time step of the damped TTSH equation in its
// spectral-velocity (Leray) form.
//
// State of an instance on an N x N grid (M = N/4 the 1/2-rule radius):
//   st  [2][M+1][2M+2]   unitary spectrum v_hat, column m_x = 0..M, position
//                        p = m_y (m_y >= 0) or m_y + 2M + 1 (m_y < 0); FP32 or
//                        FP64.  Modes with m_x^2 + m_y^2 > M^2 are kept at 0.
//   X   [3][MP4/4][N][4] v_x, v_y, omega transformed back along y only
//                        ("mixed domain"), scaled so that the row transform
//                        alone yields the real field; columns m_x = 0..M are
//                        interleaved by groups of four (MP4 = M+1 rounded up to
//                        a multiple of 4): entry (m_x, y) sits at
//                        (m_x/4) 4N + 4y + m_x%4.  The column pass reads and
//                        writes whole 4-column slabs; the row pass reads runs
//                        of (rows per workgroup) x 32 bytes.
// Per step:
//   row pass    X -> inverse row C2R (two real rows per complex transform) ->
//               real-space forcing  N = -(beta|v|^2 + gamma_v K) v - lambda0
//               omega v_perp  (and G = -gamma_w K omega) -> forward row
//               transform of N_x + i N_y, values at m_x and N - m_x for
//               m_x <= M -> Y [2 or 3][MP4/4][N][4];  also the row sums of
//               -(beta|v|^2 + gamma_v K) v, which feed the k = 0 rule.
//   column pass Y -> forward column FFT -> k-space update (FP64) of v_hat ->
//               new st -> omega_hat -> inverse column FFT of v_x, v_y, omega ->
//               X for the next step.
//
// The k-space update is the velocity form of Algorithm 1 (Appendix C):
//   0 < m^2 <= M^2:  v' = P(k)[A v + B dt N_hat] + B dt (i k_y, -i k_x) G_hat / k^2
//   m = 0:           v'(0) = A(0) v(0) + B(0) dt DFT[-(beta|v|^2 + gamma_v K) v](0)
//                    (eq. (7): advection and the gamma_w term do not enter)
//   m^2 > M^2:       v' = 0                                  (1/2-rule cutoff)
//   m_x = 0 column:  v'(k) <- (v'(k) + v'(-k)^*)/2           (Hermitian correction)
// with (A, B) = (e^{L dt}, e^{L dt}) for the paper's integrating-factor Euler
// (computed per mode in FP64, see LinCoef),
// and L(k) = -alpha - Gamma0 k^2 - Gamma2 k^4.  The curl of this update is the
// paper's vorticity update: (v.grad)v = grad(|v|^2/2) + omega v_perp, and the
// projection removes the gradient.
#pragma once

#include "common.hpp"
#include "fft.hpp"

#ifndef TTSH_LDS_OFF
#define TTSH_LDS_OFF 8
#endif

namespace ttsh {

// Coefficients of the linear one-step map u' = A u + B dt f, evaluated per
// mode in FP64 from the integer m^2: L = -alpha - Gamma0 k^2 - Gamma2 k^4,
// k^2 = dk^2 m^2, z = L dt;  scheme 0: A = B = e^z (integrating-factor Euler),
// 1: A = e^z, B = (e^z - 1)/z, 2: A = B = 1/(1 - z).  Scheme 3, the
// second-order exponential Runge-Kutta method (Cox and Matthews 2002,
// ETD2RK), takes two column passes per step: stage 1 (column MODE 2) is the
// scheme-1 map into a second state a, stage 2 (MODE 3) is
// u' = a + phi_2(z) dt (f(a) - f(u)) with phi_2(z) = (e^z - 1 - z)/z^2.
struct LinCoef {
  double alpha, gamma0, gamma2, dt, dt_over_N;
  int scheme;
};

// phi_2(z) = (e^z - 1 - z)/z^2; its Taylor series sum_j z^j/(j+2)! below
// |z| = 1e-2, where the closed form loses digits to cancellation
__device__ __forceinline__ double phi2(double z) {
  if (fabs(z) < 1e-2) {
    double s = 1.0 / 40320.0;  // 1/8!
    s = fma(s, z, 1.0 / 5040.0);
    s = fma(s, z, 1.0 / 720.0);
    s = fma(s, z, 1.0 / 120.0);
    s = fma(s, z, 1.0 / 24.0);
    s = fma(s, z, 1.0 / 6.0);
    return fma(s, z, 0.5);
  }
  return (expm1(z) - z) / (z * z);
}

// phi_1, phi_2, phi_3 at z (phi_k(z) = sum_j z^j/(j+k)!): below |z| = 1/2 the
// series, 16 terms by Horner (the first term left out is below
// 2^-16/16! < 1e-18 of the sum); elsewhere phi_1 = expm1(z)/z and the
// recurrence phi_k = (phi_{k-1} - 1/(k-1)!)/z, whose subtractions then lose
// at most a few bits
struct InvFact {
  double v[19];
  constexpr InvFact() : v() {
    double f = 1.0;
    v[0] = 1.0;
    for (int i = 1; i < 19; ++i) {
      f *= i;
      v[i] = 1.0 / f;
    }
  }
};

__device__ __forceinline__ void phi123(double z, double& p1, double& p2, double& p3) {
  constexpr InvFact inv;
  if (fabs(z) < 0.5) {
    double a1 = inv.v[16], a2 = inv.v[17], a3 = inv.v[18];
#pragma unroll
    for (int j = 14; j >= 0; --j) {
      a1 = fma(a1, z, inv.v[j + 1]);
      a2 = fma(a2, z, inv.v[j + 2]);
      a3 = fma(a3, z, inv.v[j + 3]);
    }
    p1 = a1;
    p2 = a2;
    p3 = a3;
  } else {
    p1 = expm1(z) / z;
    p2 = (p1 - 1.0) / z;
    p3 = (p2 - 0.5) / z;
  }
}

// phi_1 alone, the same way
__device__ __forceinline__ double phi1(double z) {
  constexpr InvFact inv;
  if (fabs(z) < 0.5) {
    double a1 = inv.v[16];
#pragma unroll
    for (int j = 14; j >= 0; --j) a1 = fma(a1, z, inv.v[j + 1]);
    return a1;
  }
  return expm1(z) / z;
}

// Weights of an ETDRK4 stage (Cox and Matthews 2002) at z = L dt: the stage
// is  u_out = A base + dt (w_new F_new + w_u F(u) + w_acc (F(a) + F(b)))
//   MODE 4 (a):  A = e^{z/2}, w_new = phi_1(z/2)/2                     (base u)
//   MODE 5 (b):  A = e^{z/2}, w_new = phi_1(z/2)/2                     (base u)
//   MODE 6 (c):  A = e^{z/2}, w_new = phi_1(z/2), w_u = -phi_1(z/2)/2  (base a)
//   MODE 7 (u'): A = e^z, w_u = f1, w_acc = 2 f2, w_new = f3           (base u)
//                with f1 = phi_1 - 3 phi_2 + 4 phi_3, f2 = phi_2 - 2 phi_3,
//                f3 = -phi_2 + 4 phi_3 at z
template <int MODE>
__device__ __forceinline__ void etd4_weights(const LinCoef& c, double dk, int m2, double& A, double& wn, double& wu,
                                             double& wa) {
  const double k2 = dk * dk * (double)m2;
  const double z = (-c.alpha - c.gamma0 * k2 - c.gamma2 * k2 * k2) * c.dt;
  if constexpr (MODE == 7) {
    double p1, p2, p3;
    phi123(z, p1, p2, p3);
    A = exp(z);
    wu = p1 - 3.0 * p2 + 4.0 * p3;
    wa = 2.0 * (p2 - 2.0 * p3);
    wn = -p2 + 4.0 * p3;
  } else {
    A = exp(0.5 * z);
    const double q = 0.5 * phi1(0.5 * z);
    wn = MODE == 6 ? 2.0 * q : q;
    wu = MODE == 6 ? -q : 0.0;
    wa = 0.0;
  }
}

// (A, B) of column MODE 0 (one-stage schemes) or of an ETD2RK stage
// (MODE 2: A = e^z, B = phi_1(z); MODE 3: A = 1, B = phi_2(z))
template <int MODE>
__device__ __forceinline__ void linear_ab(const LinCoef& c, double dk, int m2, double& A, double& B) {
  const double k2 = dk * dk * (double)m2;
  const double z = (-c.alpha - c.gamma0 * k2 - c.gamma2 * k2 * k2) * c.dt;
  if constexpr (MODE == 3) {
    A = 1.0;
    B = phi2(z);
  } else if (MODE == 2 || c.scheme == 1) {
    A = exp(z);
    B = (z == 0.0) ? 1.0 : expm1(z) / z;
  } else if (c.scheme == 2) {
    A = B = 1.0 / (1.0 - z);
  } else {
    A = B = exp(z);
  }
}

template <class T>
struct alignas(4 * sizeof(T)) CPair {
  C2<T> a, b;
};

template <class T>
struct RowCoef {
  T beta, gamma_v, lambda0, gamma_w;
};

template <int N, int SCH = kSchedDefault>
struct Geo {
  static constexpr int E = kFftE;
  static constexpr int TT = N / E;       // threads per transform
  static constexpr int M = N / 4;        // dealiasing radius
  static constexpr int MP = M + 1;       // stored columns m_x = 0..M
  static constexpr int SP = 2 * M + 2;   // stored positions per state column
  static constexpr int NP = Padded<N, SCH>::value;
  static constexpr int MP4 = (MP + 3) / 4 * 4;  // mixed-domain columns, padded
  // LDS stride between transform groups that share a wavefront: TTSH_LDS_OFF
  // complex entries off a multiple of 32 (chosen by measuring LDS bank
  // conflicts on gfx950).
  static constexpr int LS = (fft_slots(3) * NP + 31) / 32 * 32 + TTSH_LDS_OFF;
};

// index of mixed-domain entry (field f, column m, row y)
template <int N>
__device__ __forceinline__ size_t mix_idx(int f, int m, int y) {
  return (size_t)f * Geo<N>::MP4 * N + (size_t)(m >> 2) * (4 * N) + 4 * y + (m & 3);
}

// z = p + i q
template <class T>
__device__ __forceinline__ C2<T> pack_pq(C2<T> p, C2<T> q) {
  return mk(p.x - q.y, p.y + q.x);
}

// ---------------------------------------------------------------------------
// row pass: RP row pairs per workgroup, TT threads per pair; `tile` selects
// rows 2 RP tile .. 2 RP (tile + 1) - 1 of instance `inst`
// ---------------------------------------------------------------------------
template <int N, int RP, class T, int SCH = kSchedDefault>
struct RowSmem {
  static constexpr size_t lds = (size_t)RP * Geo<N, SCH>::LS * sizeof(C2<T>);
  static constexpr size_t bytes = lds + (size_t)(RP * Geo<N, SCH>::TT / 64) * RP * 4 * sizeof(T);
};

// The row pass's output rows in contiguous form.  For field f and slab s
// (columns 4s..4s+3) the 2 RP rows of a tile are one run of 8 RP complex
// values in memory (rows 2 RP tile.., four columns each).  The forcing values
// are first placed in LDS in that order, then every run leaves as 16-byte
// pieces taken by consecutive threads, so that a wavefront writes whole
// 64 RP-byte runs instead of scattering 8-byte values over 4-column slabs
// (the row pass ran ~3.5 % faster that way on gfx950).  Runs sit one 16-byte
// piece apart in LDS so that the writes of four consecutive columns of
// successive slabs spread over the banks.
template <int N, int RP, class T>
struct RowStage {
  static constexpr int S = Geo<N>::MP4 / 4;                // slabs
  static constexpr int PC = 16 / (int)sizeof(C2<T>);       // complex values per piece
  static constexpr int QR = 8 * RP / PC;                   // pieces per run
  static constexpr int QS = QR + 1;                        // LDS pieces per run
  static constexpr int RS = QS * PC;                       // LDS complex values per run
  static constexpr size_t bytes(int fields) { return (size_t)fields * S * QS * 16; }
  // LDS complex index of (field f, column m, tile row r)
  __device__ static __forceinline__ int at(int f, int m, int r) {
    return (f * S + (m >> 2)) * RS + 4 * r + (m & 3);
  }
};

// the NF fields' runs of rows row0.. from LDS to memory (field stride fs,
// slab stride 4 N complex values)
template <int N, int RP, class T, int NT, int NF>
__device__ __forceinline__ void store_runs(C2<T>* mem, size_t fs, int row0, const unsigned char* lds, int tid) {
  using RS = RowStage<N, RP, T>;
  constexpr int NQ = NF * RS::S * RS::QR;
  const uint4* L = reinterpret_cast<const uint4*>(lds);
#pragma unroll
  for (int g0 = 0; g0 < NQ; g0 += NT) {
    const int g = g0 + tid;
    if (g < NQ) {
      const int run = g / RS::QR, w = g - run * RS::QR;
      const int f = run / RS::S, sl = run - f * RS::S;
      uint4* q = reinterpret_cast<uint4*>(mem + f * fs + (size_t)sl * 4 * N + 4 * row0) + w;
      *q = L[run * RS::QS + w];
    }
  }
}

template <int N, int RP, class T, bool GW, int SCH = kSchedDefault>
__device__ __forceinline__ void row_body(const C2<T>* __restrict__ X, C2<T>* __restrict__ Y,
                                         const T* __restrict__ K, T* __restrict__ rowsum,
                                         const C2<T>* __restrict__ tw, const RowCoef<T>& c,
                                         size_t inst, int tile, unsigned char* smem) {
  using G = Geo<N, SCH>;
  constexpr int E = G::E, TT = G::TT, M = G::M, MP = G::MP, NP = G::NP;
  constexpr int NFY = GW ? 3 : 2;
  constexpr int NT = RP * TT;
  constexpr int NW = NT / 64;
  static_assert(NT % 64 == 0, "row pass needs whole wavefronts");
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem);
  T(*red)[RP][4] = reinterpret_cast<T(*)[RP][4]>(smem + RowSmem<N, RP, T, SCH>::lds);

  const int tid = threadIdx.x;
  const int lane = tid % RP;
  const int t = tid / RP;
  // lets the compiler drop the zero band of the pruned inverse transforms and
  // the unused outputs of the pruned forward ones
  __builtin_assume(t >= 0 && t < TT);
  const int y0 = (tile * RP + lane) * 2;
  constexpr int MP4 = G::MP4;
  const C2<T>* Xp = X + inst * 3 * MP4 * N;
  C2<T>* Yp = Y + inst * NFY * MP4 * N;
  const T* Kp = K + inst * N * N;
  C2<T>* L = lds + lane * G::LS;

  // gather Z(m) over the full row spectrum from the stored m_x = 0..M half
  C2<T> z[3][E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = t + e * TT;
    const bool lo = idx <= M;
    const bool hi = idx >= N - M;
    const int m = lo ? idx : N - idx;
    CPair<T> a, b, w;
    a.a = a.b = b.a = b.b = w.a = w.b = mk<T>(0, 0);
    if (lo || hi) {
      a.a = Xp[mix_idx<N>(0, m, y0)];
      a.b = Xp[mix_idx<N>(0, m, y0 + 1)];
      b.a = Xp[mix_idx<N>(1, m, y0)];
      b.b = Xp[mix_idx<N>(1, m, y0 + 1)];
      w.a = Xp[mix_idx<N>(2, m, y0)];
      w.b = Xp[mix_idx<N>(2, m, y0 + 1)];
    }
    if (idx == 0) {  // real transform: the m_x = 0 term is real
      a.a.y = a.b.y = b.a.y = b.b.y = w.a.y = w.b.y = 0;
    }
    if (hi) {
      a.a = conj(a.a); a.b = conj(a.b);
      b.a = conj(b.a); b.b = conj(b.b);
      w.a = conj(w.a); w.b = conj(w.b);
    }
    z[0][e] = pack_pq(a.a, b.a);  // v_x + i v_y, row y0
    z[1][e] = pack_pq(a.b, b.b);  // v_x + i v_y, row y0+1
    z[2][e] = pack_pq(w.a, w.b);  // omega(y0) + i omega(y0+1)
  }
  fft<N, +1, 3, SCH, NT == 64>(z, L, t, tw);

  // mask rows, loaded after the inverse transforms: issued before them they
  // would hold 16 registers through the transforms (the row pass ran ~5 %
  // slower that way on gfx950)
  T kr[2][E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = t + e * TT;
    kr[0][e] = Kp[(size_t)y0 * N + x];
    kr[1][e] = Kp[(size_t)(y0 + 1) * N + x];
  }

  // real-space forcing at x = t + e*TT
  C2<T> wv[NFY][E];
  T s1[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
  for (int e = 0; e < E; ++e) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const T vx = z[r][e].x, vy = z[r][e].y;
      const T om = r ? z[2][e].y : z[2][e].x;
      const T s = c.beta * (vx * vx + vy * vy) + c.gamma_v * kr[r][e];
      const T r1x = -s * vx, r1y = -s * vy;
      s1[r][0] += r1x;
      s1[r][1] += r1y;
      wv[r][e] = mk(r1x + c.lambda0 * om * vy, r1y - c.lambda0 * om * vx);
    }
    if constexpr (GW)
      wv[NFY - 1][e] = mk(-c.gamma_w * kr[0][e] * z[2][e].x, -c.gamma_w * kr[1][e] * z[2][e].y);
  }
  fft<N, -1, NFY, SCH, NT == 64>(wv, L, t, tw);

#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q) s1[r][q] = wave_sum_from(s1[r][q], RP);
  if ((tid & 63) < RP) {
    red[tid >> 6][lane][0] = s1[0][0];
    red[tid >> 6][lane][1] = s1[0][1];
    red[tid >> 6][lane][2] = s1[1][0];
    red[tid >> 6][lane][3] = s1[1][1];
  }
  if constexpr (GW) {
    // G of the two rows shares one transform: split it through LDS,
    // G_y0(m) = (W(m) + W(N-m)^*)/2, G_y1(m) = -i (W(m) - W(N-m)^*)/2
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = t + e * TT;
      if (idx <= M || idx >= N - M) L[lds_pad<SCH>(idx)] = wv[2][e];
    }
    __syncthreads();
    const T h = (T)0.5;
#pragma unroll
    for (int e = 0; e <= M / TT; ++e) {
      const int m = t + e * TT;
      if (m <= M) {
        const C2<T> Wm = L[lds_pad<SCH>(m)];
        const C2<T> Wn = L[lds_pad<SCH>((N - m) & (N - 1))];
        Yp[mix_idx<N>(2, m, y0)] = mk(h * (Wm.x + Wn.x), h * (Wm.y - Wn.y));
        Yp[mix_idx<N>(2, m, y0 + 1)] = mk(h * (Wm.y + Wn.y), -h * (Wm.x - Wn.x));
      }
    }
  }
  __syncthreads();

  // Outputs.  The forcing rows are stored unsplit: Y[0][m][y] = W_y(m) and
  // Y[1][m][y] = W_y(N - m) (m = 0..M) with W_y = FFT(N_x + i N_y) of row y;
  // the column pass, whose thread loads both, separates
  // N_x_hat = (W(m) + W(N-m)^*)/2, N_y_hat = -i (W(m) - W(N-m)^*)/2.  The
  // values go to LDS in run order (the slab padding past m = M gets zeros,
  // which no reader uses) and leave as whole runs.
  using RS = RowStage<N, RP, T>;
  static_assert(RS::bytes(2) <= RowSmem<N, RP, T, SCH>::lds, "output runs exceed the transform scratch");
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = t + e * TT;
    if (idx < MP4) {
      const bool v = idx <= M;
      lds[RS::at(0, idx, 2 * lane)] = v ? wv[0][e] : mk<T>(0, 0);
      lds[RS::at(0, idx, 2 * lane + 1)] = v ? wv[1][e] : mk<T>(0, 0);
    }
    const int m = (N - idx) & (N - 1);
    if (m < MP4) {
      const bool v = m <= M;
      lds[RS::at(1, m, 2 * lane)] = v ? wv[0][e] : mk<T>(0, 0);
      lds[RS::at(1, m, 2 * lane + 1)] = v ? wv[1][e] : mk<T>(0, 0);
    }
  }
  lds_sync<NT == 64>();
  store_runs<N, RP, T, NT, 2>(Yp, (size_t)MP4 * N, tile * RP * 2, smem, tid);
  if (tid < RP) {
    T acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += red[w][tid][q];
    T* rs = rowsum + inst * 2 * N;
    rs[y0] = acc[0];
    rs[N + y0] = acc[1];
    rs[y0 + 1] = acc[2];
    rs[N + y0 + 1] = acc[3];
  }
}

// ---------------------------------------------------------------------------
// column pass: TC columns per workgroup, TT threads per column
// MODE 0: full step;  MODE 1: only state -> X (after the state was set)
// ---------------------------------------------------------------------------
template <int N, int TC, class T, bool GW, int SCH = kSchedDefault>
struct ColSmem {
  static constexpr size_t fft = (size_t)TC * Geo<N, SCH>::LS * sizeof(C2<T>);
  static constexpr size_t herm = (size_t)N * sizeof(C2<double>);
  static constexpr size_t bytes = fft > herm ? fft : herm;
};

// u(m_y) <- (u(m_y) + u(-m_y)^*)/2 over one column held as u[e] = entry
// t + e*TT by the threads with `active`; H holds N entries of LDS, and every
// thread of the workgroup must call this
template <int N>
__device__ __forceinline__ void hermitian_fix(C2<double> (&u)[kFftE], C2<double>* H, int t, bool active) {
  constexpr int E = kFftE, TT = N / E;
  __syncthreads();
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) H[t + e * TT] = u[e];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = cscale(u[e] + conj(H[(N - (t + e * TT)) & (N - 1)]), 0.5);
  }
  __syncthreads();
}

// MODE 2 / 3: the two stages of ETD2RK.  Stage 1 reads st and writes the
// stage state st2, and keeps its forcing spectra (compact, as the state:
// [NFY][M+1][2M+2]) in fst and its k = 0 forcing sums in s1st; stage 2 reads
// st2 and the kept values and writes st.
// MODE 4..7: the four stages of ETDRK4 (weights in etd4_weights).  Per
// instance fst holds two slots [2][NFY][M+1][2M+2] (slot 0: F(u), slot 1:
// F(a) + F(b)) and s1st four k = 0 sums (the same two, x and y).  Stage a
// (MODE 4) reads st, writes st2 = a and slot 0; stage b (5) reads st and
// writes slot 1; stage c (6) reads st2 and slot 0 and adds to slot 1; the
// last stage (7) reads st and both slots and writes st.  Stages b and c
// leave no state behind: only their mixed-domain fields X, which the next
// row pass turns into F(b) and F(c).
template <int N, int TC, class T, class S, bool GW, int MODE, int SCH = kSchedDefault>
__device__ __forceinline__ void col_body(const C2<T>* __restrict__ Y, C2<T>* __restrict__ X,
                                         C2<S>* __restrict__ st, const T* __restrict__ rowsum,
                                         const double* __restrict__ dkv,
                                         const C2<T>* __restrict__ tw, const LinCoef& lc,
                                         size_t inst, int tile, unsigned char* smem,
                                         C2<S>* __restrict__ st2 = nullptr, C2<T>* __restrict__ fst = nullptr,
                                         double* __restrict__ s1st = nullptr) {
  using G = Geo<N, SCH>;
  constexpr int E = G::E, TT = G::TT, M = G::M, MP = G::MP, SP = G::SP, NP = G::NP;
  constexpr int NFY = GW ? 3 : 2;
  constexpr int NT = TC * TT;
  constexpr int NW = NT / 64;
  static_assert(NT % 64 == 0, "column pass needs whole wavefronts");

  // up to four columns share a wavefront (consecutive threads walk the
  // columns of one 4-column slab, then the rows), so that each load or store
  // instruction covers a contiguous run of the interleaved layout
  constexpr int CI = TC < 4 ? TC : 4;
  const int tid = threadIdx.x;
  const int t = (tid / CI) % TT;
  const int col = (tid / (CI * TT)) * CI + tid % CI;
  __builtin_assume(t >= 0 && t < TT);
  const int mx = tile * TC + col;
  const bool valid = mx <= M;
  const double dk = dkv[inst];
  C2<T>* L = reinterpret_cast<C2<T>*>(smem) + col * G::LS;
  constexpr int SLOTS = MODE >= 4 ? 2 : 1;                                  // kept forcing spectra
  constexpr bool STORE = !(MODE == 5 || MODE == 6);                        // the stage keeps its state
  C2<S>* stp = ((MODE == 3 || MODE == 6) ? st2 : st) + inst * 2 * MP * SP;  // state read
  C2<S>* stq = ((MODE == 2 || MODE == 4) ? st2 : st) + inst * 2 * MP * SP;  // state written
  C2<T>* fsp = (MODE >= 2) ? fst + inst * SLOTS * NFY * MP * SP : nullptr;  // kept forcing
  double sux = 0.0, suy = 0.0, sax = 0.0, say = 0.0;                       // kept k = 0 sums

  C2<T> f[NFY][E];
  double s1x = 0.0, s1y = 0.0;
  if constexpr (MODE != 1) {
    if (tile == 0) {  // sum of the row sums: DFT of the k = 0 forcing
      const T* rs = rowsum + inst * 2 * N;
      double a = 0.0, b = 0.0;
      for (int y = tid; y < N; y += NT) {
        a += (double)rs[y];
        b += (double)rs[N + y];
      }
      a = wave_sum_from(a, 1);
      b = wave_sum_from(b, 1);
      double* R = reinterpret_cast<double*>(smem);
      if ((tid & 63) == 0) {
        R[2 * (tid >> 6)] = a;
        R[2 * (tid >> 6) + 1] = b;
      }
      __syncthreads();
      for (int w = 0; w < NW; ++w) {
        s1x += R[2 * w];
        s1y += R[2 * w + 1];
      }
      double* s4 = MODE >= 4 ? s1st + 4 * inst : nullptr;
      if constexpr (MODE == 6 || MODE == 7) {  // read before the barrier, written after it
        sux = s4[0];
        suy = s4[1];
        sax = s4[2];
        say = s4[3];
      }
      __syncthreads();
      if constexpr (MODE == 4 || MODE == 5) {
        if (tid == 0) {
          s4[MODE == 4 ? 0 : 2] = s1x;
          s4[MODE == 4 ? 1 : 3] = s1y;
        }
      } else if constexpr (MODE == 6) {
        if (tid == 0) {
          s4[2] = sax + s1x;
          s4[3] = say + s1y;
        }
      } else if constexpr (MODE == 2) {
        if (tid == 0) {
          s1st[2 * inst] = s1x;
          s1st[2 * inst + 1] = s1y;
        }
      } else if constexpr (MODE == 3) {
        s1x -= s1st[2 * inst];
        s1y -= s1st[2 * inst + 1];
      }
    }
    const C2<T>* Yp = Y + inst * NFY * G::MP4 * N;
    const T h = (T)0.5;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      C2<T> w0 = mk<T>(0, 0), w1 = mk<T>(0, 0);
      if (valid) {
        w0 = Yp[mix_idx<N>(0, mx, t + e * TT)];  // W(m_x) of row y
        w1 = Yp[mix_idx<N>(1, mx, t + e * TT)];  // W(N - m_x) of row y
      }
      f[0][e] = mk(h * (w0.x + w1.x), h * (w0.y - w1.y));   // row transform of N_x
      f[1][e] = mk(h * (w0.y + w1.y), -h * (w0.x - w1.x));  // row transform of N_y
      if constexpr (GW) f[2][e] = valid ? Yp[mix_idx<N>(2, mx, t + e * TT)] : mk<T>(0, 0);
    }
    fft<N, -1, NFY, SCH, NT == 64>(f, L, t, tw);
    if constexpr (MODE == 2 || MODE == 3) {  // keep (stage 1) or subtract (stage 2) the stage-1 forcing
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int idx = t + e * TT;
        const bool lo = idx <= M, hi = idx >= N - M;
        const int pos = lo ? idx : idx - (N - 2 * M - 1);
        const int my = lo ? idx : idx - N;
        if (valid && (lo || hi) && mx * mx + my * my <= M * M) {
#pragma unroll
          for (int q = 0; q < NFY; ++q) {
            C2<T>& slot = fsp[(q * MP + mx) * SP + pos];
            if constexpr (MODE == 2)
              slot = f[q][e];
            else
              f[q][e] = f[q][e] - slot;
          }
        }
      }
    }
  }

  // k-space update in FP64
  C2<double> nx[E], ny[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = t + e * TT;
    const bool lo = idx <= M, hi = idx >= N - M;
    const int my = lo ? idx : idx - N;
    const int pos = lo ? idx : idx - (N - 2 * M - 1);
    const int m2 = mx * mx + my * my;
    nx[e] = ny[e] = mk(0.0, 0.0);
    if (valid && (lo || hi) && m2 <= M * M) {
      const C2<double> ux = cvt<double>(stp[(0 * MP + mx) * SP + pos]);
      const C2<double> uy = cvt<double>(stp[(1 * MP + mx) * SP + pos]);
      if constexpr (MODE >= 4) {
        // ETDRK4 stage: the combination of the new forcing with the kept ones,
        // kept spectra updated on the way
        double A, wn, wu, wa;
        etd4_weights<MODE>(lc, dk, m2, A, wn, wu, wa);
        C2<double> g[NFY];
#pragma unroll
        for (int q = 0; q < NFY; ++q) {
          C2<T>* s0 = fsp + (q * MP + mx) * SP + pos;
          C2<T>* s1 = fsp + ((NFY + q) * MP + mx) * SP + pos;
          const C2<T> fn = f[q][e];
          g[q] = cscale(cvt<double>(fn), wn);
          if constexpr (MODE == 4) *s0 = fn;
          if constexpr (MODE == 5) *s1 = fn;
          if constexpr (MODE == 6) {
            g[q] = g[q] + cscale(cvt<double>(*s0), wu);
            *s1 = *s1 + fn;
          }
          if constexpr (MODE == 7) g[q] = g[q] + cscale(cvt<double>(*s0), wu) + cscale(cvt<double>(*s1), wa);
        }
        const double dt_over_N = lc.dt_over_N;
        if (m2 == 0) {
          nx[e] = cscale(ux, A) + mk(dt_over_N * (wn * s1x + wu * sux + wa * sax), 0.0);
          ny[e] = cscale(uy, A) + mk(dt_over_N * (wn * s1y + wu * suy + wa * say), 0.0);
        } else {
          double inv_m2;
          {
            const double dm = (double)m2;
            double r = (double)__frcp_rn((float)m2);
            r = r * (2.0 - dm * r);
            inv_m2 = r * (2.0 - dm * r);
          }
          C2<double> qx = cscale(ux, A) + cscale(g[0], dt_over_N);
          C2<double> qy = cscale(uy, A) + cscale(g[1], dt_over_N);
          const double dmx = mx, dmy = my;
          const C2<double> d = cscale(mk(dmx * qx.x + dmy * qy.x, dmx * qx.y + dmy * qy.y), inv_m2);
          qx = qx - cscale(d, dmx);
          qy = qy - cscale(d, dmy);
          if constexpr (GW) {
            const C2<double> gg = cscale(g[NFY - 1], dt_over_N * inv_m2 / dk);
            qx = qx + mk(-dmy * gg.y, dmy * gg.x);
            qy = qy + mk(dmx * gg.y, -dmx * gg.x);
          }
          nx[e] = qx;
          ny[e] = qy;
        }
      } else if constexpr (MODE != 1) {
        const double dt_over_N = lc.dt_over_N;
        double A, B;
        linear_ab<MODE>(lc, dk, m2, A, B);
        // 1/m^2: FP32 reciprocal refined by two Newton steps in FP64
        // (m^2 <= 2^16, so the result is the correctly rounded FP64 value to
        // within an ulp)
        double inv_m2 = 0.0;
        if (m2 > 0) {
          const double dm = (double)m2;
          double r = (double)__frcp_rn((float)m2);
          r = r * (2.0 - dm * r);
          r = r * (2.0 - dm * r);
          inv_m2 = r;
        }
        if (m2 == 0) {
          nx[e] = cscale(ux, A) + mk(B * dt_over_N * s1x, 0.0);
          ny[e] = cscale(uy, A) + mk(B * dt_over_N * s1y, 0.0);
        } else {
          // project the whole update (state and forcing), so that rounding
          // never leaves a divergent part for e^{L dt} to amplify
          const double bs = B * dt_over_N;
          C2<double> qx = cscale(ux, A) + cscale(cvt<double>(f[0][e]), bs);
          C2<double> qy = cscale(uy, A) + cscale(cvt<double>(f[1][e]), bs);
          const double dmx = mx, dmy = my;
          const C2<double> d = cscale(mk(dmx * qx.x + dmy * qy.x, dmx * qx.y + dmy * qy.y), inv_m2);
          qx = qx - cscale(d, dmx);
          qy = qy - cscale(d, dmy);
          if constexpr (GW) {
            const C2<double> g = cscale(cvt<double>(f[2][e]), bs * inv_m2 / dk);
            qx = qx + mk(-dmy * g.y, dmy * g.x);
            qy = qy + mk(dmx * g.y, -dmx * g.x);
          }
          nx[e] = qx;
          ny[e] = qy;
        }
      } else {
        nx[e] = ux;
        ny[e] = uy;
      }
    }
  }

  if constexpr (MODE != 1) {
    if (tile == 0) {  // Hermitian correction on the m_x = 0 column, x then y
      C2<double>* H = reinterpret_cast<C2<double>*>(smem);
      hermitian_fix<N>(nx, H, t, col == 0);
      hermitian_fix<N>(ny, H, t, col == 0);
    }
    // round to the stored precision; the transforms below start from the
    // stored values, so the stored spectrum is the whole state of the run
#pragma unroll
    for (int e = 0; e < E; ++e) {
      nx[e] = cvt<double>(cvt<S>(nx[e]));
      ny[e] = cvt<double>(cvt<S>(ny[e]));
    }
    if (valid && STORE) {
      // modes outside the 1/2-rule disk stay zero in memory and are not rewritten
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int idx = t + e * TT;
        const bool lo = idx <= M, hi = idx >= N - M;
        const int pos = lo ? idx : idx - (N - 2 * M - 1);
        const int my = lo ? idx : idx - N;
        if ((lo || hi) && mx * mx + my * my <= M * M) {
          stq[(0 * MP + mx) * SP + pos] = cvt<S>(nx[e]);
          stq[(1 * MP + mx) * SP + pos] = cvt<S>(ny[e]);
        }
      }
    }
  }

  // inverse column transforms of v_x, v_y and omega = i dk (m_x v_y - m_y v_x)
  const double sN = 1.0 / N;
  C2<T> z[3][E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = t + e * TT;
    const double dmy = (idx <= M) ? idx : idx - N;
    const C2<double> cw = cscale(ny[e], (double)mx) - cscale(nx[e], dmy);
    z[0][e] = cvt<T>(cscale(nx[e], sN));
    z[1][e] = cvt<T>(cscale(ny[e], sN));
    z[2][e] = cvt<T>(mk(-cw.y * dk * sN, cw.x * dk * sN));
  }
  fft<N, +1, 3, SCH, NT == 64>(z, L, t, tw);
  if (valid) {
    C2<T>* Xp = X + inst * 3 * G::MP4 * N;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int e = 0; e < E; ++e) Xp[mix_idx<N>(q, mx, t + e * TT)] = z[q][e];
  }
}

}  // namespace ttsh
