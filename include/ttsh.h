/*
 * ttsh.h -- C interface of libttsh.so: time stepping of the confined polar
 * active fluid velocity equation (incompressible Toner-Tu/Swift-Hohenberg,
 * "TTSH") with the damping-mask treatment of arbitrary boundaries, on AMD
 * Instinct MI355X (gfx950).
 *
 * Model (paper: method section, eqs. (1)-(4); general coefficient form):
 *   div v = 0,
 *   dv/dt + lambda0 (v.grad) v = -grad p + lambda1 grad|v|^2
 *        - (alpha + beta|v|^2) v + Gamma0 lap v - Gamma2 lap^2 v - gamma_v K v,
 *   and in the vorticity equation the extra term -gamma_w K omega (eq. (4)).
 * The paper's (a, b, lambda, gamma_v, gamma_w) is alpha = 1 - a, beta = b,
 * Gamma0 = -2, Gamma2 = 1, lambda0 = lambda, lambda1 = 0.
 *
 * Time step: Algorithm 1 of Appendix C (pseudo-spectral, unitary DFT,
 * exponential multiplier on the linear part, Euler on the rest, 1/2-rule
 * cutoff m_x^2 + m_y^2 > (N/4)^2, k = 0 rule from the averaged equation (7),
 * Hermitian correction, stream-function velocity), evaluated in the
 * equivalent spectral-velocity form with a Leray projection.
 *
 * Conventions
 *   Real fields are row-major [component][y][x] (component 0 = x) of float64;
 *   grid node (i, j) sits at x = (j - N/2) L/N, y = (i - N/2) L/N.
 *   Spectra use the paper's unitary DFT  f_hat(k) = N^-1 sum_x f(x) e^{-ik.x},
 *   k = (2 pi / L) m, and derivative multiplier +ik.
 *   A "compact state" is [2][2M+1][M+1] complex float64 (re, im interleaved),
 *   M = N/4: entry [c][m_y + M][m_x] holds v_hat_c(m_x, m_y) for m_x = 0..M,
 *   m_y = -M..M; modes with m_x < 0 follow from v_hat(-k) = v_hat(k)^*.
 *
 * Memory ("where" arguments): TTSH_HOST for host pointers, TTSH_DEVICE for
 *   device pointers.  The caller owns every buffer it passes; the library
 *   copies in or out and never keeps a pointer after the call returns.  Device
 *   buffers passed to asynchronous calls must stay valid until the work queued
 *   on the context's stream has completed (ttsh_sync).
 *
 * Errors: every int-returning call returns TTSH_OK (0) or a negative code;
 *   ttsh_last_error() gives a message for the calling thread.  No exception
 *   crosses the interface and the library never terminates the process.
 *
 * Threads: a context may be used by one thread at a time.
 */
#ifndef TTSH_H
#define TTSH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ttsh_ctx ttsh_ctx;

enum {
  TTSH_OK = 0,
  TTSH_EINVAL = -1,       /* invalid argument (null pointer, index, size) */
  TTSH_EUNSUPPORTED = -2, /* grid size or option not supported */
  TTSH_EHIP = -3,         /* HIP runtime error (no device, launch failure) */
  TTSH_ENONFINITE = -4,   /* NaN/Inf met in an input or in the state */
  TTSH_ENOMEM = -5        /* device allocation failed */
};

enum { TTSH_HOST = 0, TTSH_DEVICE = 1 };

/* One-step map of the stiff linear part, u' = A u + B dt f with
 * L = -alpha - Gamma0 k^2 - Gamma2 k^4, z = L dt:
 *   TTSH_IFEULER  A = B = exp(z)              (Algorithm 1, the default)
 *   TTSH_ETD1     A = exp(z), B = (exp(z) - 1)/z
 *   TTSH_IMEX     A = B = 1/(1 - z)
 *   TTSH_ETDRK2   second-order exponential Runge-Kutta (Cox and Matthews,
 *                 J. Comput. Phys. 176 (2002), ETD2RK): a = exp(z) u +
 *                 dt phi1(z) f(u), then u' = a + dt phi2(z) (f(a) - f(u)),
 *                 phi2(z) = (exp(z) - 1 - z)/z^2; two forcing evaluations
 *                 (twice the kernels) per step and, per instance, a second
 *                 state and the stage-1 forcing spectra on the device.
 *   TTSH_ETDRK4   fourth-order exponential Runge-Kutta (Cox and Matthews,
 *                 ETDRK4): with h = dt,
 *                   a = e^{z/2} u + (h/2) phi1(z/2) f(u)
 *                   b = e^{z/2} u + (h/2) phi1(z/2) f(a)
 *                   c = e^{z/2} a + (h/2) phi1(z/2) (2 f(b) - f(u))
 *                   u' = e^z u + h [f1 f(u) + 2 f2 (f(a) + f(b)) + f3 f(c)],
 *                 f1 = phi1 - 3 phi2 + 4 phi3, f2 = phi2 - 2 phi3,
 *                 f3 = -phi2 + 4 phi3, phi3(z) = (e^z - 1 - z - z^2/2)/z^3;
 *                 four forcing evaluations per step and, per instance, a
 *                 second state and two kept forcing spectra.
 * Every stage of the Runge-Kutta schemes applies Algorithm 1's rules
 * (projection of the whole update, k = 0 rule on rhs1, 1/2-rule cutoff,
 * Hermitian correction).                                                    */
enum { TTSH_IFEULER = 0, TTSH_ETD1 = 1, TTSH_IMEX = 2, TTSH_ETDRK2 = 3, TTSH_ETDRK4 = 4 };

/* Arithmetic of the step (precision argument of ttsh_create):
 *   TTSH_FP64         everything in FP64;
 *   TTSH_FP32         FFTs, real-space terms and the stored spectrum in FP32;
 *                     the linear factors, the k-space update and all norms in FP64;
 *   TTSH_FP32_STATE64 as TTSH_FP32 but the stored spectrum kept in FP64.     */
enum { TTSH_FP32 = 32, TTSH_FP64 = 64, TTSH_FP32_STATE64 = 96 };

typedef struct {
  double alpha, beta, gamma0, gamma2, lambda0, lambda1;
  double gamma_v; /* velocity damping in the wall, -gamma_v K v  (eq. (4)) */
  double gamma_w; /* vorticity damping in the wall, -gamma_w K omega (eq. (4)) */
  double dt;
  int scheme;     /* TTSH_IFEULER, TTSH_ETD1, TTSH_IMEX, TTSH_ETDRK2 or TTSH_ETDRK4 */
} ttsh_params;

/* Options for ttsh_set_option. */
enum {
  TTSH_OPT_GRAPH_STEPS = 1, /* steps captured per HIP graph (0 = no graph); default 50 */
  TTSH_OPT_BLOCK = 2,       /* workgroup size of the step kernels: 64, 128 or 256
                               (8 x size >= largest N), 0 = chosen from the batch */
  TTSH_OPT_GUARD = 4,       /* 1: ttsh_sync checks the state for NaN/Inf; default 1 */
  TTSH_OPT_SPLIT = 8,       /* bit 0: row pass, bit 1: column pass launched once per grid
                               size (kernels compiled for that size) instead of once for
                               all sizes; default 0 */
  TTSH_OPT_GUARD_EVERY = 16,/* with the guard on: steps between the NaN/Inf checks that
                               ttsh_step queues (part of the captured graphs; one launch
                               per grid size over all its instances, flags kept on the
                               device until ttsh_sync reports them); 0 = check only in
                               ttsh_sync; default 50 */
  TTSH_OPT_GROUPS = 17      /* 1 or 2: instance groups that ttsh_step advances
                               concurrently.  With 2, every grid size's instances are
                               split into two halves (in instance order), each half
                               stepping with its own launches, graphs and stream, so
                               that one half's row pass runs beside the other half's
                               column pass; results are the same bit for bit.
                               2 needs at least two instances (TTSH_EINVAL).
                               Default 1; ttsh_tune chooses. */
};

/* Create a context holding n_inst independent instances advanced together.
 *   N[i]   grid points per side of instance i: 64, 128, 256, 512, 1024, 2048,
 *          4096 or 8192 (2048: its passes run with 256-thread workgroups, in
 *          FP64 with about 70 KB of LDS per workgroup; 4096 and 8192, the
 *          paper's production sizes: N/8 threads per workgroup, one row pair
 *          or column each, up to 139 KB of LDS; 8192 needs TTSH_FP32 or
 *          TTSH_FP32_STATE64, else TTSH_EUNSUPPORTED).  Contexts with a grid
 *          above 1024 launch every pass once per grid size.
 *   L[i]   box side of instance i (> 0)
 *   p      coefficients shared by all instances
 *   precision  TTSH_FP32, TTSH_FP64 or TTSH_FP32_STATE64
 *   stream hipStream_t the work is queued on (NULL = the default stream)
 * The state starts at zero and the mask at K = 0.
 * Errors: TTSH_EINVAL, TTSH_EUNSUPPORTED, TTSH_EHIP, TTSH_ENOMEM.           */
int ttsh_create(ttsh_ctx** out, int n_inst, const int* N, const double* L, const ttsh_params* p,
                int precision, void* stream);

/* Release every device buffer and graph of the context (synchronises). */
void ttsh_destroy(ttsh_ctx* ctx);

/* Mask K(x) >= 0 of instance inst, [N][N] float64 (method section: K ~ 0
 * inside the system, ~ 1 in the wall).  Stored in the run precision.       */
int ttsh_set_mask(ttsh_ctx* ctx, int inst, const double* K, int where);

/* Read the stored mask back as [N][N] float64. */
int ttsh_get_mask(ttsh_ctx* ctx, int inst, double* K, int where);

/* Smoothed wall K = prod_c 1/2 [1 + tanh((|x - c| - R_c)/xi)] over n_circ
 * circles (1 <= n_circ <= 8) with centres (cx, cy) and radii R (host
 * arrays), evaluated in FP64 at the nodes (the tanh interpolation the method
 * section mentions; a product of circle outsides gives the dumbbell).       */
int ttsh_mask_tanh(ttsh_ctx* ctx, int inst, int n_circ, const double* cx, const double* cy,
                   const double* R, double xi);

/* Algorithm 2 (Appendix D): from a binary field K_naive [N][N] uint8 (nonzero
 * = wall), K = (Re iDFT[DFT[K_naive] with m_x^2 + m_y^2 > (N/8)^2 zeroed])^2. */
int ttsh_mask_from_binary(ttsh_ctx* ctx, int inst, const uint8_t* K_naive, int where);

/* Set the velocity of instance inst from a real field v [2][N][N] float64:
 * DFT, 1/2-rule cutoff, Leray projection (k != 0); the k = 0 mode is kept.
 * A field holding NaN or Inf is refused with TTSH_ENONFINITE before the
 * instance is touched (its state stays as it was).  Synchronous.           */
int ttsh_set_field(ttsh_ctx* ctx, int inst, const double* v, int where);

/* Real velocity v [2][N][N] and, if omega is not NULL, vorticity omega [N][N]
 * (omega = d_x v_y - d_y v_x) of instance inst, float64.  Synchronous.      */
int ttsh_get_field(ttsh_ctx* ctx, int inst, double* v, double* omega, int where);

/* Coarse real velocity of instance inst on an Nc x Nc grid of the same box
 * (Nc one of 64..2048, at most the context's largest N): the modes inside
 * both grids' 1/2-rule disks are copied by integer mode index, scaled by Nc/N
 * for the unitary DFT, and transformed back.  Output: device float32,
 * channels-last with a stride: component c of node (i, j) goes to
 * out[(i*Nc + j)*pix_stride + c], c = 0 (x), 1 (y); pix_stride >= 2.
 * Asynchronous on the context's stream.                                    */
int ttsh_get_field_coarse(ttsh_ctx* ctx, int inst, int Nc, float* out, int64_t pix_stride);

/* Order parameters of instance inst from its real-space fields (FP64, fixed
 * summation order; node (i, j) at x = (j - N/2) L/N, y = (i - N/2) L/N):
 *   out[0] = Psi, the vortex order parameter about (cx, cy) (circle
 *            section): ([sum |e_theta . v| / sum |v|] - 2/pi) / (1 - 2/pi);
 *   out[1] = Psi_2 (two-chamber section): with w_l, w_r the vorticity at the
 *            nodes of largest |omega| left of x = cx and at or right of it
 *            (ties to the first node in row-major order),
 *            |w_l + w_r| / (|w_l| + |w_r|).
 * Synchronous.                                                              */
int ttsh_order(ttsh_ctx* ctx, int inst, double cx, double cy, double* out);

/* Psi_2 of instance inst with the regions of the two-chamber section (sec.
 * "Dumbbell" geometry, order parameter of the two cavities): the nodes within
 * D/2 of either cavity centre, (cx - D/2, cy) for the left one (nodes left of
 * x = cx) and (cx + D/2, cy) for the right one (nodes at or right of x = cx),
 * D the distance between the centres.  Otherwise as out[1] of ttsh_order:
 * *psi2 = |w_l + w_r| / (|w_l| + |w_r|), or NaN if a region holds no node.
 * The disk test rounds each operation of
 * (x - c_x)^2 + (y - c_y)^2 <= (D/2)^2 separately (no fused multiply-add).
 * D must be positive and finite (else EINVAL).  Synchronous.               */
int ttsh_order_dumbbell(ttsh_ctx* ctx, int inst, double cx, double cy, double D, double* psi2);

/* Lyapunov exponents by Benettin's method (circle section, exponents of the
 * transition: perturbed copies of the state advanced with the same step and
 * re-orthonormalised by a QR decomposition).  Instances pert[0..p-1] hold
 * perturbed copies of instance base (same grid size, distinct, not base;
 * 1 <= p <= 16).  With d_v = (X_v - X_base)/eps the deviations of their
 * compact states, the call factors D = Q R by modified Gram-Schmidt in FP64
 * (in the order v = 0..p-1) under the inner product of the real fields
 * (sum over the grid nodes of v_a . v_b, i.e. the compact spectrum with
 * weight 1 on m_x = 0 and 2 on m_x > 0), writes X_v = X_base + eps q_v
 * (rounded to the stored precision; X_base unchanged) and returns
 * log_r[v] = log R_vv (host, [p]).  Calling it every tau steps and averaging
 * log_r / (tau dt) gives the p largest exponents.  eps is absolute, in the
 * units of the state's Parseval norm; it must be positive and finite
 * (EINVAL), and small enough for linear growth yet above the rounding of
 * the stored precision (FP64 states are the intended use).  A deviation with
 * nothing left after the projections gives ENONFINITE (the perturbed states
 * are then unspecified).  Uses a scratch of p FP64 compact states, grown on
 * demand.  Synchronous.                                                     */
int ttsh_lyap_qr(ttsh_ctx* ctx, int base, const int* pert, int p, double eps, double* log_r);

/* Temporal power spectral density of the vorticity (circle section, eq.
 * (PSD)): S(f) = (1/N^2) sum_x |sum_t omega(x, t) e^{-2 pi i f t}|^2, the sum
 * over the sampled times t at which ttsh_psd_accumulate is called, f in cycles
 * per unit time (Omega = 2 pi f).  The sums are kept in the spectral domain
 * (Parseval over x): acc is a caller-owned device buffer of
 * nf * 2 * (N/4 + 1) * (N/2 + 2) complex doubles (16 bytes each), zeroed by
 * the caller before the first sample; layout [nf][2][N/4+1][N/2+2] (+f, -f
 * sums per stored mode).  ttsh_psd_accumulate adds instance inst's
 * vorticity spectrum at time t, weighted by e^{-2 pi i f t}, for the nf
 * frequencies freqs (host array, 1 <= nf <= 4096, finite; EINVAL otherwise);
 * asynchronous on the context's stream (acc must stay valid until the work
 * completes; accumulations into one buffer are ordered by the stream).
 * ttsh_psd_finish reads a buffer built for grid size N and writes S[nf]
 * (host); synchronous.  Results do not depend on the order of the samples
 * beyond rounding, and are reproducible run to run.                        */
int ttsh_psd_accumulate(ttsh_ctx* ctx, int inst, int nf, const double* freqs, double t, void* acc);
int ttsh_psd_finish(ttsh_ctx* ctx, int N, int nf, const void* acc, double* S);

/* Vortex count of instance inst (the topological defects of the direction of
 * v, used to tell single vortices, pairs and disordered states apart): over
 * the grid cells whose four corner nodes all have K < kmax and |v| > vmin, the
 * winding number n of v around the cell (+1 at vortex centres of either sense
 * of rotation, -1 at saddles), and over the nodes with K < kmax but
 * |v| <= vmin whose eight neighbours qualify (a defect sitting on a node, as
 * at the centre of a symmetric vortex), the winding number around that ring;
 * from the real-space field in FP64.
 * out[0] = sum of n over cells with n > 0, out[1] = sum of -n over cells with
 * n < 0 (host ints).  vmin >= 0 excludes nodes where the direction of v is not
 * defined (stagnant wall region); vmin < 0 is EINVAL.  Synchronous.         */
int ttsh_vortices(ttsh_ctx* ctx, int inst, double kmax, double vmin, int* out);

/* Inverse of ttsh_get_field_coarse: set instance inst from a coarse real
 * velocity on an Nc x Nc grid of the same box (device float32, layout as in
 * ttsh_get_field_coarse).  The field is transformed, cut to the coarse 1/2
 * rule, Leray-projected (as in ttsh_set_field), and its modes are copied into
 * the instance's grid by integer mode index, scaled by N/Nc (modes beyond the
 * instance's own 1/2-rule disk are dropped).  Asynchronous.                 */
int ttsh_set_field_coarse(ttsh_ctx* ctx, int inst, int Nc, const float* v, int64_t pix_stride);

/* Project a batch of real velocity fields on an N x N periodic grid in place
 * onto the solver's state space: 1/2-rule cutoff (m^2 > (N/4)^2 dropped) and
 * Leray projection (sec. "Numerical method": divergence-free velocity), the
 * mean (k = 0) kept.  v: device float32, field b, node (i, j), component c at
 * v[((b*N + i)*N + j)*pix_stride + c].  If norms is non-null (host, [batch][2])
 * it receives, per projected field, sum_x |v|^2 and sum_x |w|^2 with w the
 * vorticity in integer-mode units (the physical enstrophy times (L/2 pi)^2),
 * and the call synchronises; else it is asynchronous.  Uses the context's
 * stream and grows a scratch buffer of 2 * batch * N^2 complex doubles.    */
int ttsh_project_coarse(ttsh_ctx* ctx, int N, float* v, int64_t pix_stride, int batch, double* norms);

/* Compact state in / out (layout above).  set_state rounds to the stored
 * precision, sets the modes outside the 1/2-rule disk (m_x^2 + m_y^2 > M^2)
 * to zero and performs no other projection; for a state that is zero outside
 * the disk, get_state(set_state(s)) returns s bit for bit when the stored
 * precision is FP64.  get_state is synchronous.                             */
int ttsh_set_state(ttsh_ctx* ctx, int inst, const double* vhat, int where);
int ttsh_get_state(ttsh_ctx* ctx, int inst, double* vhat, int where);

/* Advance every instance by nsteps >= 0 steps.  Asynchronous on the
 * context's stream.  With TTSH_OPT_GRAPH_STEPS = G > 0, whole chunks of G
 * steps replay one captured HIP graph and a remaining tail of r < G steps
 * replays a graph of r steps (captured on first use and kept while calls end
 * with the same tail); with G = 0 every kernel is launched directly.  With
 * TTSH_OPT_GROUPS = 2 each instance group replays graphs of its own on a
 * stream the library owns; those streams start after the work queued on the
 * context's stream before the call, and the context's stream waits for them
 * at the end of the call, so the ordering is that of a single stream.      */
int ttsh_step(ttsh_ctx* ctx, int64_t nsteps);

/* Continuation between stages (hysteresis protocol of the circle section:
 * each run starts from the final state of the previous one, with a small
 * random kick): for q = 0..n-1, simultaneously,
 *   state[dst[q]] <- resample(state[src[q]]) + P DFT[noise_q]
 * where resample copies the spectrum by integer mode index (zero padding or
 * truncation between grid sizes, scaled by N_dst/N_src for the unitary DFT),
 * P is the 1/2-rule cutoff plus the Leray projection (as in ttsh_set_field),
 * and noise_q [2][N_dst][N_dst] is drawn on the device by the counter-based
 * generator Philox-4x32-10 (Salmon et al., SC'11): key = (seed mod 2^32,
 * seed >> 32), counter = (i N_dst + j, dst[q], 0, 0) for node (i, j), and
 * output word c gives component c as noise_amp (2 u - 1), u = (word >> 8) 2^-24,
 * evaluated in FP64 (uniform on [-noise_amp, noise_amp)).  noise_amp = 0 adds
 * no noise.  dst and src are host arrays of instance indices; destinations
 * must be distinct; a destination may also be a source (all sources are read
 * before any destination is written).  Allocates a device scratch of the
 * destinations' compact FP64 spectra for the call.  Synchronous.
 * Errors: TTSH_EINVAL (indices, duplicates, non-finite noise_amp),
 * TTSH_ENOMEM, TTSH_EHIP.                                                   */
int ttsh_reseed(ttsh_ctx* ctx, int n, const int* dst, const int* src, double noise_amp, uint64_t seed);

/* ttsh_reseed without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, the same kernels and the same
 * result bit for bit; the destinations' resampled spectra go to a fixed
 * 64 MiB scratch in the library's device memory instead of a per-call
 * buffer, so the destinations' compact FP64 spectra, 32 (N_dst/4 + 1)
 * (N_dst/2 + 2) bytes each, may total at most 64 MiB (TTSH_EINVAL
 * otherwise, before any work is queued): the radius sweep's 64 destinations
 * (12 x 128^2, 16 x 256^2, 36 x 512^2) take 41.5 MiB; 15 destinations of
 * 1024^2 fit, 16 do not.
 * The scratch is shared by every call on one GPU and keeps the last call's
 * contents: calls that overlap on one GPU (two contexts on different
 * streams, or two threads) race; order them on one stream or synchronise.
 * Asynchronous on the context's stream (no synchronisation, no host
 * staging).                                                               */
int ttsh_reseed_noalloc(ttsh_ctx* ctx, int n, const int* dst, const int* src, double noise_amp,
                        uint64_t seed);

/* As ttsh_reseed, with caller-drawn noise: noise_q [2][N_dst][N_dst] float64
 * is the q-th block of `noise` (blocks stored back to back in the order of
 * dst; noise may be NULL for none), on the host (where = TTSH_HOST) or the
 * device (TTSH_DEVICE).  Synchronous.                                       */
int ttsh_reseed_field(ttsh_ctx* ctx, int n, const int* dst, const int* src, const double* noise,
                      int where);

/* FP64 diagnostics of instance inst (synchronous):
 * out[0] = sum_x |v|^2, out[1] = <v_x>, out[2] = <v_y>, out[3] = max |k . v_hat|. */
int ttsh_norms(ttsh_ctx* ctx, int inst, double out[4]);

/* Wait for the context's queued work; with TTSH_OPT_GUARD set, check every
 * instance's state once more and return TTSH_ENONFINITE if that check or any
 * check queued by ttsh_step since the last ttsh_sync found NaN/Inf (the
 * message names the lowest such instance); the flags are then cleared.     */
int ttsh_sync(ttsh_ctx* ctx);

/* Measurement: launch the row pass nsteps >= 1 times back to back, then the
 * column pass (integrating-factor Euler form) nsteps times back to back, each
 * run between two HIP events on the context's stream, and return the mean
 * launch durations in microseconds: out[0] = row pass, out[1] = column pass
 * (each launch covers every instance).  The row pass always reads the same
 * fields; the column pass re-applies its update with the same forcing, so
 * the state changes: save it first if it matters.  Synchronous.            */
int ttsh_pass_times(ttsh_ctx* ctx, int64_t nsteps, double* out);

/* Autotuner: for each of the two passes of a step, independently, time
 * nsteps back-to-back launches (as ttsh_pass_times, after two warm-up steps)
 * of every candidate configuration, in two rounds over all candidates, and
 * keep the fastest (each candidate's faster round):
 *   workgroup size 64, 128 or 256 (the rows or columns per tile follow:
 *   size / (N/8) for a grid of N points);
 *   one launch for all grid sizes, or one launch per grid size;
 *   with one launch for all sizes in the FP32 arithmetic, the transform
 *   schedule: the LDS padding (one slot per 8, 16 or 32 entries) and, for
 *   grids that are not a power of 8, whether the leftover radix (2 or 4)
 *   runs first or last (schedule code 2 * log2(padding period) + first:
 *   6, 7, 8 (the default: padding 16, radix last), 9, 10, 11).
 * Then whole steps (replayed as ttsh_step runs them, nsteps per candidate,
 * two rounds) decide between the column-pass sizes (each with its fastest
 * split and schedule) and between one and two concurrent instance groups
 * (TTSH_OPT_GROUPS), the row pass keeping its choice.
 * The state the context had before the call is restored.  cfg_out (7 ints,
 * may be NULL): row-pass size, column-pass size, row split (0/1), column
 * split (0/1), row schedule, column schedule, groups (the layout of
 * ttsh_set_tuning); us_out (may be NULL): microseconds per whole step of that
 * choice.  A later TTSH_OPT_BLOCK / TTSH_OPT_SPLIT / TTSH_OPT_GROUPS
 * overrides it.  Synchronous.                                               */
int ttsh_tune(ttsh_ctx* ctx, int64_t nsteps, int* cfg_out, double* us_out);

/* The launch configuration in use (7 ints, as cfg_out of ttsh_tune), and
 * setting one found earlier (for instance from a cache of tuner results)
 * without timing anything.  set: TTSH_EINVAL if a size does not fit the
 * context, a split flag is not 0/1, a schedule is unknown or used where
 * only the default exists (FP64 or FP32-state-64 arithmetic, one launch per
 * grid size, grids of 2048), or groups is not 1 or 2.                      */
int ttsh_get_tuning(ttsh_ctx* ctx, int* cfg);
int ttsh_set_tuning(ttsh_ctx* ctx, const int* cfg);

/* Name of the current HIP device's architecture (e.g. "gfx950:sramecc+:xnack-")
 * into out (NUL-terminated, at most n bytes); the key of tuner caches.     */
int ttsh_device_arch(char* out, int n);

/* Number of distinct grid sizes (size classes) in the context; their sizes in
 * increasing order go to N_out (may be NULL).                               */
int ttsh_num_classes(ttsh_ctx* ctx, int* N_out);

/* Set an option (TTSH_OPT_*); invalidates captured graphs. */
int ttsh_set_option(ttsh_ctx* ctx, int key, int64_t value);

/* Unitary 2D DFT (Appendix C definition) of `batch` complex N x N arrays,
 * device pointers, interleaved float64 [batch][N][N][2]; inverse != 0 for the
 * iDFT.  precision 32 runs the library's FP32 transform (inputs rounded),
 * 64 the FP64 one.  Synchronous; in and out may alias.                      */
int ttsh_fft2(const double* in, double* out, int N, int batch, int inverse, int precision);

/* Streaming-bandwidth probe (measurement only; no part of the method): a
 * kernel that reads `reads` arrays and writes `writes` arrays of `elems`
 * 16-byte elements each, element by element, with `blocks` workgroups of 256
 * threads; (reads, writes) is one of (1,1), (2,1), (3,1), (5,2), (1,0),
 * (0,1).  buf is a caller-owned device buffer of (reads + max(writes, 1)) *
 * elems * 16 bytes, 16-byte aligned, inputs first; a read-only run needs the
 * buffer zero-filled.  One untimed launch, then `reps` launches back to back on
 * the null stream between two HIP events; *us_out = mean microseconds per
 * launch.  Synchronous.                                                     */
int ttsh_stream_bench(int reads, int writes, int64_t elems, int blocks, int reps, void* buf, double* us_out);

/* Message of the last failed call on this thread ("" if none). */
const char* ttsh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TTSH_H */
