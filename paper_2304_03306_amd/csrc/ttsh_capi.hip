// Host runtime and C interface of libttsh.so (declared in include/ttsh.h).
//
// A context groups its instances by grid size ("size classes"); each class
// owns contiguous device arrays for its instances, so that one launch of the
// row pass and one of the column pass advance the whole class.  A step is
// [row pass, column pass] for every class; chunks of steps are captured once
// into a HIP graph and replayed on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ttsh.h"
#include "aux.hpp"
#include "launch.hpp"
#include "step_multi.hpp"

using namespace ttsh;

// Scratch of ttsh_reseed_noalloc: the destinations' resampled compact FP64
// spectra of one call, back to back.  It lives in the code object's device
// memory, so the call allocates nothing; every GPU that loads the library
// holds its own copy until the process ends.  In host code the name `scratch`
// is a host-side stand-in, not a device address: the runtime gives each
// device's address through hipGetSymbolAddress (see resolve_scratch), and
// only that address is passed to kernels.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kMaxGroups = 2;  // concurrent instance groups of ttsh_step
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace ttsh {
const SizeOps* ops_64();
const SizeOps* ops_128();
const SizeOps* ops_256();
const SizeOps* ops_512();
const SizeOps* ops_1024();
const SizeOps* ops_2048();
const SizeOps* ops_4096();
const SizeOps* ops_8192();
const BigOps* big_ops_4096_32();
const BigOps* big_ops_4096_64();
const BigOps* big_ops_4096_96();
const BigOps* big_ops_8192_32();
const BigOps* big_ops_8192_96();
const BigOps* big_ops(int N, int prec) {
  switch (N * 100 + prec) {
    case 409632: return big_ops_4096_32();
    case 409664: return big_ops_4096_64();
    case 409696: return big_ops_4096_96();
    case 819232: return big_ops_8192_32();
    case 819296: return big_ops_8192_96();
    default: return nullptr;
  }
}
const SizeOps* size_ops(int N) {
  switch (N) {
    case 64: return ops_64();
    case 128: return ops_128();
    case 256: return ops_256();
    case 512: return ops_512();
    case 1024: return ops_1024();
    case 2048: return ops_2048();
    case 4096: return ops_4096();
    case 8192: return ops_8192();
    default: return nullptr;
  }
}
#define TTSH_DECL(p)                   \
  const MultiOps* multi_ops_##p##_64();  \
  const MultiOps* multi_ops_##p##_128(); \
  const MultiOps* multi_ops_##p##_256();
TTSH_DECL(32)
TTSH_DECL(64)
TTSH_DECL(96)
#undef TTSH_DECL
#define TTSH_DECL_SCHED(b)                 \
  const SchedOps* sched_ops_##b##_6();   \
  const SchedOps* sched_ops_##b##_10();  \
  const SchedOps* sched_ops_##b##_9();   \
  const SchedOps* sched_ops_##b##_7();   \
  const SchedOps* sched_ops_##b##_11();
TTSH_DECL_SCHED(64)
TTSH_DECL_SCHED(128)
TTSH_DECL_SCHED(256)
#undef TTSH_DECL_SCHED
const SchedOps* sched_ops(int bs, int sch) {
  switch (bs * 100 + sch) {
#define TTSH_CASE(b, s) \
  case b * 100 + s: return sched_ops_##b##_##s();
    TTSH_CASE(64, 6) TTSH_CASE(64, 10) TTSH_CASE(64, 9) TTSH_CASE(64, 7) TTSH_CASE(64, 11)
    TTSH_CASE(128, 6) TTSH_CASE(128, 10) TTSH_CASE(128, 9) TTSH_CASE(128, 7) TTSH_CASE(128, 11)
    TTSH_CASE(256, 6) TTSH_CASE(256, 10) TTSH_CASE(256, 9) TTSH_CASE(256, 7) TTSH_CASE(256, 11)
#undef TTSH_CASE
    default: return nullptr;
  }
}
const MultiOps* multi_ops(int prec, int bs) {
  switch (prec * 1000 + bs) {
    case 32064: return multi_ops_32_64();
    case 32128: return multi_ops_32_128();
    case 32256: return multi_ops_32_256();
    case 64064: return multi_ops_64_64();
    case 64128: return multi_ops_64_128();
    case 64256: return multi_ops_64_256();
    case 96064: return multi_ops_96_64();
    case 96128: return multi_ops_96_128();
    case 96256: return multi_ops_96_256();
    default: return nullptr;
  }
}
}  // namespace ttsh

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

namespace ttsh {
int record_error(int code, const char* msg) {
  g_err = msg ? msg : "";
  return code;
}
}  // namespace ttsh

namespace {

// device address of `scratch` per HIP device, taken once per device with that
// device current (at the first ttsh_create there)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(TTSH_EUNSUPPORTED, "device index beyond the scratch address table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return TTSH_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(TTSH_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = p;
  return TTSH_OK;
}

}  // namespace

namespace {

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(TTSH_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t elem_real(int prec) { return prec == 64 ? sizeof(double) : sizeof(float); }
// kept forcing slots per instance of an exponential Runge-Kutta scheme (0: none)
int etd_slots(int scheme) { return scheme == TTSH_ETDRK2 ? 1 : scheme == TTSH_ETDRK4 ? 2 : 0; }
size_t elem_state(int prec) { return prec == 32 ? 2 * sizeof(float) : 2 * sizeof(double); }

struct SizeClass {
  int N = 0;
  std::vector<int> ids;  // context instance ids, in order
  void* X = nullptr;
  void* Y = nullptr;
  void* st = nullptr;
  void* K = nullptr;
  void* rowsum = nullptr;
  double* dk = nullptr;
  void* tw = nullptr;    // run precision
  void* st2 = nullptr;   // ETD2RK / ETDRK4: stage state (as st), kept forcing spectra, k = 0 sums
  void* fst = nullptr;
  double* s1st = nullptr;
  int* gflags = nullptr;  // the class's guard flags, in the order of ids (inside the context's dflags)
  // per-instance strides in elements
  // mixed-domain arrays hold M+1 columns padded to a multiple of 4
  size_t mp4() const { return (size_t)((N / 4 + 1 + 3) / 4 * 4); }
  size_t sX() const { return (size_t)3 * mp4() * N; }
  size_t sY(int gw) const { return (size_t)(gw ? 3 : 2) * mp4() * N; }
  size_t sSt() const { return (size_t)2 * (N / 4 + 1) * (N / 2 + 2); }
  // compact forcing spectra of one kept slot (ETD2RK keeps one, ETDRK4 two), complex elements
  size_t sF(int gw) const { return (size_t)(gw ? 3 : 2) * (N / 4 + 1) * (N / 2 + 2); }
  size_t sK() const { return (size_t)N * N; }
};

}  // namespace

struct ttsh_ctx {
  int n_inst = 0;
  std::vector<int> N;
  std::vector<double> L;
  ttsh_params p{};
  int prec = 32;
  int gw = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  std::vector<SizeClass> cls;
  std::vector<std::pair<int, int>> loc;  // instance -> (class, index in class)
  std::map<int, void*> tw64;             // FP64 twiddles per N (set-up paths)
  std::map<int, void*> tw32;             // FP32 twiddles per N
  void* scr0 = nullptr;                  // FP64 complex N^2 of the largest N
  void* scr1 = nullptr;
  double* dnorm = nullptr;               // [n_inst][5]; kNormBlocks x 5 partials follow
  int* dflags = nullptr;                 // [n_inst] non-finite flags of the guard
  int guard_every = 50;                  // steps between guard checks inside ttsh_step (0: only at ttsh_sync)
  void* pb0 = nullptr;                   // batched coarse-field spectra (grown on demand)
  void* pb1 = nullptr;
  size_t pb_cap = 0;                     // bytes of each
  double* pnorm = nullptr;               // [pnorm_cap][2]
  int pnorm_cap = 0;
  void* lyq = nullptr;                   // Lyapunov vectors: kMaxLyap logs, then [p][state] FP64
  size_t lyq_cap = 0;                    // bytes
  double* psdf = nullptr;                // PSD frequencies [kMaxPsdFreqs], then S [kMaxPsdFreqs]
  std::vector<double> psd_freqs;         // the frequencies in psdf
  int graph_steps = 50;
  int bs = 0;       // workgroup size of the column pass in use
  int bs_row = 0;   // workgroup size of the row pass in use
  int opt_bs = 0;   // requested by TTSH_OPT_BLOCK (0 = chosen)
  int split_row = 0, split_col = 0;  // one launch per size class (TTSH_OPT_SPLIT)
  int sched_row = kSchedDefault;     // transform schedule of the row pass (multi-size launch, FP32)
  int sched_col = kSchedDefault;     // and of the one-stage column pass
  int guard = 1;
  int device = 0;                        // HIP device current at creation
  hipGraph_t graph = nullptr;            // graph_steps steps
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph_rem = nullptr;        // rem_steps (< graph_steps) steps: the tail of the last call
  hipGraphExec_t gexec_rem = nullptr;
  int rem_steps = 0;
  // Concurrent instance groups (TTSH_OPT_GROUPS): with groups = 2 every size
  // class is split into two halves, and each half steps on a stream of its
  // own with graphs of its own, so that the row pass of one half runs on the
  // GPU beside the column pass of the other (the two passes are bound by
  // different units: the transforms' arithmetic and the memory traffic).
  int groups = 1;
  hipStream_t gstream[kMaxGroups] = {};
  hipEvent_t gfork = nullptr;
  hipEvent_t gjoin[kMaxGroups] = {};
  hipGraph_t ggraph[kMaxGroups] = {};
  hipGraphExec_t ggexec[kMaxGroups] = {};
  hipGraph_t ggraph_rem[kMaxGroups] = {};
  hipGraphExec_t ggexec_rem[kMaxGroups] = {};
};

namespace {

void drop_one(hipGraph_t& g, hipGraphExec_t& x) {
  if (x) (void)hipGraphExecDestroy(x);
  if (g) (void)hipGraphDestroy(g);
  x = nullptr;
  g = nullptr;
}

// Executable graphs may still run from an earlier asynchronous ttsh_step: the
// graphs are only destroyed after the context's stream, which every step call
// ends on (the group streams join it), has drained.
void drop_graph(ttsh_ctx* c) {
  bool any = c->gexec || c->gexec_rem;
  for (int g = 0; g < kMaxGroups; ++g) any = any || c->ggexec[g] || c->ggexec_rem[g];
  if (any) (void)hipStreamSynchronize(c->stream);
  drop_one(c->graph, c->gexec);
  drop_one(c->graph_rem, c->gexec_rem);
  for (int g = 0; g < kMaxGroups; ++g) {
    drop_one(c->ggraph[g], c->ggexec[g]);
    drop_one(c->ggraph_rem[g], c->ggexec_rem[g]);
  }
  c->rem_steps = 0;
}

int make_twiddles(int N, bool fp64, void** out) {
  std::vector<double> w(2 * N);
  for (int j = 0; j < N; ++j) {
    const double a = 2.0 * M_PI * (double)j / (double)N;
    w[2 * j] = std::cos(a);
    w[2 * j + 1] = -std::sin(a);
  }
  if (fp64) {
    HIPCHK(hipMalloc(out, sizeof(double) * 2 * N));
    HIPCHK(hipMemcpy(*out, w.data(), sizeof(double) * 2 * N, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(2 * N);
    for (int j = 0; j < 2 * N; ++j) f[j] = (float)w[j];
    HIPCHK(hipMalloc(out, sizeof(float) * 2 * N));
    HIPCHK(hipMemcpy(*out, f.data(), sizeof(float) * 2 * N, hipMemcpyHostToDevice));
  }
  return TTSH_OK;
}

int max_N(const ttsh_ctx* c) {
  int m = 0;
  for (auto& k : c->cls) m = std::max(m, k.N);
  return m;
}

// the tiles of a size-N class fit the per-tile LDS limit at workgroup size BS
// (transform precision T; the column pass with and without the vorticity source)
template <class T, int BS>
bool tiles_fit(int N, int gw) {
  return row_smem_of<T, BS>(N) > 0 && col_smem_of<T, BS, false>(N) > 0 && (!gw || col_smem_of<T, BS, true>(N) > 0);
}

// the largest size served by the 64..256-thread kernels (0 if none)
int max_small_N(const ttsh_ctx* c) {
  int m = 0;
  for (auto& k : c->cls)
    if (k.N <= kMaxBlockN) m = std::max(m, k.N);
  return m;
}

// workgroup size of a class's tiles in one pass: the chosen size, or N/8 for
// the production sizes (one row pair or column per workgroup)
int class_bs(const ttsh_ctx* c, int N, int row) { return N > kMaxBlockN ? N / 8 : (row ? c->bs_row : c->bs); }

// A workgroup of bs threads carries one transform of length N with N/8
// threads, so bs is usable when 8 bs >= N for every size class up to 2048
// and every such class's tiles fit the LDS limit (FP64 tiles of many small
// columns do not); larger classes have workgroups of their own size.
bool bs_valid(const ttsh_ctx* c, int bs) {
  if (!(bs == 64 || bs == 128 || bs == 256) || 8 * bs < max_small_N(c)) return false;
  const bool f64 = c->prec == 64;
  for (auto& k : c->cls) {
    if (k.N > kMaxBlockN) continue;
    bool ok = false;
    if (bs == 64) ok = f64 ? tiles_fit<double, 64>(k.N, c->gw) : tiles_fit<float, 64>(k.N, c->gw);
    if (bs == 128) ok = f64 ? tiles_fit<double, 128>(k.N, c->gw) : tiles_fit<float, 128>(k.N, c->gw);
    if (bs == 256) ok = f64 ? tiles_fit<double, 256>(k.N, c->gw) : tiles_fit<float, 256>(k.N, c->gw);
    if (!ok) return false;
  }
  return true;
}

// Default workgroup size: the largest one that still gives >= 2048 row-pass
// workgroups (8 per compute unit), else the smallest usable one.
int choose_bs(ttsh_ctx* c) {
  if (c->opt_bs) {
    if (!bs_valid(c, c->opt_bs)) return fail(TTSH_EUNSUPPORTED, "workgroup size not usable for this context");
    c->bs = c->bs_row = c->opt_bs;
    return TTSH_OK;
  }
  long pts = 0;
  for (size_t i = 0; i < c->N.size(); ++i) pts += (long)c->N[i] * c->N[i];
  int best = 0;
  for (int bs : {64, 128, 256}) {
    if (!bs_valid(c, bs)) continue;
    if (!best || pts / (16L * bs) >= 2048) best = bs;
  }
  if (!best) return fail(TTSH_EUNSUPPORTED, "no workgroup size fits N");
  c->bs = c->bs_row = best;
  return TTSH_OK;
}

ClassArgs class_args(ttsh_ctx* c, SizeClass& k, int first, int count, int row) {
  ClassArgs a{};
  const size_t er = elem_real(c->prec), es = elem_state(c->prec);
  const int R = class_bs(c, k.N, row) / (k.N / 8);
  a.N = k.N;
  a.n = count;
  a.tiles = row ? k.N / (2 * R) : (k.N / 4 + 1 + R - 1) / R;
  a.X_in = (const char*)k.X + first * k.sX() * 2 * er;
  a.X_out = (char*)k.X + first * k.sX() * 2 * er;
  a.Y = (char*)k.Y + first * k.sY(c->gw) * 2 * er;
  a.st = (char*)k.st + first * k.sSt() * es;
  a.K = (const char*)k.K + first * k.sK() * er;
  a.rowsum = (char*)k.rowsum + first * (size_t)2 * k.N * er;
  a.dk = k.dk + first;
  a.tw = k.tw;
  if (k.st2) {
    const int slots = etd_slots(c->p.scheme);
    a.st2 = (char*)k.st2 + first * k.sSt() * es;
    a.fst = (char*)k.fst + first * slots * k.sF(c->gw) * 2 * er;
    a.s1st = k.s1st + 2 * slots * first;
  }
  return a;
}

// instances [first, end) of class k that belong to group g of G (contiguous
// halves of the class, so that both groups carry every grid size)
std::pair<int, int> group_range(const SizeClass& k, int g, int G) {
  const int n = (int)k.ids.size();
  return {(int)((int64_t)n * g / G), (int)((int64_t)n * (g + 1) / G)};
}

// Launch arguments of one pass over group g of G (classes without instances
// in the group are left out; ncls = 0 if the group is empty).
MultiArgs group_args(ttsh_ctx* c, int row, int g, int G) {
  MultiArgs m{};
  m.beta = c->p.beta;
  m.gamma_v = c->p.gamma_v;
  m.lambda0 = c->p.lambda0;
  m.gamma_w = c->p.gamma_w;
  m.lc = LinCoef{c->p.alpha, c->p.gamma0, c->p.gamma2, c->p.dt, 0.0, c->p.scheme};
  int blocks = 0;
  for (auto& k : c->cls) {
    const auto [first, end] = group_range(k, g, G);
    if (end <= first) continue;
    ClassArgs a = class_args(c, k, first, end - first, row);
    m.start[m.ncls] = blocks;
    m.c[m.ncls++] = a;
    blocks += a.tiles * (end - first);
  }
  m.start[m.ncls] = blocks;
  return m;
}

// Launch arguments of one pass: all instances (inst < 0) or one instance.
MultiArgs multi_args(ttsh_ctx* c, int row, int inst) {
  MultiArgs m{};
  m.beta = c->p.beta;
  m.gamma_v = c->p.gamma_v;
  m.lambda0 = c->p.lambda0;
  m.gamma_w = c->p.gamma_w;
  m.lc = LinCoef{c->p.alpha, c->p.gamma0, c->p.gamma2, c->p.dt, 0.0, c->p.scheme};
  int blocks = 0;
  auto add = [&](SizeClass& k, int first, int count) {
    ClassArgs a = class_args(c, k, first, count, row);
    m.start[m.ncls] = blocks;
    m.c[m.ncls++] = a;
    blocks += a.tiles * count;
  };
  if (inst < 0) {
    for (auto& k : c->cls) add(k, 0, (int)k.ids.size());
  } else {
    auto [ci, j] = c->loc[inst];
    add(c->cls[ci], j, 1);
  }
  m.start[m.ncls] = blocks;
  return m;
}

// contexts with 2048-point grids always launch per size class (the multi-size
// kernels are not compiled for that size)
bool must_split(const ttsh_ctx* c) { return max_N(c) > 1024; }

// a non-default transform schedule exists for the multi-size launches of the
// FP32 arithmetic (row pass, one-stage column pass)
bool sched_usable(const ttsh_ctx* c, int split) { return c->prec == 32 && !split && !must_split(c); }

// the launch arguments of class q of m alone
MultiArgs only_class(const MultiArgs& m, int q) {
  MultiArgs o = m;
  o.ncls = 1;
  o.c[0] = m.c[q];
  o.start[0] = 0;
  o.start[1] = m.start[q + 1] - m.start[q];
  return o;
}

hipError_t launch_row(ttsh_ctx* c, const MultiArgs& m, hipStream_t s) {
  const bool split = c->split_row || must_split(c);
  if (c->sched_row != kSchedDefault && sched_usable(c, split))
    return sched_ops(c->bs_row, c->sched_row)->row(m, c->gw, s);
  const int tp = c->prec == 64 ? 64 : 32;  // the row pass depends on the transform precision only
  const MultiOps* o = multi_ops(tp, c->bs_row);
  if (!split) return o->row(m, c->gw, s);
  for (int q = 0; q < m.ncls; ++q) {
    const MultiArgs a = only_class(m, q);
    const hipError_t e = a.c[0].N > kMaxBlockN ? big_ops(a.c[0].N, tp)->row(a, c->gw, s) : o->row_split(a, c->gw, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t launch_col(ttsh_ctx* c, const MultiArgs& m, int mode, hipStream_t s) {
  const bool split = c->split_col || must_split(c);
  if (mode == 0 && c->sched_col != kSchedDefault && sched_usable(c, split))
    return sched_ops(c->bs, c->sched_col)->col(m, c->gw, s);
  const MultiOps* o = multi_ops(c->prec, c->bs);
  if (!split) return o->col(m, c->gw, mode, s);
  for (int q = 0; q < m.ncls; ++q) {
    const MultiArgs a = only_class(m, q);
    const hipError_t e =
        a.c[0].N > kMaxBlockN ? big_ops(a.c[0].N, c->prec)->col(a, c->gw, mode, s) : o->col_split(a, c->gw, mode, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_guard(ttsh_ctx* c, hipStream_t s, int g = 0, int G = 1);

// n steps of group g of G on stream s
int enqueue_steps(ttsh_ctx* c, int64_t n, hipStream_t s, int g = 0, int G = 1) {
  if (n <= 0) return TTSH_OK;
  const MultiArgs r = group_args(c, 1, g, G), q = group_args(c, 0, g, G);
  if (r.ncls == 0) return TTSH_OK;
  // column-pass modes of one step, each after a row pass that evaluates the
  // forcing of the state the previous one left in X
  static const int one[] = {0}, etd2[] = {2, 3}, etd4[] = {4, 5, 6, 7};
  const int* modes = one;
  int nm = 1;
  if (c->p.scheme == TTSH_ETDRK2) modes = etd2, nm = 2;
  if (c->p.scheme == TTSH_ETDRK4) modes = etd4, nm = 4;
  for (int64_t i = 0; i < n; ++i) {
    for (int j = 0; j < nm; ++j) {
      HIPCHK(launch_row(c, r, s));
      HIPCHK(launch_col(c, q, modes[j], s));
    }
    // the guard after every guard_every steps of this sequence (inside a
    // captured chunk of G steps: after steps guard_every, 2 guard_every, ...)
    if (c->guard && c->guard_every > 0 && (i + 1) % c->guard_every == 0) HIPCHK(launch_guard(c, s, g, G));
  }
  return TTSH_OK;
}

// capture `steps` steps of group g of G into a graph and instantiate it
int build_graph(ttsh_ctx* c, int steps, hipGraph_t* graph, hipGraphExec_t* gexec, int grp = 0, int G = 1) {
  HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_steps(c, steps, c->cap, grp, G);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (rc != TTSH_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(TTSH_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  *graph = g;
  HIPCHK(hipGraphInstantiate(gexec, g, nullptr, nullptr, 0));
  return TTSH_OK;
}

int check_inst(ttsh_ctx* c, int inst) {
  if (!c) return fail(TTSH_EINVAL, "null context");
  if (inst < 0 || inst >= c->n_inst) return fail(TTSH_EINVAL, "instance index out of range");
  return TTSH_OK;
}

// device pointer to instance data of class k at index j
template <class Tp>
Tp* at(void* base, size_t stride_elems, size_t elem_bytes, int j) {
  return (Tp*)((char*)base + (size_t)j * stride_elems * elem_bytes);
}

int stage_in(ttsh_ctx* c, const void* src, size_t bytes, int where, const void** dev) {
  if (!src) return fail(TTSH_EINVAL, "null input pointer");
  if (where == TTSH_DEVICE) {
    *dev = src;
    return TTSH_OK;
  }
  if (where != TTSH_HOST) return fail(TTSH_EINVAL, "where must be TTSH_HOST or TTSH_DEVICE");
  HIPCHK(hipMemcpyAsync(c->scr1, src, bytes, hipMemcpyHostToDevice, c->stream));
  *dev = c->scr1;
  return TTSH_OK;
}

const unsigned kB = 256;
unsigned nblk(size_t n) { return (unsigned)((n + kB - 1) / kB); }

// X of one instance from its state
int refresh_x(ttsh_ctx* c, int inst) {
  HIPCHK(launch_col(c, multi_args(c, 0, inst), 1, c->stream));
  return TTSH_OK;
}

// Z (FP64, e.g. scr0) holds the unnormalised FFT of v_x + i v_y, or is null
// for no field; `add` optional.
int pack_into_state(ttsh_ctx* c, int inst, const void* Z, const void* add) {
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, M = N / 4;
  const size_t n = (size_t)(M + 1) * (2 * M + 2);
  if (c->prec == 32) {
    hipLaunchKernelGGL(k_pack_state<float>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       (const C2<double>*)Z, (const C2<double>*)add,
                       at<C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), N);
  } else {
    hipLaunchKernelGGL(k_pack_state<double>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       (const C2<double>*)Z, (const C2<double>*)add,
                       at<C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), N);
  }
  HIPCHK(hipGetLastError());
  return TTSH_OK;
}

// FP64 twiddles for a grid size that may differ from the context's sizes
int twiddles64(ttsh_ctx* c, int N, const void** out) {
  auto it = c->tw64.find(N);
  if (it == c->tw64.end()) {
    void* t = nullptr;
    int rc = make_twiddles(N, true, &t);
    if (rc) return rc;
    it = c->tw64.emplace(N, t).first;
  }
  *out = it->second;
  return TTSH_OK;
}

// forward FP64 FFT of a real field pair v [2][N][N] (device) into scr0
int field_to_spectrum(ttsh_ctx* c, int N, const double* v) {
  const int n = N * N;
  hipLaunchKernelGGL(k_pack_xy, dim3(nblk(n)), dim3(kB), 0, c->stream, v, (C2<double>*)c->scr0, n);
  HIPCHK(hipGetLastError());
  HIPCHK(size_ops(N)->fft2(c->scr0, 1, -1, 1, c->tw64[N], c->stream));
  return TTSH_OK;
}

int norms_into(ttsh_ctx* c, int inst, double* dout) {
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const double dk = 2.0 * M_PI / c->L[inst];
  double* part = c->dnorm + 5 * c->n_inst;
  if (c->prec == 32)
    hipLaunchKernelGGL(k_norms<float>, dim3(kNormBlocks), dim3(256), 0, c->stream,
                       at<const C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), k.N, dk, part);
  else
    hipLaunchKernelGGL(k_norms<double>, dim3(kNormBlocks), dim3(256), 0, c->stream,
                       at<const C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), k.N, dk, part);
  hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(64), 0, c->stream, (const double*)part, kNormBlocks, dout);
  HIPCHK(hipGetLastError());
  return TTSH_OK;
}

// the non-finite guard over every instance: sets the flags of the instances
// that hold NaN or Inf (ttsh_sync reads and clears them); the flags of a
// class are stored in the class's instance order
hipError_t launch_guard(ttsh_ctx* c, hipStream_t s, int g, int G) {
  for (auto& k : c->cls) {
    const auto [first, end] = group_range(k, g, G);
    if (end <= first) continue;
    const size_t per = (size_t)2 * (k.N / 4 + 1) * (k.N / 2 + 2);
    const dim3 grid((unsigned)std::min<size_t>((per + 2047) / 2048, 64), (unsigned)(end - first));
    if (c->prec == 32)
      hipLaunchKernelGGL(k_guard<float>, grid, dim3(256), 0, s, (const C2<float>*)k.st + first * per, k.N,
                         k.gflags + first);
    else
      hipLaunchKernelGGL(k_guard<double>, grid, dim3(256), 0, s, (const C2<double>*)k.st + first * per, k.N,
                         k.gflags + first);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// streams and events of the concurrent groups, made on first use
int ensure_groups(ttsh_ctx* c) {
  if (!c->gfork && hipEventCreateWithFlags(&c->gfork, hipEventDisableTiming) != hipSuccess)
    return fail(TTSH_EHIP, "event creation failed");
  for (int g = 0; g < c->groups; ++g) {
    if (!c->gstream[g] && hipStreamCreateWithFlags(&c->gstream[g], hipStreamNonBlocking) != hipSuccess)
      return fail(TTSH_EHIP, "stream creation failed");
    if (!c->gjoin[g] && hipEventCreateWithFlags(&c->gjoin[g], hipEventDisableTiming) != hipSuccess)
      return fail(TTSH_EHIP, "event creation failed");
  }
  return TTSH_OK;
}

// the work of step_groups between the fork and the join
int step_groups_body(ttsh_ctx* c, int64_t nsteps, int G) {
  int rc;
  if (c->graph_steps <= 0) {
    for (int g = 0; g < G; ++g)
      if ((rc = enqueue_steps(c, nsteps, c->gstream[g], g, G))) return rc;
  } else {
    int64_t left = nsteps;
    if (left >= c->graph_steps) {
      for (int g = 0; g < G; ++g)
        if (!c->ggexec[g] && (rc = build_graph(c, c->graph_steps, &c->ggraph[g], &c->ggexec[g], g, G))) return rc;
      for (; left >= c->graph_steps; left -= c->graph_steps)
        for (int g = 0; g < G; ++g) HIPCHK(hipGraphLaunch(c->ggexec[g], c->gstream[g]));
    }
    if (left > 0) {
      if (c->rem_steps != (int)left) {
        // an old tail may still run from an earlier call, whose end the
        // context's stream has joined; this call's work is queued behind it
        bool old = false;
        for (int g = 0; g < G; ++g) old = old || c->ggexec_rem[g];
        if (old) HIPCHK(hipStreamSynchronize(c->stream));
        for (int g = 0; g < G; ++g) drop_one(c->ggraph_rem[g], c->ggexec_rem[g]);
      }
      for (int g = 0; g < G; ++g)
        if (!c->ggexec_rem[g] && (rc = build_graph(c, (int)left, &c->ggraph_rem[g], &c->ggexec_rem[g], g, G)))
          return rc;
      c->rem_steps = (int)left;
      for (int g = 0; g < G; ++g) HIPCHK(hipGraphLaunch(c->ggexec_rem[g], c->gstream[g]));
    }
  }
  return TTSH_OK;
}

// ttsh_step with the instances in c->groups groups: the group streams wait
// for the work queued on the context's stream, replay their graphs chunk by
// chunk (each group its own), and the context's stream waits for all of
// them, so that the call is ordered like a single-stream one.  The join is
// queued on every path after the fork, so that whatever was launched on a
// group stream before an error is still ordered ahead of later work.
int step_groups(ttsh_ctx* c, int64_t nsteps) {
  if (nsteps == 0) return TTSH_OK;
  int rc = ensure_groups(c);
  if (rc) return rc;
  const int G = c->groups;
  HIPCHK(hipEventRecord(c->gfork, c->stream));
  for (int g = 0; g < G; ++g) HIPCHK(hipStreamWaitEvent(c->gstream[g], c->gfork, 0));
  rc = step_groups_body(c, nsteps, G);
  for (int g = 0; g < G; ++g) {
    const hipError_t e1 = hipEventRecord(c->gjoin[g], c->gstream[g]);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(c->stream, c->gjoin[g], 0) : e1;
    if (e2 != hipSuccess && rc == TTSH_OK) rc = fail(TTSH_EHIP, std::string("stream join: ") + hipGetErrorString(e2));
  }
  return rc;
}

// ---- continuation (reseed) ----------------------------------------------------
int reseed_check(ttsh_ctx* c, int n, const int* dst, const int* src) {
  if (!c) return fail(TTSH_EINVAL, "null context");
  if (n < 0 || (n > 0 && (!dst || !src))) return fail(TTSH_EINVAL, "bad reseed lists");
  for (int q = 0; q < n; ++q) {
    if (dst[q] < 0 || dst[q] >= c->n_inst || src[q] < 0 || src[q] >= c->n_inst)
      return fail(TTSH_EINVAL, "reseed index out of range");
    for (int r = 0; r < q; ++r)
      if (dst[r] == dst[q]) return fail(TTSH_EINVAL, "duplicate reseed destination");
  }
  return TTSH_OK;
}

// compact FP64 spectra of every destination, back to back: the scratch a
// reseed needs to read all sources before any destination is written
size_t reseed_scratch_elems(const ttsh_ctx* c, int n, const int* dst) {
  size_t e = 0;
  for (int q = 0; q < n; ++q) {
    const int Nd = c->N[dst[q]];
    e += (size_t)2 * (Nd / 4 + 1) * (Nd / 2 + 2);
  }
  return e;
}

// the noise added at a reseed: caller fields (`fields`, [2][N][N] per
// destination, back to back) or, if fields is null and amp != 0, the
// device's Philox stream
struct Noise {
  const double* fields = nullptr;
  int where = TTSH_HOST;
  double amp = 0.0;
  uint64_t seed = 0;
};

// state[dst[q]] <- resample(state[src[q]]) + P DFT(noise_q); `tmp` holds
// reseed_scratch_elems complex doubles.  Asynchronous, except that host noise
// fields are staged through scr1 one destination at a time.
int reseed_impl(ttsh_ctx* c, int n, const int* dst, const int* src, const Noise& nz, C2<double>* tmp) {
  // gather every resampled source first
  size_t off = 0;
  for (int q = 0; q < n; ++q) {
    auto [cs, js] = c->loc[src[q]];
    SizeClass& ks = c->cls[cs];
    const int Nd = c->N[dst[q]];
    const size_t cnt = (size_t)2 * (Nd / 4 + 1) * (Nd / 2 + 2);
    if (c->prec == 32)
      hipLaunchKernelGGL(k_resample<float>, dim3(nblk(cnt)), dim3(kB), 0, c->stream,
                         at<const C2<float>>(ks.st, ks.sSt(), sizeof(C2<float>), js), ks.N, tmp + off, Nd);
    else
      hipLaunchKernelGGL(k_resample<double>, dim3(nblk(cnt)), dim3(kB), 0, c->stream,
                         at<const C2<double>>(ks.st, ks.sSt(), sizeof(C2<double>), js), ks.N, tmp + off, Nd);
    HIPCHK(hipGetLastError());
    off += cnt;
  }
  off = 0;
  size_t noff = 0;
  for (int q = 0; q < n; ++q) {
    const int Nd = c->N[dst[q]];
    int rc;
    const void* Z = nullptr;
    if (nz.fields) {
      const void* dev = nullptr;
      if ((rc = stage_in(c, nz.fields + noff, sizeof(double) * 2 * Nd * Nd, nz.where, &dev))) return rc;
      if ((rc = field_to_spectrum(c, Nd, (const double*)dev))) return rc;
      noff += (size_t)2 * Nd * Nd;
      Z = c->scr0;
    } else if (nz.amp != 0.0) {
      hipLaunchKernelGGL(k_philox_noise, dim3(nblk((size_t)Nd * Nd)), dim3(kB), 0, c->stream, (C2<double>*)c->scr0, Nd,
                         (uint32_t)dst[q], (uint32_t)(nz.seed & 0xFFFFFFFFu), (uint32_t)(nz.seed >> 32), nz.amp);
      HIPCHK(hipGetLastError());
      HIPCHK(size_ops(Nd)->fft2(c->scr0, 1, -1, 1, c->tw64[Nd], c->stream));
      Z = c->scr0;
    }
    if ((rc = pack_into_state(c, dst[q], Z, tmp + off))) return rc;
    if ((rc = refresh_x(c, dst[q]))) return rc;
    off += (size_t)2 * (Nd / 4 + 1) * (Nd / 2 + 2);
    if (nz.fields && nz.where == TTSH_HOST) HIPCHK(hipStreamSynchronize(c->stream));
  }
  return TTSH_OK;
}

void free_ctx(ttsh_ctx* c) {
  if (!c) return;
  drop_graph(c);
  for (auto& k : c->cls) {
    for (void* p : {k.X, k.Y, k.st, k.K, k.rowsum, (void*)k.dk, k.tw, k.st2, k.fst, (void*)k.s1st})
      if (p) hipFree(p);
  }
  for (auto& kv : c->tw64) hipFree(kv.second);
  for (auto& kv : c->tw32) hipFree(kv.second);
  if (c->scr0) hipFree(c->scr0);
  if (c->scr1) hipFree(c->scr1);
  if (c->dnorm) hipFree(c->dnorm);
  if (c->dflags) hipFree(c->dflags);
  for (void* p : {c->pb0, c->pb1, (void*)c->pnorm, c->lyq, (void*)c->psdf})
    if (p) hipFree(p);
  if (c->cap) hipStreamDestroy(c->cap);
  for (int g = 0; g < kMaxGroups; ++g) {
    if (c->gstream[g]) hipStreamDestroy(c->gstream[g]);
    if (c->gjoin[g]) hipEventDestroy(c->gjoin[g]);
  }
  if (c->gfork) hipEventDestroy(c->gfork);
  delete c;
}

}  // namespace

extern "C" {

const char* ttsh_last_error(void) { return g_err.c_str(); }

int ttsh_create(ttsh_ctx** out, int n_inst, const int* N, const double* L, const ttsh_params* p,
                int precision, void* stream) {
  if (!out || !N || !L || !p) return fail(TTSH_EINVAL, "null argument");
  *out = nullptr;
  if (n_inst < 1 || n_inst > 4096) return fail(TTSH_EINVAL, "n_inst must be in 1..4096");
  if (precision != TTSH_FP32 && precision != TTSH_FP64 && precision != TTSH_FP32_STATE64)
    return fail(TTSH_EINVAL, "precision must be TTSH_FP32, TTSH_FP64 or TTSH_FP32_STATE64");
  if (p->scheme < TTSH_IFEULER || p->scheme > TTSH_ETDRK4) return fail(TTSH_EINVAL, "unknown scheme");
  const double coef[] = {p->alpha, p->beta, p->gamma0, p->gamma2, p->lambda0, p->lambda1, p->gamma_v, p->gamma_w, p->dt};
  for (double v : coef)
    if (!std::isfinite(v)) return fail(TTSH_EINVAL, "non-finite coefficient");
  if (!(p->dt > 0)) return fail(TTSH_EINVAL, "dt must be > 0");
  for (int i = 0; i < n_inst; ++i) {
    if (!size_ops(N[i]))
      return fail(TTSH_EUNSUPPORTED, "N must be one of 64, 128, 256, 512, 1024, 2048, 4096, 8192");
    if (N[i] > kMaxBlockN && !big_ops(N[i], precision))
      return fail(TTSH_EUNSUPPORTED, "8192 points per side need FP32 transforms (TTSH_FP32 or TTSH_FP32_STATE64)");
    if (!(L[i] > 0) || !std::isfinite(L[i])) return fail(TTSH_EINVAL, "L must be > 0");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(TTSH_EHIP, "no HIP device available");

  ttsh_ctx* c = new ttsh_ctx();
  c->n_inst = n_inst;
  c->N.assign(N, N + n_inst);
  c->L.assign(L, L + n_inst);
  c->p = *p;
  c->prec = precision;
  c->gw = p->gamma_w != 0.0;
  c->stream = (hipStream_t)stream;
  c->loc.resize(n_inst);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(TTSH_EHIP, "hipGetDevice failed");
  }
  if (int rc = resolve_scratch(c->device)) {
    delete c;
    return rc;
  }
  auto bail = [&](int rc) {
    free_ctx(c);
    return rc;
  };

  std::vector<int> sizes(N, N + n_inst);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  const size_t er = elem_real(precision), es = elem_state(precision);
  for (int Nc : sizes) {
    SizeClass k;
    k.N = Nc;
    for (int i = 0; i < n_inst; ++i)
      if (N[i] == Nc) {
        c->loc[i] = {(int)c->cls.size(), (int)k.ids.size()};
        k.ids.push_back(i);
      }
    const size_t n = k.ids.size();
    struct Alloc {
      void** p;
      size_t bytes;
    };
    std::vector<Alloc> al = {{&k.X, n * k.sX() * 2 * er},       {&k.Y, n * k.sY(c->gw) * 2 * er},
                             {&k.st, n * k.sSt() * es},         {&k.K, n * k.sK() * er},
                             {&k.rowsum, n * 2 * (size_t)Nc * er}, {(void**)&k.dk, n * sizeof(double)}};
    if (const int slots = etd_slots(p->scheme)) {
      al.push_back({&k.st2, n * k.sSt() * es});
      al.push_back({&k.fst, n * slots * k.sF(c->gw) * 2 * er});
      al.push_back({(void**)&k.s1st, n * 2 * slots * sizeof(double)});
    }
    for (auto& a : al) {
      if (hipMalloc(a.p, a.bytes) != hipSuccess) {
        c->cls.push_back(k);
        return bail(fail(TTSH_ENOMEM, "device allocation failed"));
      }
      if (hipMemset(*a.p, 0, a.bytes) != hipSuccess) {
        c->cls.push_back(k);
        return bail(fail(TTSH_EHIP, "hipMemset failed"));
      }
    }
    std::vector<double> dks;
    for (int id : k.ids) dks.push_back(2.0 * M_PI / L[id]);
    c->cls.push_back(k);
    SizeClass& kk = c->cls.back();
    if (hipMemcpy(kk.dk, dks.data(), dks.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(TTSH_EHIP, "wavenumber upload failed"));
    int rc = make_twiddles(Nc, precision == 64, &kk.tw);
    if (rc) return bail(rc);
    void* t64 = nullptr;
    rc = make_twiddles(Nc, true, &t64);
    if (rc) return bail(rc);
    c->tw64[Nc] = t64;
  }
  const int Nmax = sizes.back();
  if (hipMalloc(&c->scr0, sizeof(double) * 2 * Nmax * Nmax) != hipSuccess ||
      hipMalloc(&c->scr1, sizeof(double) * 2 * Nmax * Nmax) != hipSuccess ||
      hipMalloc((void**)&c->dnorm, sizeof(double) * 5 * ((size_t)n_inst + kNormBlocks)) != hipSuccess ||
      hipMalloc((void**)&c->dflags, sizeof(int) * n_inst) != hipSuccess)
    return bail(fail(TTSH_ENOMEM, "scratch allocation failed"));
  if (hipMemset(c->dflags, 0, sizeof(int) * n_inst) != hipSuccess) return bail(fail(TTSH_EHIP, "hipMemset failed"));
  {
    int off = 0;
    for (auto& k : c->cls) {
      k.gflags = c->dflags + off;
      off += (int)k.ids.size();
    }
  }
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(TTSH_EHIP, "stream creation failed"));
  if (sizes.size() > (size_t)kMaxClasses) return bail(fail(TTSH_EUNSUPPORTED, "too many grid sizes"));
  int rc = choose_bs(c);
  if (rc) return bail(rc);
  *out = c;
  return TTSH_OK;
}

void ttsh_destroy(ttsh_ctx* c) {
  if (!c) return;
  hipStreamSynchronize(c->stream);
  free_ctx(c);
}

int ttsh_set_option(ttsh_ctx* c, int key, int64_t value) {
  if (!c) return fail(TTSH_EINVAL, "null context");
  switch (key) {
    case TTSH_OPT_GRAPH_STEPS:
      if (value < 0 || value > 100000) return fail(TTSH_EINVAL, "graph steps out of range");
      c->graph_steps = (int)value;
      break;
    case TTSH_OPT_BLOCK: {
      if (value != 0 && !bs_valid(c, (int)value)) return fail(TTSH_EINVAL, "workgroup size must be 0, 64, 128 or 256 with 8 x size >= N");
      c->opt_bs = (int)value;
      int rc = choose_bs(c);
      if (rc) return rc;
      break;
    }
    case TTSH_OPT_SPLIT:
      if (value < 0 || value > 3) return fail(TTSH_EINVAL, "split must be 0..3");
      c->split_row = (int)(value & 1);
      c->split_col = (int)((value >> 1) & 1);
      drop_graph(c);
      break;
    case TTSH_OPT_GUARD:
      c->guard = value != 0;
      break;
    case TTSH_OPT_GUARD_EVERY:
      if (value < 0 || value > 1000000) return fail(TTSH_EINVAL, "guard interval out of range");
      c->guard_every = (int)value;
      break;
    case TTSH_OPT_GROUPS:
      if (value < 1 || value > kMaxGroups) return fail(TTSH_EINVAL, "groups must be 1 or 2");
      if (value > c->n_inst) return fail(TTSH_EINVAL, "two groups need at least two instances");
      c->groups = (int)value;
      break;
    default:
      return fail(TTSH_EINVAL, "unknown option");
  }
  drop_graph(c);
  return TTSH_OK;
}

int ttsh_set_mask(ttsh_ctx* c, int inst, const double* K, int where) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const size_t n = (size_t)k.N * k.N;
  const void* dev = nullptr;
  if ((rc = stage_in(c, K, n * sizeof(double), where, &dev))) return rc;
  if (c->prec == 64)
    hipLaunchKernelGGL((k_convert<double, double>), dim3(nblk(n)), dim3(kB), 0, c->stream,
                       (const double*)dev, at<double>(k.K, k.sK(), 8, j), n);
  else
    hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(n)), dim3(kB), 0, c->stream,
                       (const double*)dev, at<float>(k.K, k.sK(), 4, j), n);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_get_mask(ttsh_ctx* c, int inst, double* K, int where) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!K) return fail(TTSH_EINVAL, "null output");
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const size_t n = (size_t)k.N * k.N;
  double* dst = where == TTSH_DEVICE ? K : (double*)c->scr1;
  if (c->prec == 64)
    hipLaunchKernelGGL((k_convert<double, double>), dim3(nblk(n)), dim3(kB), 0, c->stream,
                       at<const double>(k.K, k.sK(), 8, j), dst, n);
  else
    hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(n)), dim3(kB), 0, c->stream,
                       at<const float>(k.K, k.sK(), 4, j), dst, n);
  HIPCHK(hipGetLastError());
  if (where != TTSH_DEVICE) HIPCHK(hipMemcpyAsync(K, dst, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_mask_tanh(ttsh_ctx* c, int inst, int n_circ, const double* cx, const double* cy,
                   const double* R, double xi) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (n_circ < 1 || n_circ > 8 || !cx || !cy || !R) return fail(TTSH_EINVAL, "need 1..8 circles");
  if (!(xi > 0) || !std::isfinite(xi)) return fail(TTSH_EINVAL, "xi must be > 0");
  Circles cc{};
  cc.n = n_circ;
  for (int q = 0; q < n_circ; ++q) {
    if (!std::isfinite(cx[q]) || !std::isfinite(cy[q]) || !std::isfinite(R[q])) return fail(TTSH_EINVAL, "non-finite circle");
    cc.cx[q] = cx[q];
    cc.cy[q] = cy[q];
    cc.R[q] = R[q];
  }
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int n = k.N * k.N;
  const double dx = c->L[inst] / k.N;
  if (c->prec == 64)
    hipLaunchKernelGGL(k_mask_tanh<double>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       at<double>(k.K, k.sK(), 8, j), k.N, dx, cc, xi);
  else
    hipLaunchKernelGGL(k_mask_tanh<float>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       at<float>(k.K, k.sK(), 4, j), k.N, dx, cc, xi);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_mask_from_binary(ttsh_ctx* c, int inst, const uint8_t* Kn, int where) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, n = N * N;
  const void* dev = nullptr;
  if ((rc = stage_in(c, Kn, (size_t)n, where, &dev))) return rc;
  hipLaunchKernelGGL(k_binary_to_c, dim3(nblk(n)), dim3(kB), 0, c->stream, (const uint8_t*)dev,
                     (C2<double>*)c->scr0, n);
  HIPCHK(hipGetLastError());
  HIPCHK(size_ops(N)->fft2(c->scr0, 1, -1, 1, c->tw64[N], c->stream));
  hipLaunchKernelGGL(k_lowpass, dim3(nblk(n)), dim3(kB), 0, c->stream, (C2<double>*)c->scr0, N,
                     (N / 8) * (N / 8), 1.0 / ((double)N * N));
  HIPCHK(hipGetLastError());
  HIPCHK(size_ops(N)->fft2(c->scr0, 1, +1, 1, c->tw64[N], c->stream));
  if (c->prec == 64)
    hipLaunchKernelGGL(k_square_real<double>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       (const C2<double>*)c->scr0, at<double>(k.K, k.sK(), 8, j), n);
  else
    hipLaunchKernelGGL(k_square_real<float>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       (const C2<double>*)c->scr0, at<float>(k.K, k.sK(), 4, j), n);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_set_field(ttsh_ctx* c, int inst, const double* v, int where) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  const int N = c->N[inst];
  const void* dev = nullptr;
  if ((rc = stage_in(c, v, sizeof(double) * 2 * N * N, where, &dev))) return rc;
  if ((rc = field_to_spectrum(c, N, (const double*)dev))) return rc;
  // the k = 0 entry of the transform is the sum of every input value, so it is
  // finite exactly when the input holds no NaN or Inf (barring overflow of the
  // sum, which is refused too); checked before the state is written
  double z0[2];
  HIPCHK(hipMemcpyAsync(z0, c->scr0, sizeof(z0), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (!std::isfinite(z0[0]) || !std::isfinite(z0[1]))
    return fail(TTSH_ENONFINITE, "non-finite value in the input field (state left unchanged)");
  if ((rc = pack_into_state(c, inst, c->scr0, nullptr))) return rc;
  if ((rc = refresh_x(c, inst))) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_get_field(ttsh_ctx* c, int inst, double* v, double* omega, int where) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!v) return fail(TTSH_EINVAL, "null output");
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, n = N * N;
  const double dk = 2.0 * M_PI / c->L[inst];
  for (int what = 0; what < (omega ? 2 : 1); ++what) {
    if (c->prec == 32)
      hipLaunchKernelGGL(k_state_to_full<float>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                         at<const C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), (C2<double>*)c->scr0, N, dk, what);
    else
      hipLaunchKernelGGL(k_state_to_full<double>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                         at<const C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), (C2<double>*)c->scr0, N, dk, what);
    HIPCHK(hipGetLastError());
    HIPCHK(size_ops(N)->fft2(c->scr0, 1, +1, 1, c->tw64[N], c->stream));
    double* out = what == 0 ? v : omega;
    double* dst = where == TTSH_DEVICE ? out : (double*)c->scr1;
    if (what == 0)
      hipLaunchKernelGGL(k_unpack_xy, dim3(nblk(n)), dim3(kB), 0, c->stream, (const C2<double>*)c->scr0, dst, n);
    else
      hipLaunchKernelGGL(k_real_part, dim3(nblk(n)), dim3(kB), 0, c->stream, (const C2<double>*)c->scr0, dst, n);
    HIPCHK(hipGetLastError());
    if (where != TTSH_DEVICE)
      HIPCHK(hipMemcpyAsync(out, dst, sizeof(double) * (what == 0 ? 2 : 1) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return TTSH_OK;
}

int ttsh_get_field_coarse(ttsh_ctx* c, int inst, int Nc, float* out, int64_t pix_stride) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!out) return fail(TTSH_EINVAL, "null output");
  if (pix_stride < 2) return fail(TTSH_EINVAL, "pix_stride must be >= 2");
  if (!size_ops(Nc)) return fail(TTSH_EUNSUPPORTED, "Nc must be one of 64, 128, 256, 512, 1024, 2048, 4096, 8192");
  if (Nc > max_N(c)) return fail(TTSH_EINVAL, "Nc larger than the context's largest grid");
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, n = Nc * Nc;
  // compact FP64 spectrum at Nc in scr1, full spectrum in scr0 (both hold
  // max_N^2 complex values, enough for Nc <= max_N)
  const size_t ncomp = (size_t)2 * (Nc / 4 + 1) * (Nc / 2 + 2);
  C2<double>* comp = (C2<double>*)c->scr1;
  if (c->prec == 32)
    hipLaunchKernelGGL(k_resample<float>, dim3(nblk(ncomp)), dim3(kB), 0, c->stream,
                       at<const C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), N, comp, Nc);
  else
    hipLaunchKernelGGL(k_resample<double>, dim3(nblk(ncomp)), dim3(kB), 0, c->stream,
                       at<const C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), N, comp, Nc);
  hipLaunchKernelGGL(k_state_to_full<double>, dim3(nblk(n)), dim3(kB), 0, c->stream, comp,
                     (C2<double>*)c->scr0, Nc, 2.0 * M_PI / c->L[inst], 0);
  HIPCHK(hipGetLastError());
  const void* tw = nullptr;
  if ((rc = twiddles64(c, Nc, &tw))) return rc;
  HIPCHK(size_ops(Nc)->fft2(c->scr0, 1, +1, 1, tw, c->stream));
  hipLaunchKernelGGL(k_unpack_xy_strided, dim3(nblk(n)), dim3(kB), 0, c->stream, (const C2<double>*)c->scr0,
                     out, n, (long long)pix_stride);
  HIPCHK(hipGetLastError());
  return TTSH_OK;
}

int ttsh_set_field_coarse(ttsh_ctx* c, int inst, int Nc, const float* v, int64_t pix_stride) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!v) return fail(TTSH_EINVAL, "null input");
  if (pix_stride < 2) return fail(TTSH_EINVAL, "pix_stride must be >= 2");
  if (!size_ops(Nc)) return fail(TTSH_EUNSUPPORTED, "Nc must be one of 64, 128, 256, 512, 1024, 2048, 4096, 8192");
  if (Nc > max_N(c)) return fail(TTSH_EINVAL, "Nc larger than the context's largest grid");
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, n = Nc * Nc, Mc = Nc / 4;
  const void* tw = nullptr;
  if ((rc = twiddles64(c, Nc, &tw))) return rc;
  // spectrum at Nc (scr0) -> projected compact FP64 state at Nc (scr1) ->
  // resampled to N (scr0) -> stored precision
  hipLaunchKernelGGL(k_pack_xy_strided, dim3(nblk(n)), dim3(kB), 0, c->stream, v, (long long)pix_stride,
                     (C2<double>*)c->scr0, n);
  HIPCHK(hipGetLastError());
  HIPCHK(size_ops(Nc)->fft2(c->scr0, 1, -1, 1, tw, c->stream));
  const size_t nc = (size_t)(Mc + 1) * (2 * Mc + 2);
  hipLaunchKernelGGL(k_pack_state<double>, dim3(nblk(nc)), dim3(kB), 0, c->stream, (const C2<double>*)c->scr0,
                     (const C2<double>*)nullptr, (C2<double>*)c->scr1, Nc);
  const size_t ns = k.sSt();
  hipLaunchKernelGGL(k_resample<double>, dim3(nblk(ns)), dim3(kB), 0, c->stream, (const C2<double>*)c->scr1, Nc,
                     (C2<double>*)c->scr0, N);
  if (c->prec == 32)
    hipLaunchKernelGGL(k_convert_c<float>, dim3(nblk(ns)), dim3(kB), 0, c->stream, (const C2<double>*)c->scr0,
                       at<C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), ns);
  else
    hipLaunchKernelGGL(k_convert_c<double>, dim3(nblk(ns)), dim3(kB), 0, c->stream, (const C2<double>*)c->scr0,
                       at<C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), ns);
  HIPCHK(hipGetLastError());
  return refresh_x(c, inst);
}

int ttsh_project_coarse(ttsh_ctx* c, int N, float* v, int64_t pix_stride, int batch, double* norms) {
  if (!c) return fail(TTSH_EINVAL, "null context");
  if (!v) return fail(TTSH_EINVAL, "null field");
  if (pix_stride < 2) return fail(TTSH_EINVAL, "pix_stride must be >= 2");
  if (batch < 1) return fail(TTSH_EINVAL, "batch must be >= 1");
  if (!size_ops(N)) return fail(TTSH_EUNSUPPORTED, "N must be one of 64, 128, 256, 512, 1024, 2048, 4096, 8192");
  const size_t n = (size_t)batch * N * N;
  if (n > (size_t)INT32_MAX) return fail(TTSH_EINVAL, "batch too large");
  const size_t bytes = n * sizeof(C2<double>);
  if (bytes > c->pb_cap) {
    for (void** p : {&c->pb0, &c->pb1})
      if (*p) {
        hipFree(*p);
        *p = nullptr;
      }
    c->pb_cap = 0;
    if (hipMalloc(&c->pb0, bytes) != hipSuccess || hipMalloc(&c->pb1, bytes) != hipSuccess)
      return fail(TTSH_ENOMEM, "projection buffers");
    c->pb_cap = bytes;
  }
  if (norms && batch > c->pnorm_cap) {
    if (c->pnorm) hipFree(c->pnorm);
    c->pnorm = nullptr;
    c->pnorm_cap = 0;
    if (hipMalloc((void**)&c->pnorm, sizeof(double) * 2 * batch) != hipSuccess)
      return fail(TTSH_ENOMEM, "norm buffer");
    c->pnorm_cap = batch;
  }
  int rc;
  const void* tw = nullptr;
  if ((rc = twiddles64(c, N, &tw))) return rc;
  hipLaunchKernelGGL(k_pack_xy_strided, dim3(nblk(n)), dim3(kB), 0, c->stream, (const float*)v,
                     (long long)pix_stride, (C2<double>*)c->pb0, (int)n);
  HIPCHK(hipGetLastError());
  HIPCHK(size_ops(N)->fft2(c->pb0, batch, -1, 1, tw, c->stream));
  hipLaunchKernelGGL(k_project_full, dim3(nblk(n)), dim3(kB), 0, c->stream, (const C2<double>*)c->pb0,
                     (C2<double>*)c->pb1, N, (int)n);
  HIPCHK(hipGetLastError());
  if (norms) {
    hipLaunchKernelGGL(k_full_norms, dim3(batch), dim3(256), 0, c->stream, (const C2<double>*)c->pb1, N,
                       c->pnorm);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(size_ops(N)->fft2(c->pb1, batch, +1, 1, tw, c->stream));
  hipLaunchKernelGGL(k_unpack_xy_strided, dim3(nblk(n)), dim3(kB), 0, c->stream, (const C2<double>*)c->pb1, v,
                     (int)n, (long long)pix_stride);
  HIPCHK(hipGetLastError());
  if (norms) {
    HIPCHK(hipMemcpyAsync(norms, c->pnorm, sizeof(double) * 2 * batch, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return TTSH_OK;
}

// Order parameters into dnorm[0] (Psi, from the velocity) and dnorm[1] (Psi_2,
// from the vorticity), the first from_what of them skipped; the host receives
// dnorm[from_what..1] in out[0..].
static int order_impl(ttsh_ctx* c, int inst, double cx, double cy, double D, int from_what, double* out) {
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, n = N * N;
  const double L = c->L[inst], dk = 2.0 * M_PI / L, dx = L / N;
  for (int what = from_what; what < 2; ++what) {
    if (c->prec == 32)
      hipLaunchKernelGGL(k_state_to_full<float>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                         at<const C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), (C2<double>*)c->scr0, N, dk, what);
    else
      hipLaunchKernelGGL(k_state_to_full<double>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                         at<const C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), (C2<double>*)c->scr0, N, dk, what);
    HIPCHK(hipGetLastError());
    HIPCHK(size_ops(N)->fft2(c->scr0, 1, +1, 1, c->tw64[N], c->stream));
    // partials in scr1 (free here; at least 64^2 complex doubles, 4 per workgroup needed)
    const int nb = order_blocks(N);
    double* part = (double*)c->scr1;
    if (what == 0) {
      hipLaunchKernelGGL(k_order_psi, dim3(nb), dim3(1024), 0, c->stream, (const C2<double>*)c->scr0, N, dx, cx, cy,
                         part);
      hipLaunchKernelGGL(k_order_psi_final, dim3(1), dim3(256), 0, c->stream, (const double*)part, nb, c->dnorm);
    } else {
      hipLaunchKernelGGL(k_order_psi2, dim3(nb), dim3(1024), 0, c->stream, (const C2<double>*)c->scr0, N, dx, cx,
                         cy, D, part);
      hipLaunchKernelGGL(k_order_psi2_final, dim3(1), dim3(256), 0, c->stream, (const C2<double>*)c->scr0,
                         (const double*)part, nb, c->dnorm);
    }
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipMemcpyAsync(out, c->dnorm + from_what, (2 - from_what) * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_order(ttsh_ctx* c, int inst, double cx, double cy, double* out) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!out) return fail(TTSH_EINVAL, "null output");
  return order_impl(c, inst, cx, cy, 0.0, 0, out);
}

int ttsh_order_dumbbell(ttsh_ctx* c, int inst, double cx, double cy, double D, double* psi2) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!psi2) return fail(TTSH_EINVAL, "null output");
  if (!(D > 0.0) || !std::isfinite(D)) return fail(TTSH_EINVAL, "D must be positive and finite");
  return order_impl(c, inst, cx, cy, D, 1, psi2);
}

int ttsh_lyap_qr(ttsh_ctx* c, int base, const int* pert, int p, double eps, double* log_r) {
  int rc = check_inst(c, base);
  if (rc) return rc;
  if (!pert || !log_r) return fail(TTSH_EINVAL, "null argument");
  if (p < 1 || p > kMaxLyap) return fail(TTSH_EINVAL, "p must be 1..16");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(TTSH_EINVAL, "eps must be positive and finite");
  auto [ci, jb] = c->loc[base];
  SizeClass& k = c->cls[ci];
  const size_t es = c->prec == 32 ? sizeof(C2<float>) : sizeof(C2<double>);
  void* st[kMaxLyap];
  for (int v = 0; v < p; ++v) {
    if ((rc = check_inst(c, pert[v]))) return rc;
    if (pert[v] == base) return fail(TTSH_EINVAL, "a perturbed instance is the base instance");
    for (int u = 0; u < v; ++u)
      if (pert[u] == pert[v]) return fail(TTSH_EINVAL, "perturbed instances must be distinct");
    if (c->loc[pert[v]].first != ci) return fail(TTSH_EINVAL, "perturbed instances must have the base's grid size");
    st[v] = (char*)k.st + (size_t)c->loc[pert[v]].second * k.sSt() * es;
  }
  const int N = k.N;
  const size_t n = k.sSt();  // complex entries per state, both components
  const int nb = (int)((n + 1023) / 1024);
  // scratch: logs [kMaxLyap], two partial buffers [nb], then the p vectors
  const size_t head = sizeof(double) * (kMaxLyap + 2 * (size_t)nb);
  const size_t head_al = (head + 255) / 256 * 256;
  const size_t bytes = head_al + (size_t)p * n * sizeof(C2<double>);
  if (bytes > c->lyq_cap) {
    if (c->lyq) hipFree(c->lyq);
    c->lyq = nullptr;
    c->lyq_cap = 0;
    if (hipMalloc(&c->lyq, bytes) != hipSuccess) return fail(TTSH_ENOMEM, "Lyapunov vectors");
    c->lyq_cap = bytes;
  }
  double* dlogs = (double*)c->lyq;
  double* pa = dlogs + kMaxLyap;
  double* pb = pa + nb;
  C2<double>* q = (C2<double>*)((char*)c->lyq + head_al);
  for (int v = 0; v < p; ++v) {
    C2<double>* qv = q + (size_t)v * n;
    const C2<double>* qd = v > 0 ? q : nullptr;  // first projection onto q_0, or the norm
    if (c->prec == 32)
      hipLaunchKernelGGL(k_lyap_init<float>, dim3(nb), dim3(1024), 0, c->stream,
                         at<const C2<float>>(k.st, k.sSt(), sizeof(C2<float>), jb), (const C2<float>*)st[v], N, eps,
                         qv, qd, pa);
    else
      hipLaunchKernelGGL(k_lyap_init<double>, dim3(nb), dim3(1024), 0, c->stream,
                         at<const C2<double>>(k.st, k.sSt(), sizeof(C2<double>), jb), (const C2<double>*)st[v], N,
                         eps, qv, qd, pa);
    for (int u = 0; u < v; ++u) {
      const C2<double>* nxt = u + 1 < v ? q + (size_t)(u + 1) * n : nullptr;
      hipLaunchKernelGGL(k_lyap_axpy, dim3(nb), dim3(1024), 0, c->stream, qv, (const C2<double>*)(q + (size_t)u * n),
                         (const double*)pa, nb, N, nxt, pb);
      std::swap(pa, pb);
    }
    if (c->prec == 32)
      hipLaunchKernelGGL(k_lyap_scale<float>, dim3(nb), dim3(1024), 0, c->stream,
                         at<const C2<float>>(k.st, k.sSt(), sizeof(C2<float>), jb), (C2<float>*)st[v], qv,
                         (const double*)pa, nb, N, eps, dlogs + v);
    else
      hipLaunchKernelGGL(k_lyap_scale<double>, dim3(nb), dim3(1024), 0, c->stream,
                         at<const C2<double>>(k.st, k.sSt(), sizeof(C2<double>), jb), (C2<double>*)st[v], qv,
                         (const double*)pa, nb, N, eps, dlogs + v);
    HIPCHK(hipGetLastError());
  }
  for (int v = 0; v < p; ++v)
    if ((rc = refresh_x(c, pert[v]))) return rc;
  HIPCHK(hipMemcpyAsync(log_r, dlogs, p * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int v = 0; v < p; ++v)
    if (!std::isfinite(log_r[v]))
      return fail(TTSH_ENONFINITE, "perturbation " + std::to_string(v) + " has no component left (degenerate or non-finite)");
  return TTSH_OK;
}

int ttsh_psd_accumulate(ttsh_ctx* c, int inst, int nf, const double* freqs, double t, void* acc) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!freqs || !acc) return fail(TTSH_EINVAL, "null argument");
  if (nf < 1 || nf > kMaxPsdFreqs) return fail(TTSH_EINVAL, "nf must be 1..4096");
  if (!std::isfinite(t)) return fail(TTSH_EINVAL, "t must be finite");
  for (int j = 0; j < nf; ++j)
    if (!std::isfinite(freqs[j])) return fail(TTSH_EINVAL, "frequencies must be finite");
  if (!c->psdf && hipMalloc((void**)&c->psdf, sizeof(double) * 2 * kMaxPsdFreqs) != hipSuccess)
    return fail(TTSH_ENOMEM, "PSD frequencies");
  if (c->psd_freqs.size() != (size_t)nf || !std::equal(freqs, freqs + nf, c->psd_freqs.begin())) {
    HIPCHK(hipStreamSynchronize(c->stream));  // earlier launches may still read psdf
    HIPCHK(hipMemcpy(c->psdf, freqs, sizeof(double) * nf, hipMemcpyHostToDevice));
    c->psd_freqs.assign(freqs, freqs + nf);
  }
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, M = N / 4;
  const int nm = (M + 1) * (2 * M + 2);
  const double dk = 2.0 * M_PI / c->L[inst];
  const dim3 grid((nm + 255) / 256, (nf + 255) / 256);
  if (c->prec == 32)
    hipLaunchKernelGGL(k_psd_acc<float>, grid, dim3(256), 0, c->stream,
                       at<const C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), N, dk, c->psdf, nf, t,
                       (C2<double>*)acc);
  else
    hipLaunchKernelGGL(k_psd_acc<double>, grid, dim3(256), 0, c->stream,
                       at<const C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), N, dk, c->psdf, nf, t,
                       (C2<double>*)acc);
  HIPCHK(hipGetLastError());
  return TTSH_OK;
}

int ttsh_psd_finish(ttsh_ctx* c, int N, int nf, const void* acc, double* S) {
  if (!c) return fail(TTSH_EINVAL, "null context");
  if (!acc || !S) return fail(TTSH_EINVAL, "null argument");
  if (!size_ops(N)) return fail(TTSH_EUNSUPPORTED, "N must be one of 64, 128, 256, 512, 1024, 2048, 4096, 8192");
  if (nf < 1 || nf > kMaxPsdFreqs) return fail(TTSH_EINVAL, "nf must be 1..4096");
  if (!c->psdf && hipMalloc((void**)&c->psdf, sizeof(double) * 2 * kMaxPsdFreqs) != hipSuccess)
    return fail(TTSH_ENOMEM, "PSD frequencies");
  double* dS = c->psdf + kMaxPsdFreqs;
  hipLaunchKernelGGL(k_psd_finish, dim3(nf), dim3(1024), 0, c->stream, (const C2<double>*)acc, N, dS);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(S, dS, sizeof(double) * nf, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_vortices(ttsh_ctx* c, int inst, double kmax, double vmin, int* out) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!out) return fail(TTSH_EINVAL, "null output");
  if (!(vmin >= 0.0)) return fail(TTSH_EINVAL, "vmin must be >= 0");
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, n = N * N;
  const double dk = 2.0 * M_PI / c->L[inst];
  if (c->prec == 32)
    hipLaunchKernelGGL(k_state_to_full<float>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       at<const C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), (C2<double>*)c->scr0, N, dk, 0);
  else
    hipLaunchKernelGGL(k_state_to_full<double>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       at<const C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), (C2<double>*)c->scr0, N, dk, 0);
  HIPCHK(hipGetLastError());
  HIPCHK(size_ops(N)->fft2(c->scr0, 1, +1, 1, c->tw64[N], c->stream));
  int* dcount = reinterpret_cast<int*>(c->dnorm);  // [2], inside the norms scratch
  const int nb = order_blocks(N);
  int* part = (int*)c->scr1;  // per-workgroup partials (scr1 is free here)
  if (c->prec == 64)
    hipLaunchKernelGGL(k_vortex_count<double>, dim3(nb), dim3(1024), 0, c->stream, (const C2<double>*)c->scr0,
                       at<const double>(k.K, k.sK(), sizeof(double), j), N, kmax, vmin, part);
  else
    hipLaunchKernelGGL(k_vortex_count<float>, dim3(nb), dim3(1024), 0, c->stream, (const C2<double>*)c->scr0,
                       at<const float>(k.K, k.sK(), sizeof(float), j), N, kmax, vmin, part);
  hipLaunchKernelGGL(k_vortex_final, dim3(1), dim3(256), 0, c->stream, (const int*)part, nb, dcount);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(out, dcount, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_set_state(ttsh_ctx* c, int inst, const double* vhat, int where) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, M = N / 4;
  const size_t nabi = (size_t)2 * (2 * M + 1) * (M + 1);
  const void* dev = nullptr;
  if ((rc = stage_in(c, vhat, nabi * 2 * sizeof(double), where, &dev))) return rc;
  const size_t n = k.sSt();
  if (c->prec == 32)
    hipLaunchKernelGGL(k_abi_to_state<float>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       (const C2<double>*)dev, at<C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), N);
  else
    hipLaunchKernelGGL(k_abi_to_state<double>, dim3(nblk(n)), dim3(kB), 0, c->stream,
                       (const C2<double>*)dev, at<C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), N);
  HIPCHK(hipGetLastError());
  if ((rc = refresh_x(c, inst))) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_get_state(ttsh_ctx* c, int inst, double* vhat, int where) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!vhat) return fail(TTSH_EINVAL, "null output");
  auto [ci, j] = c->loc[inst];
  SizeClass& k = c->cls[ci];
  const int N = k.N, M = N / 4;
  const size_t nabi = (size_t)2 * (2 * M + 1) * (M + 1);
  C2<double>* dst = where == TTSH_DEVICE ? (C2<double>*)vhat : (C2<double>*)c->scr1;
  if (c->prec == 32)
    hipLaunchKernelGGL(k_state_to_abi<float>, dim3(nblk(nabi)), dim3(kB), 0, c->stream,
                       at<const C2<float>>(k.st, k.sSt(), sizeof(C2<float>), j), dst, N);
  else
    hipLaunchKernelGGL(k_state_to_abi<double>, dim3(nblk(nabi)), dim3(kB), 0, c->stream,
                       at<const C2<double>>(k.st, k.sSt(), sizeof(C2<double>), j), dst, N);
  HIPCHK(hipGetLastError());
  if (where != TTSH_DEVICE)
    HIPCHK(hipMemcpyAsync(vhat, dst, nabi * sizeof(C2<double>), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return TTSH_OK;
}

int ttsh_step(ttsh_ctx* c, int64_t nsteps) {
  if (!c) return fail(TTSH_EINVAL, "null context");
  if (nsteps < 0) return fail(TTSH_EINVAL, "nsteps must be >= 0");
  if (c->groups > 1) return step_groups(c, nsteps);
  if (c->graph_steps <= 0) return enqueue_steps(c, nsteps, c->stream);
  int rc;
  int64_t left = nsteps;
  if (left >= c->graph_steps) {
    if (!c->gexec && (rc = build_graph(c, c->graph_steps, &c->graph, &c->gexec))) return rc;
    while (left >= c->graph_steps) {
      HIPCHK(hipGraphLaunch(c->gexec, c->stream));
      left -= c->graph_steps;
    }
  }
  if (left > 0) {
    // the tail shorter than a chunk replays a graph of its own length, kept
    // until a call ends with a different tail
    if (c->gexec_rem && c->rem_steps != (int)left) {
      // the old tail may still run from the previous call (stream order): wait
      HIPCHK(hipStreamSynchronize(c->stream));
      drop_one(c->graph_rem, c->gexec_rem);
      c->rem_steps = 0;
    }
    if (!c->gexec_rem) {
      if ((rc = build_graph(c, (int)left, &c->graph_rem, &c->gexec_rem))) return rc;
      c->rem_steps = (int)left;
    }
    HIPCHK(hipGraphLaunch(c->gexec_rem, c->stream));
  }
  return TTSH_OK;
}

int ttsh_reseed(ttsh_ctx* c, int n, const int* dst, const int* src, double noise_amp, uint64_t seed) {
  int rc = reseed_check(c, n, dst, src);
  if (rc) return rc;
  if (!std::isfinite(noise_amp)) return fail(TTSH_EINVAL, "noise_amp must be finite");
  C2<double>* tmp = nullptr;
  const size_t need = reseed_scratch_elems(c, n, dst);
  if (need > 0 && hipMalloc((void**)&tmp, need * sizeof(C2<double>)) != hipSuccess)
    return fail(TTSH_ENOMEM, "reseed scratch allocation failed");
  Noise nz;
  nz.amp = noise_amp;
  nz.seed = seed;
  rc = reseed_impl(c, n, dst, src, nz, tmp);
  hipStreamSynchronize(c->stream);
  if (tmp) hipFree(tmp);
  return rc;
}

int ttsh_reseed_noalloc(ttsh_ctx* c, int n, const int* dst, const int* src, double noise_amp, uint64_t seed) {
  int rc = reseed_check(c, n, dst, src);
  if (rc) return rc;
  if (!std::isfinite(noise_amp)) return fail(TTSH_EINVAL, "noise_amp must be finite");
  const size_t need = reseed_scratch_elems(c, n, dst) * sizeof(C2<double>);
  if (need > kNoAllocScratchBytes)
    return fail(TTSH_EINVAL, "the destinations' spectra (" + std::to_string(need) +
                                 " bytes) exceed the 64 MiB scratch of ttsh_reseed_noalloc");
  void* ptr = g_scratch_ptr[c->device];
  if (!ptr) return fail(TTSH_EHIP, "scratch address not resolved for the context's device");
  Noise nz;
  nz.amp = noise_amp;
  nz.seed = seed;
  return reseed_impl(c, n, dst, src, nz, (C2<double>*)ptr);
}

int ttsh_reseed_field(ttsh_ctx* c, int n, const int* dst, const int* src, const double* noise, int where) {
  int rc = reseed_check(c, n, dst, src);
  if (rc) return rc;
  if (noise && where != TTSH_HOST && where != TTSH_DEVICE) return fail(TTSH_EINVAL, "bad where");
  C2<double>* tmp = nullptr;
  const size_t need = reseed_scratch_elems(c, n, dst);
  if (need > 0 && hipMalloc((void**)&tmp, need * sizeof(C2<double>)) != hipSuccess)
    return fail(TTSH_ENOMEM, "reseed scratch allocation failed");
  Noise nz;
  nz.fields = noise;
  nz.where = where;
  rc = reseed_impl(c, n, dst, src, nz, tmp);
  hipStreamSynchronize(c->stream);
  if (tmp) hipFree(tmp);
  return rc;
}

int ttsh_norms(ttsh_ctx* c, int inst, double out[4]) {
  int rc = check_inst(c, inst);
  if (rc) return rc;
  if (!out) return fail(TTSH_EINVAL, "null output");
  if ((rc = norms_into(c, inst, c->dnorm))) return rc;
  double h[5];
  HIPCHK(hipMemcpyAsync(h, c->dnorm, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int q = 0; q < 4; ++q) out[q] = h[q];
  if (h[4] != 0.0) return fail(TTSH_ENONFINITE, "non-finite value in the state");
  return TTSH_OK;
}

int ttsh_sync(ttsh_ctx* c) {
  if (!c) return fail(TTSH_EINVAL, "null context");
  HIPCHK(hipStreamSynchronize(c->stream));
  if (!c->guard) return TTSH_OK;
  // a last check of the current states on top of the ones the steps ran,
  // then read and clear the flags
  HIPCHK(launch_guard(c, c->stream));
  std::vector<int> h(c->n_inst);
  HIPCHK(hipMemcpyAsync(h.data(), c->dflags, sizeof(int) * h.size(), hipMemcpyDeviceToHost, c->stream));
  hipLaunchKernelGGL(k_fill_int, dim3(nblk(c->n_inst)), dim3(kB), 0, c->stream, c->dflags, c->n_inst, 0);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  int first = -1, bad = 0;
  for (auto& k : c->cls)
    for (size_t j = 0; j < k.ids.size(); ++j)
      if (h[(size_t)(k.gflags - c->dflags) + j]) {
        ++bad;
        if (first < 0 || k.ids[j] < first) first = k.ids[j];
      }
  if (bad) {
    return fail(TTSH_ENONFINITE, "non-finite value in instance " + std::to_string(first) +
                                     (bad > 1 ? " (and " + std::to_string(bad - 1) + " more)" : std::string()));
  }
  return TTSH_OK;
}

int ttsh_num_classes(ttsh_ctx* c, int* N_out) {
  if (!c) return fail(TTSH_EINVAL, "null context");
  if (N_out)
    for (size_t i = 0; i < c->cls.size(); ++i) N_out[i] = c->cls[i].N;
  return (int)c->cls.size();
}

int ttsh_pass_times(ttsh_ctx* c, int64_t nsteps, double* out) {
  if (!c || !out) return fail(TTSH_EINVAL, "null argument");
  if (nsteps < 1 || nsteps > 1000000) return fail(TTSH_EINVAL, "nsteps must be in 1..1e6");
  hipEvent_t ev[3];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  const MultiArgs r = multi_args(c, 1, -1), q = multi_args(c, 0, -1);
  int rc = TTSH_OK;
  // nsteps row passes back to back, then nsteps column passes: each pass
  // takes the same inputs every time (the row pass only reads the state's
  // mixed-domain fields; the column pass re-applies its update with the same
  // forcing), so the mean over the run is the launch duration without the
  // cost of an event pair per launch
  hipEventRecord(ev[0], c->stream);
  for (int64_t s = 0; s < nsteps && rc == TTSH_OK; ++s)
    if (launch_row(c, r, c->stream) != hipSuccess) rc = fail(TTSH_EHIP, "row pass launch failed");
  hipEventRecord(ev[1], c->stream);
  for (int64_t s = 0; s < nsteps && rc == TTSH_OK; ++s)
    if (launch_col(c, q, 0, c->stream) != hipSuccess) rc = fail(TTSH_EHIP, "column pass launch failed");
  hipEventRecord(ev[2], c->stream);
  if (rc == TTSH_OK && hipEventSynchronize(ev[2]) != hipSuccess) rc = fail(TTSH_EHIP, "sync failed");
  float m0 = 0, m1 = 0;
  if (rc == TTSH_OK) {
    hipEventElapsedTime(&m0, ev[0], ev[1]);
    hipEventElapsedTime(&m1, ev[1], ev[2]);
  }
  for (auto& e : ev) hipEventDestroy(e);
  if (rc) return rc;
  out[0] = 1000.0 * m0 / (double)nsteps;
  out[1] = 1000.0 * m1 / (double)nsteps;
  return TTSH_OK;
}

int ttsh_tune(ttsh_ctx* c, int64_t nsteps, int* cfg_out, double* us_out) {
  if (!c) return fail(TTSH_EINVAL, "null context");
  if (nsteps < 1 || nsteps > 100000) return fail(TTSH_EINVAL, "nsteps must be in 1..1e5");
  // save the state and the mixed-domain v, omega of every class
  std::vector<void*> save;
  size_t bytes_total = 0;
  const size_t er = elem_real(c->prec), es = elem_state(c->prec);
  for (auto& k : c->cls) bytes_total += k.ids.size() * (k.sSt() * es + k.sX() * 2 * er);
  void* buf = nullptr;
  if (hipMalloc(&buf, bytes_total) != hipSuccess) return fail(TTSH_ENOMEM, "tuner scratch allocation failed");
  auto copy_all = [&](bool to_buf) -> hipError_t {
    char* p = (char*)buf;
    for (auto& k : c->cls) {
      const size_t bs_ = k.ids.size() * k.sSt() * es, bx = k.ids.size() * k.sX() * 2 * er;
      hipError_t e = to_buf ? hipMemcpyAsync(p, k.st, bs_, hipMemcpyDeviceToDevice, c->stream)
                            : hipMemcpyAsync(k.st, p, bs_, hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return e;
      p += bs_;
      e = to_buf ? hipMemcpyAsync(p, k.X, bx, hipMemcpyDeviceToDevice, c->stream)
                 : hipMemcpyAsync(k.X, p, bx, hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return e;
      p += bx;
    }
    return hipSuccess;
  };
  int rc = TTSH_OK;
  if (copy_all(true) != hipSuccess) rc = fail(TTSH_EHIP, "tuner save failed");
  const int keep[7] = {c->bs_row, c->bs, c->split_row, c->split_col, c->sched_row, c->sched_col, c->groups};
  int best_row[3] = {0, 0, kSchedDefault}, best_col[3] = {0, 0, kSchedDefault};  // bs, split, schedule
  double row_us = 0.0, col_us = 0.0;
  // every candidate is timed in two rounds (all candidates once, then all
  // again) and keeps its faster time, which evens out drifts of the clock
  struct Cand {
    int bs, split, sch;
    double row, col;
  };
  std::vector<Cand> cands;
  for (int split = must_split(c) ? 1 : 0; split < 2; ++split)
    for (int bs : {64, 128, 256}) {
      if (!bs_valid(c, bs)) continue;
      const int nsch = sched_usable(c, split) ? 1 + kNumSchedVariants : 1;
      for (int q = 0; q < nsch; ++q) cands.push_back({bs, split, q == 0 ? kSchedDefault : kSchedVariants[q - 1], 1e30, 1e30});
    }
  for (int round = 0; round < 2 && rc == TTSH_OK; ++round)
    for (Cand& k : cands) {
      c->bs = c->bs_row = k.bs;
      c->split_row = c->split_col = k.split;
      c->sched_row = c->sched_col = k.sch;
      double t[2];
      if (enqueue_steps(c, 2, c->stream) != TTSH_OK) { rc = TTSH_EHIP; break; }  // warm-up
      if ((rc = ttsh_pass_times(c, nsteps, t)) != TTSH_OK) break;
      k.row = std::min(k.row, t[0]);
      k.col = std::min(k.col, t[1]);
    }
  for (const Cand& k : cands) {
    if (!best_row[0] || k.row < row_us) { best_row[0] = k.bs; best_row[1] = k.split; best_row[2] = k.sch; row_us = k.row; }
    if (!best_col[0] || k.col < col_us) { best_col[0] = k.bs; best_col[1] = k.split; best_col[2] = k.sch; col_us = k.col; }
  }
  // Whole steps decide the column workgroup size and the number of
  // concurrent groups: with two groups the row pass of one runs beside the
  // column pass of the other, and the column size that is fastest alone need
  // not be the one that shares the GPU best.  The row pass keeps its choice;
  // each column size brings its fastest (split, schedule); each candidate is
  // replayed as ttsh_step runs it (graphs, group streams), two rounds.
  int best_groups = 1;
  double step_us = row_us + col_us;
  // the per-pass runs re-applied column updates with fixed forcing (unstable
  // modes may have overflowed): whole steps start from the saved state, with
  // the guard off so that they leave no flags for the next ttsh_sync
  if (rc == TTSH_OK && copy_all(false) != hipSuccess) rc = fail(TTSH_EHIP, "tuner restore failed");
  const int keep_guard = c->guard;
  c->guard = 0;
  if (rc == TTSH_OK && best_row[0]) {
    struct Whole {
      int bs, split, sch, groups;
      double us;
    };
    std::vector<Whole> whole;
    for (int bs : {64, 128, 256}) {
      const Cand* b = nullptr;
      for (const Cand& k : cands)
        if (k.bs == bs && (!b || k.col < b->col)) b = &k;
      if (!b) continue;
      for (int G = 1; G <= std::min(kMaxGroups, c->n_inst); ++G) whole.push_back({bs, b->split, b->sch, G, 1e30});
    }
    hipEvent_t w0 = nullptr, w1 = nullptr;
    if (hipEventCreate(&w0) != hipSuccess || hipEventCreate(&w1) != hipSuccess)
      rc = fail(TTSH_EHIP, "event creation failed");
    for (int round = 0; round < 2 && rc == TTSH_OK; ++round)
      for (Whole& w : whole) {
        c->bs_row = best_row[0];
        c->split_row = best_row[1];
        c->sched_row = best_row[2];
        c->bs = w.bs;
        c->split_col = w.split;
        c->sched_col = w.sch;
        c->groups = w.groups;
        drop_graph(c);
        if ((rc = ttsh_step(c, nsteps)) != TTSH_OK) break;  // captures the graphs
        hipEventRecord(w0, c->stream);
        if ((rc = ttsh_step(c, nsteps)) != TTSH_OK) break;
        hipEventRecord(w1, c->stream);
        if (hipEventSynchronize(w1) != hipSuccess) {
          rc = fail(TTSH_EHIP, "sync failed");
          break;
        }
        float ms = 0.f;
        hipEventElapsedTime(&ms, w0, w1);
        w.us = std::min(w.us, 1000.0 * ms / (double)nsteps);
      }
    if (w0) hipEventDestroy(w0);
    if (w1) hipEventDestroy(w1);
    const Whole* win = nullptr;
    for (const Whole& w : whole)
      if (!win || w.us < win->us) win = &w;
    if (rc == TTSH_OK && win) {
      best_col[0] = win->bs;
      best_col[1] = win->split;
      best_col[2] = win->sch;
      best_groups = win->groups;
      step_us = win->us;
    }
    drop_graph(c);
  }
  c->guard = keep_guard;
  if (copy_all(false) != hipSuccess && rc == TTSH_OK) rc = fail(TTSH_EHIP, "tuner restore failed");
  hipStreamSynchronize(c->stream);
  hipFree(buf);
  if (rc != TTSH_OK || !best_row[0]) {
    c->bs_row = keep[0];
    c->bs = keep[1];
    c->split_row = keep[2];
    c->split_col = keep[3];
    c->sched_row = keep[4];
    c->sched_col = keep[5];
    c->groups = keep[6];
    drop_graph(c);
    return rc ? rc : fail(TTSH_EUNSUPPORTED, "no workgroup size to tune");
  }
  // the two passes are tuned independently (the data layout depends on
  // neither the workgroup size nor the transform schedule)
  c->bs_row = best_row[0];
  c->split_row = best_row[1];
  c->sched_row = best_row[2];
  c->bs = best_col[0];
  c->split_col = best_col[1];
  c->sched_col = best_col[2];
  c->groups = best_groups;
  c->opt_bs = 0;
  drop_graph(c);
  if (cfg_out) {
    const int cfg[7] = {best_row[0], best_col[0], best_row[1], best_col[1], best_row[2], best_col[2], best_groups};
    std::copy(cfg, cfg + 7, cfg_out);
  }
  if (us_out) *us_out = step_us;
  return TTSH_OK;
}

int ttsh_device_arch(char* out, int n) {
  if (!out || n < 1) return fail(TTSH_EINVAL, "null or empty output");
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(TTSH_EHIP, "no HIP device available");
  std::snprintf(out, (size_t)n, "%s", prop.gcnArchName);
  return TTSH_OK;
}

int ttsh_get_tuning(ttsh_ctx* c, int* cfg) {
  if (!c || !cfg) return fail(TTSH_EINVAL, "null argument");
  const int v[7] = {c->bs_row, c->bs, c->split_row || must_split(c), c->split_col || must_split(c), c->sched_row,
                    c->sched_col, c->groups};
  std::copy(v, v + 7, cfg);
  return TTSH_OK;
}

int ttsh_set_tuning(ttsh_ctx* c, const int* cfg) {
  if (!c || !cfg) return fail(TTSH_EINVAL, "null argument");
  for (int q = 0; q < 2; ++q)
    if (!bs_valid(c, cfg[q])) return fail(TTSH_EINVAL, "workgroup size not usable for this context");
  for (int q = 2; q < 4; ++q)
    if (cfg[q] != 0 && cfg[q] != 1) return fail(TTSH_EINVAL, "split flags must be 0 or 1");
  for (int q = 4; q < 6; ++q) {
    const int sch = cfg[q];
    const bool known = sch == kSchedDefault || std::find(kSchedVariants, kSchedVariants + kNumSchedVariants, sch) !=
                                                   kSchedVariants + kNumSchedVariants;
    if (!known) return fail(TTSH_EINVAL, "unknown transform schedule");
    if (sch != kSchedDefault && !sched_usable(c, cfg[q - 2]))
      return fail(TTSH_EINVAL, "a non-default schedule needs the FP32 arithmetic and the multi-size launch");
  }
  if (cfg[6] < 1 || cfg[6] > kMaxGroups) return fail(TTSH_EINVAL, "groups must be 1 or 2");
  if (cfg[6] > c->n_inst) return fail(TTSH_EINVAL, "two groups need at least two instances");
  c->bs_row = cfg[0];
  c->bs = cfg[1];
  c->split_row = cfg[2];
  c->split_col = cfg[3];
  c->sched_row = cfg[4];
  c->sched_col = cfg[5];
  c->groups = cfg[6];
  c->opt_bs = 0;
  drop_graph(c);
  return TTSH_OK;
}

int ttsh_fft2(const double* in, double* out, int N, int batch, int inverse, int precision) {
  if (!in || !out) return fail(TTSH_EINVAL, "null pointer");
  const SizeOps* ops = size_ops(N);
  if (!ops) return fail(TTSH_EUNSUPPORTED, "N must be one of 64, 128, 256, 512, 1024, 2048, 4096, 8192");
  if (batch < 1) return fail(TTSH_EINVAL, "batch must be >= 1");
  if (precision != 32 && precision != 64) return fail(TTSH_EINVAL, "precision must be 32 or 64");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(TTSH_EHIP, "no HIP device available");
  const bool f64 = precision == 64;
  const size_t n = (size_t)batch * N * N;
  void* tw = nullptr;
  void* buf = nullptr;
  int rc = make_twiddles(N, f64, &tw);
  if (rc) return rc;
  auto done = [&](int r) {
    hipDeviceSynchronize();
    if (tw) hipFree(tw);
    if (buf) hipFree(buf);
    return r;
  };
  if (hipMalloc(&buf, n * (f64 ? 16 : 8)) != hipSuccess) return done(fail(TTSH_ENOMEM, "allocation failed"));
  if (f64) {
    if (hipMemcpy(buf, in, n * 16, hipMemcpyDeviceToDevice) != hipSuccess) return done(fail(TTSH_EHIP, "copy failed"));
  } else {
    hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(2 * n)), dim3(kB), 0, 0, in, (float*)buf, 2 * n);
  }
  if (ops->fft2(buf, batch, inverse ? +1 : -1, f64, tw, 0) != hipSuccess) return done(fail(TTSH_EHIP, "fft launch failed"));
  if (f64) {
    hipLaunchKernelGGL(k_scale_c, dim3(nblk(n)), dim3(kB), 0, 0, (C2<double>*)buf, 1.0 / N, n);
    if (hipMemcpy(out, buf, n * 16, hipMemcpyDeviceToDevice) != hipSuccess) return done(fail(TTSH_EHIP, "copy failed"));
  } else {
    hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(2 * n)), dim3(kB), 0, 0, (const float*)buf, out, 2 * n);
    hipLaunchKernelGGL(k_scale_c, dim3(nblk(n)), dim3(kB), 0, 0, (C2<double>*)out, 1.0 / N, n);
  }
  if (hipGetLastError() != hipSuccess) return done(fail(TTSH_EHIP, "kernel launch failed"));
  return done(TTSH_OK);
}

}  // extern "C"
