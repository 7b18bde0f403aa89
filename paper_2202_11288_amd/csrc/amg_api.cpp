// C ABI of the library (include/amg.h): hierarchy setup, level matvecs, the
// block V-cycle of Algorithm 2 and the outer iteration of Sec. 5 on one
// MI355X.  All device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/amg.h"
#include "amg_device.hpp"
#include "amg_host.hpp"
#include "fft_lds.hpp"

using namespace amg;

namespace {

// levels with L <= 2^kTailLog run in the one-workgroup tail kernels (amg_device.hpp)

// Levels above the coarsest with at most this many unknowns are folded into
// one dense operator of the cycle below them (form_sub_vcycle,
// form_sub_wcycle).  A W-cycle visits the bottom levels so often that a
// product with a 511 x 511 matrix still beats the sub-cycles it replaces; a
// V-cycle visits them once, and 255 is where the product stops paying.
constexpr int kSubDenseMax = 255;
constexpr int kSubDenseMaxW = 511;

struct Plan {
  int logL, logL1, logL2, tcols;
  bool tail;
};

// The hand-chosen geometry of a four-step level of size 2^logL (and the
// tail's for logL <= kTailLog).
Plan default_plan(int logL) {
  Plan p{};
  p.logL = logL;
  p.tail = logL <= kTailLog;
  if (p.tail) {
    p.logL1 = logL;
    p.logL2 = 0;
    p.tcols = 1;
    return p;
  }
  // rows of L1 <= kCap4/2 complex (two rows per workgroup: 64 KB of LDS for
  // FP64), columns of L2 in tiles of T columns with T*L2 <= kCap4.  L >= 2^22
  // take rows of 4096 (a row pair of 2 kCap4 on twice the threads): with rows
  // of 2048 the columns of L = 2^23 would come in tiles of 2 (8-byte row
  // segments, which made its column passes line-bound) and those of L = 2^22
  // in tiles of 4 rather than 8.  L = 2^20 takes rows of 2048 for the same
  // reason: columns of 512 in tiles of 8 rather than columns of 1024 in 4
  p.logL1 = logL >= 22 ? 12 : (logL == 20 ? 11 : std::min(11, (logL + 1) / 2));
  p.logL2 = logL - p.logL1;
  int t = std::max(1, std::min(16, kCap4 >> p.logL2));
  while (t > 4 && ((1 << p.logL1) / t) < 256) t >>= 1;
  // the largest levels: tiles of 2 kCap4 (twice the columns, so twice the
  // bytes per row segment) while that still leaves a tile per CU
  if ((t << p.logL2) == kCap4 && ((1 << p.logL1) / (2 * t)) >= 256) t *= 2;
  p.tcols = t;
  return p;
}

bool same_geometry(const Plan& a, const Plan& b) {
  return a.logL == b.logL && a.logL1 == b.logL1 && a.logL2 == b.logL2 && a.tcols == b.tcols;
}

// Alternative geometries of a size: every (row length, column tile) whose
// row-pass and column-pass kernel instances are the ones some default plan
// runs (the same code, other strides and tile counts), default first.
std::vector<Plan> plan_candidates(int logL) {
  std::vector<Plan> out;
  const Plan d = default_plan(logL);
  out.push_back(d);
  if (d.tail) return out;
  struct ColInst { int logL2, tcols; };
  std::vector<ColInst> cols;
  std::vector<int> rows;
  for (int k = kTailLog + 1; k <= 23; ++k) {
    const Plan q = default_plan(k);
    bool seen = false;
    for (const ColInst& c : cols) seen = seen || (c.logL2 == q.logL2 && c.tcols == q.tcols);
    if (!seen) cols.push_back({q.logL2, q.tcols});
    if (std::find(rows.begin(), rows.end(), q.logL1) == rows.end()) rows.push_back(q.logL1);
  }
  for (int l1 : rows)
    for (const ColInst& c : cols) {
      if (l1 + c.logL2 != logL || (1 << l1) / c.tcols < 64) continue;
      Plan p = d;
      p.logL1 = l1;
      p.logL2 = c.logL2;
      p.tcols = c.tcols;
      if (!same_geometry(p, d)) out.push_back(p);
    }
  return out;
}

// Geometries in use per size (process-wide): the default, or the one that
// amg_plan_set or amg_autotune chose; read when a hierarchy is set up.
struct PlanChoice {
  bool set = false;
  Plan p{};
  double us_default = 0, us_best = 0;
  int candidates = 0, rejected = 0;
};
std::mutex g_plan_mu;
PlanChoice g_plan[32];

Plan plan_level(int64_t n) {
  int logL = 0;
  while ((int64_t(1) << logL) < 2 * (n + 1)) ++logL;
  std::lock_guard<std::mutex> g(g_plan_mu);
  if (logL < 32 && g_plan[logL].set) return g_plan[logL].p;
  return default_plan(logL);
}

struct LevelRes {
  int64_t n = 0;
  Plan plan{};
  bool sym = false;
  double o = 0, dv = 0, dw = 0;
  double *g1d = nullptr, *g2d = nullptr;
  float *g1f = nullptr, *g2f = nullptr;
  double *pd = nullptr, *qd = nullptr, *xid = nullptr, *zetad = nullptr;
  float *pf = nullptr, *qf = nullptr, *xif = nullptr, *zetaf = nullptr;
  double *bd = nullptr, *ud = nullptr, *rd = nullptr, *scald = nullptr;
  float *bf = nullptr, *uf = nullptr, *rf = nullptr, *scalf = nullptr;
  // band (weakly singular model): sub, main, super, 1 / diagonal, product
  double *bsubd = nullptr, *bmaind = nullptr, *bsupd = nullptr, *dinvd = nullptr, *bcd = nullptr;
  float *bsubf = nullptr, *bmainf = nullptr, *bsupf = nullptr, *dinvf = nullptr, *bcf = nullptr;

  template <typename T>
  LevelDev<T> dev() const;
};

template <>
LevelDev<double> LevelRes::dev<double>() const {
  LevelDev<double> v{};
  v.n = (int)n;
  v.logL = plan.logL;
  v.logL1 = plan.logL1;
  v.logL2 = plan.logL2;
  v.tcols = plan.tcols;
  v.sym = sym;
  v.g1 = g1d;
  v.g2 = g2d;
  v.p = pd;
  v.q = qd;
  v.xi = xid;
  v.zeta = zetad;
  v.o = o;
  v.dv = dv;
  v.dw = dw;
  v.b = bd;
  v.u = ud;
  v.r = rd;
  v.scal = scald;
  v.bsub = bsubd;
  v.bmain = bmaind;
  v.bsup = bsupd;
  v.dinv = dinvd;
  v.bc = bcd;
  return v;
}

template <>
LevelDev<float> LevelRes::dev<float>() const {
  LevelDev<float> v{};
  v.n = (int)n;
  v.logL = plan.logL;
  v.logL1 = plan.logL1;
  v.logL2 = plan.logL2;
  v.tcols = plan.tcols;
  v.sym = sym;
  v.g1 = g1f;
  v.g2 = g2f;
  v.p = pf;
  v.q = qf;
  v.xi = xif;
  v.zeta = zetaf;
  v.o = (float)o;
  v.dv = (float)dv;
  v.dw = (float)dw;
  v.b = bf;
  v.u = uf;
  v.r = rf;
  v.scal = scalf;
  v.bsub = bsubf;
  v.bmain = bmainf;
  v.bsup = bsupf;
  v.dinv = dinvf;
  v.bc = bcf;
  return v;
}

}  // namespace

// Event-based timing of selected launches (AMG_FLAG_PROFILE).
// Finest-level passes are kept apart by precision (FP32 kinds = FP64 kind + 4).
enum ProfKind {
  PK_COL_FWD = 0, PK_ROW, PK_COL_INV, PK_SWEEP,
  PK_COL_FWD32, PK_ROW32, PK_COL_INV32, PK_SWEEP32,
  PK_TAIL, PK_VCYCLE, PK_OUTER, PK_COUNT
};
static const char* const kProfNames[PK_COUNT] = {
    "fp64_finest_col_fwd", "fp64_finest_row", "fp64_finest_col_inv", "fp64_finest_sweep",
    "fp32_finest_col_fwd", "fp32_finest_row", "fp32_finest_col_inv", "fp32_finest_sweep",
    "tail_vcycle", "vcycle", "outer_residual"};

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<std::pair<int, std::pair<size_t, size_t>>> pending;
  int64_t launches[PK_COUNT] = {};
  double total_ms[PK_COUNT] = {};
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  // returns the index of a recorded event, or SIZE_MAX if profiling is off
  size_t mark(hipStream_t s) {
    if (!on) return SIZE_MAX;
    if (next == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return SIZE_MAX;
      pool.push_back(e);
    }
    if (hipEventRecord(pool[next], s) != hipSuccess) return SIZE_MAX;
    return next++;
  }
  void span(int kind, size_t a, size_t b) {
    if (a != SIZE_MAX && b != SIZE_MAX) pending.push_back({kind, {a, b}});
  }
  // after the stream has been synchronised
  void collect() {
    for (auto& p : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pool[p.second.first], pool[p.second.second]) == hipSuccess) {
        launches[p.first] += 1;
        total_ms[p.first] += ms;
      }
    }
    pending.clear();
    next = 0;
  }
};

struct amg_ctx {
  Profiler prof;
  KernelSpec kspec{};
  int device = 0;
  int64_t N = 0;
  amg_opts_t opts{};
  bool host_only = false;
  bool mixed = false;
  std::vector<TpxLevel> host;
  std::vector<LevelRes> lv;
  int first_tail = 0;
  int maxL_tail = 0;
  int tail_variant = 0;  // TAIL_BAND / TAIL_SYM of the tail levels (all alike)
  CoarseLU lu{};
  // The V-cycle's small-level kernel stops at level vc_last and applies lu_vc
  // there: the coarsest level's inverse, or (when a level above the coarsest
  // has at most kSubDenseMax unknowns) the dense matrix of the whole V-cycle
  // below and including that level, which is linear in its right-hand side.
  int vc_last = 0;
  CoarseLU lu_vc{};
  // AMG_FLAG_DEEP_FOLD: the cycle below the four-step levels as one dense
  // product (row-major m x m, FP64 and its FP32 rounding); m = 0: not formed
  int deep_m = 0;
  const double* deep64 = nullptr;
  const float* deep32 = nullptr;
  // The same for W-cycles: the small-level programs stop at level w_last and
  // apply lu_w there (the coarsest inverse, or the matrix of all the visits a
  // level receives each time the level above descends).
  int w_last = 0;
  CoarseLU lu_w{};
  Twiddles<double> tw64{};
  Twiddles<float> tw32{};
  cplx<double>* buf64 = nullptr;
  cplx<float>* buf32 = nullptr;
  double* dpart64 = nullptr;  // per-block dot partials (FP64 levels)
  float* dpart32 = nullptr;   // per-block dot partials (FP32 levels)
  double* npart = nullptr;    // per-block residual-norm partials
  LevelDev<double>* lvdev64 = nullptr;
  LevelDev<float>* lvdev32 = nullptr;
  SolveState* st_dev = nullptr;
  SolveState* st_host = nullptr;  // pinned
  double* hist_dev = nullptr;
  double* rout = nullptr;  // FP64 outer residual (mixed precision)
  std::vector<double> hist;
  int last_iters = 0;
  // Device memory: a handle's buffers are carved from a few large chunks
  // (the first sized by the footprint estimate), so that a setup makes a
  // handful of hipMalloc calls and amg_destroy a handful of hipFree calls
  // rather than hundreds; setup temporaries come from chunks of a per-device
  // pool that later setups reuse.
  std::vector<std::pair<void*, size_t>> dev_allocs;  // chunks (address, usable bytes)
  std::vector<std::pair<void*, size_t>> spare;       // a retired handle's chunks, for reuse
  char* bump = nullptr;
  size_t bump_used = 0, bump_cap = 0, arena_hint = 0;
  std::vector<std::pair<void*, size_t>> setup_temps;  // pool chunks
  char* tbump = nullptr;
  size_t tbump_used = 0, tbump_cap = 0;
  // V-cycle replay (see AMG_FLAG_EAGER): captured on an internal stream at
  // the handle's second V-cycle; every argument of its kernels is a
  // handle-owned buffer, so the graph stays valid for the handle's lifetime.
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t vgraph = nullptr;
  int vcycles_eager = 0;
  // conjugate gradients (inner = AMG_INNER_PCG): direction, A p, previous
  // residual (FP64, 2N-1 each) and the dot-product block partials
  double* cg_p = nullptr;
  double* cg_q = nullptr;
  double* cg_rold = nullptr;
  double* cg_part = nullptr;
  bool cg_restart = false;  // the next CG step starts a new direction sequence
  // right-hand side of amg_bdf4_step (allocated by its first call)
  double* step_b = nullptr;
  // restarted flexible GMRES (inner = AMG_INNER_GMRES): basis V ((restart+1)
  // vectors), preconditioned vectors Z (restart vectors), Hessenberg matrix,
  // rotations, rotated right-hand side, small scratch; gm_j = the next
  // Arnoldi column (host-side, read after each round's synchronisation)
  double* gm_V = nullptr;
  double* gm_Z = nullptr;
  double* gm_H = nullptr;
  double* gm_small = nullptr;  // g | cs | sn | hcur | y | hn, kGmMax + 1 each
  double* gm_part = nullptr;
  int gm_j = 0;
  // W-cycles (cycle = 2): the small-level programs for the first and the
  // later visits of the first small level
  TailOp* tail_prog[2] = {nullptr, nullptr};
  int tail_prog_n[2] = {0, 0};
  // split outer residual (AMG_FLAG_ACCURATE_RESIDUAL): the finest level's far
  // field (spectra and Cross data of the stencil entries beyond kNearM
  // half-steps, geometry and work vectors of level 0) and the near field
  // hierarchy formed on the device (stencil kernels, not AMG_FLAG_HOST_ONLY):
  // the host keeps only the level sizes, the diagonal scalars and the
  // coarsest level; gpu_sym: the levels are symmetric (known from the kernel)
  bool gpu_setup = false;
  bool gpu_sym = false;
  bool split = false;
  LevelRes far0;
  double* ynear = nullptr;
  double* near_w = nullptr;
  double* near_rl = nullptr;
  double* near_rr = nullptr;
  double near_rin[2] = {0.0, 0.0};
};

namespace {

// A failing HIP call returns AMG_EHIP; with AMG_DEBUG set in the environment
// the call, its line and the HIP error name also go to stderr.
int hip_fail(hipError_t e, const char* expr, int line) {
  static const bool dbg = std::getenv("AMG_DEBUG") != nullptr;
  if (dbg) std::fprintf(stderr, "amg: %s failed at line %d: %s\n", expr, line, hipGetErrorName(e));
  return AMG_EHIP;
}

#define HIP_TRY(expr)                                             \
  do {                                                            \
    hipError_t _e = (expr);                                       \
    if (_e != hipSuccess) return hip_fail(_e, #expr, __LINE__);   \
  } while (0)

constexpr size_t kAllocAlign = 256;     // every buffer starts on 256 bytes
constexpr size_t kAllocPad = 256;       // and is followed by this much slack
constexpr size_t kChunkGuard = 65536;   // unused tail of every chunk
constexpr size_t kChunkMin = size_t(1) << 20;

inline size_t alloc_bytes(size_t bytes) {
  return ((bytes + kAllocPad + kAllocAlign - 1) / kAllocAlign) * kAllocAlign;
}

template <typename T>
int dalloc(amg_ctx* c, T** p, size_t count) {
  if (count == 0) count = 1;
  const size_t need = alloc_bytes(count * sizeof(T));
  if (!c->bump || c->bump_used + need > c->bump_cap) {
    size_t cap = std::max(need, std::max(c->arena_hint, kChunkMin));
    c->arena_hint = 0;  // later chunks are sized by the request
    void* ptr = nullptr;
    // a spare chunk that holds the request (the largest first: the spares of
    // a handle of the same shape match its chunks in order)
    auto best = c->spare.end();
    for (auto it = c->spare.begin(); it != c->spare.end(); ++it)
      if (it->second >= need && (best == c->spare.end() || it->second > best->second)) best = it;
    if (best != c->spare.end()) {
      ptr = best->first;
      cap = best->second;
      c->spare.erase(best);
    } else if (hipMalloc(&ptr, cap + kChunkGuard) != hipSuccess) {
      return AMG_ENOMEM;
    }
    c->dev_allocs.push_back({ptr, cap});
    c->bump = static_cast<char*>(ptr);
    c->bump_used = 0;
    c->bump_cap = cap;
  }
  *p = reinterpret_cast<T*>(c->bump + c->bump_used);
  c->bump_used += need;
  return AMG_OK;
}

#define AMG_TRY(expr)               \
  do {                              \
    int _r = (expr);                \
    if (_r != AMG_OK) return _r;    \
  } while (0)

template <typename T>
int upload(amg_ctx* c, T** dst, const std::vector<T>& src, hipStream_t s) {
  AMG_TRY(dalloc(c, dst, src.size()));
  HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return AMG_OK;
}

// Per-device pool of setup scratch chunks (power-of-two sizes), kept for
// later setups up to kTempPoolMax bytes per device, freed beyond that.
constexpr size_t kTempChunkMin = size_t(64) << 20;
constexpr size_t kTempPoolMax = size_t(4) << 30;
struct TempPool {
  std::multimap<size_t, void*> free;
  size_t bytes = 0;
};
std::mutex g_tmp_mu;
std::unordered_map<int, TempPool> g_tmp;

int temp_chunk_get(int dev, size_t need, void** out, size_t* size) {
  size_t sz = kTempChunkMin;
  while (sz < need) sz <<= 1;
  {
    std::lock_guard<std::mutex> g(g_tmp_mu);
    TempPool& P = g_tmp[dev];
    auto it = P.free.lower_bound(sz);
    if (it != P.free.end() && it->first <= 4 * sz) {
      *out = it->second;
      *size = it->first;
      P.bytes -= it->first;
      P.free.erase(it);
      return AMG_OK;
    }
  }
  if (hipMalloc(out, sz + kChunkGuard) != hipSuccess) return AMG_ENOMEM;
  *size = sz;
  return AMG_OK;
}

// Setup temporaries that stay allocated until setup has synchronised its
// stream once at the end (the generators behind the spectra).
template <typename T>
int dalloc_temp(amg_ctx* c, T** p, size_t count) {
  if (count == 0) count = 1;
  const size_t need = alloc_bytes(count * sizeof(T));
  if (!c->tbump || c->tbump_used + need > c->tbump_cap) {
    void* ptr = nullptr;
    size_t sz = 0;
    AMG_TRY(temp_chunk_get(c->device, need, &ptr, &sz));
    c->setup_temps.push_back({ptr, sz});
    c->tbump = static_cast<char*>(ptr);
    c->tbump_used = 0;
    c->tbump_cap = sz;
  }
  *p = reinterpret_cast<T*>(c->tbump + c->tbump_used);
  c->tbump_used += need;
  return AMG_OK;
}
template <typename T>
int upload_temp(amg_ctx* c, T** dst, const std::vector<T>& src, hipStream_t s) {
  AMG_TRY(dalloc_temp(c, dst, src.size()));
  HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return AMG_OK;
}
// The caller has synchronised the setup stream: the chunks go back to the
// pool (or are freed once the pool is full).
void free_setup_temps(amg_ctx* c) {
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> g(g_tmp_mu);
    TempPool& P = g_tmp[c->device];
    for (const auto& t : c->setup_temps) {
      if (P.bytes + t.second <= kTempPoolMax) {
        P.free.insert({t.second, t.first});
        P.bytes += t.second;
      } else {
        drop.push_back(t.first);
      }
    }
  }
  for (void* q : drop) (void)hipFree(q);
  c->setup_temps.clear();
  c->tbump = nullptr;
  c->tbump_used = c->tbump_cap = 0;
}

std::vector<float> to_float(const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); }

bool ignores_delta(const amg_kernel_t* k) {
  return k->kind == AMG_K_GENERATORS || k->kind == AMG_K_WEAKLY_SINGULAR;
}

KernelSpec spec_of(const amg_kernel_t* k, double delta) {
  KernelSpec s;
  s.kind = k->kind;
  s.delta = delta;
  s.alpha = k->alpha;
  s.wl = k->wl;
  s.wr = k->wr;
  s.gen = k->gen;
  s.scheme = (k->kind == AMG_K_GENERATORS || k->kind == AMG_K_WEAKLY_SINGULAR) ? SCHEME_SHIFTED
                                                                                : k->scheme;
  s.gamma = k->gamma;
  return s;
}

int check_opts(const amg_opts_t* o) {
  if (o->m1 < 1 || o->m2 < 1 || o->m1 > 16 || o->m2 > 16) return AMG_ENOTSUP;
  if (!(o->omega_pre > 0 && o->omega_pre < 2) || !(o->omega_post > 0 && o->omega_post < 2))
    return AMG_EINVAL;
  if (o->coarsest_log2 < 2 || o->coarsest_log2 > 7) return AMG_EINVAL;
  if (o->precision != AMG_FP64 && o->precision != AMG_MIXED) return AMG_EINVAL;
  if (o->max_iter < 0 || o->max_iter > 100000) return AMG_EINVAL;
  if (o->flags & ~(AMG_FLAG_HOST_ONLY | AMG_FLAG_PROFILE | AMG_FLAG_EAGER |
                   AMG_FLAG_ACCURATE_RESIDUAL | AMG_FLAG_DEEP_FOLD))
    return AMG_EINVAL;
  if (o->inner != AMG_INNER_VCYCLE && o->inner != AMG_INNER_PCG && o->inner != AMG_INNER_GMRES)
    return AMG_EINVAL;
  if (o->restart < 1 || o->restart > kGmMax) return AMG_EINVAL;
  if (o->cycle != 1 && o->cycle != 2) return AMG_EINVAL;
  if (!(std::isfinite(o->scale) && o->scale > 0.0) || !std::isfinite(o->shift)) return AMG_EINVAL;
  return AMG_OK;
}

// Unknowns of the deep fold's level (AMG_FLAG_DEEP_FOLD): the first level
// with L <= 2^kTailLog below the finest, if it has more than kSubDenseMax
// unknowns; 0 otherwise.
int64_t deep_fold_size(int64_t N, const amg_opts_t* o) {
  const int64_t nc = (int64_t(1) << o->coarsest_log2) - 1;
  int64_t n = N - 1;
  for (int l = 0;; ++l) {
    if (2 * (n + 1) <= (int64_t(1) << kTailLog)) {
      const int64_t m = 2 * n + 1;
      return (l >= 1 && n > nc && m > kSubDenseMax && m <= kFoldMax) ? m : 0;
    }
    if (n <= nc) return 0;
    n = (n - 1) / 2;
  }
}

int64_t footprint(int64_t N, const amg_opts_t* o, bool sym_guess, bool band) {
  // device bytes: spectra (FP64 + FP32 if mixed), Cross vectors, vectors,
  // FFT scratch, LU, tables
  const bool mixed = o->precision == AMG_MIXED;
  int64_t bytes = 0;
  int64_t n = N - 1;
  int64_t L0 = 2 * N;
  while (n >= (int64_t(1) << o->coarsest_log2) - 1) {
    const int64_t L = 2 * (n + 1);
    const int64_t spec = (sym_guess ? 2 : 4) * L;  // reals per spectrum pair
    bytes += spec * 8 + (mixed ? spec * 4 : 0);
    bytes += 4 * n * (8 + (mixed ? 4 : 0));
    bytes += 3 * (2 * n + 1) * (mixed ? 12 : 8);
    if (band) bytes += 5 * (2 * n + 1) * (mixed ? 12 : 8);  // band, 1/diagonal, product
    if (n == (int64_t(1) << o->coarsest_log2) - 1) break;
    n = (n - 1) / 2;
  }
  bytes += L0 * 16 * 2 + (mixed ? L0 * 8 : 0);           // FFT scratch (setup uses two)
  bytes += (mixed ? (2 * N - 1) * 8 : 0);                // outer residual
  if (o->inner == AMG_INNER_PCG) bytes += 3 * (2 * N - 1) * 8 + 2 * 1024 * 8;  // p, q, r_old
  if (o->inner == AMG_INNER_GMRES)  // V, Z, H, small vectors, dot partials
    bytes += (int64_t)(2 * o->restart + 1) * (2 * N - 1) * 8 +
             (int64_t)(kGmMax + 1) * (kGmMax + 6 + 1024) * 8;
  const int64_t mc = (int64_t(2) << o->coarsest_log2) - 1;
  bytes += 2 * mc * mc * 8;
  const int64_t md = o->cycle == 2 ? kSubDenseMaxW : kSubDenseMax;
  if (mc < md) bytes += md * md * (mixed ? 12 : 8);  // the folded sub-cycle's operator
  bytes += (int64_t)(kTwM + kTw4Lo + kTw4Hi) * 24;
  if ((o->flags & AMG_FLAG_DEEP_FOLD) && o->cycle == 1) {
    const int64_t md = deep_fold_size(N, o);
    bytes += md * md * (mixed ? 12 : 8);
  }
  if (o->flags & AMG_FLAG_ACCURATE_RESIDUAL)  // far-field spectra + Cross, near-field output
    bytes += (sym_guess ? 2 : 4) * L0 * 8 + 4 * (N - 1) * 8 + (2 * N - 1) * 8 +
             (4 * kNearM + 2) * 8;
  return bytes;
}

template <typename T>
const T* deep_of(const amg_ctx* c);
template <>
const double* deep_of<double>(const amg_ctx* c) { return c->deep64; }
template <>
const float* deep_of<float>(const amg_ctx* c) { return c->deep32; }
template <typename T>
const Twiddles<T>& tw_of(const amg_ctx* c);
template <>
const Twiddles<double>& tw_of<double>(const amg_ctx* c) { return c->tw64; }
template <>
const Twiddles<float>& tw_of<float>(const amg_ctx* c) { return c->tw32; }
template <typename T>
cplx<T>* buf_of(const amg_ctx* c);
template <>
cplx<double>* buf_of<double>(const amg_ctx* c) { return c->buf64; }
template <>
cplx<float>* buf_of<float>(const amg_ctx* c) { return c->buf32; }
template <typename T>
T* dpart_of(const amg_ctx* c);
template <>
double* dpart_of<double>(const amg_ctx* c) { return c->dpart64; }
template <>
float* dpart_of<float>(const amg_ctx* c) { return c->dpart32; }
template <typename T>
const LevelDev<T>* lvdev_of(const amg_ctx* c);
template <>
const LevelDev<double>* lvdev_of<double>(const amg_ctx* c) { return c->lvdev64; }
template <>
const LevelDev<float>* lvdev_of<float>(const amg_ctx* c) { return c->lvdev32; }

// Work memory of a four-step matvec: the FFT buffer (L complex), the pass-1
// block partials of the w_o row and the level's two w_o scalars.  Null
// members: the handle's own.
template <typename T>
struct FourstepWork {
  cplx<T>* buf = nullptr;
  T* part = nullptr;
  T* scal = nullptr;
};

// One four-step matvec of level l with the given prologue and epilogue.
template <typename T>
int fourstep(amg_ctx* c, int l, int cmode, const ColIn<T>& in, int emode, const EpiOut<T>& out,
             hipStream_t s, const FourstepWork<T>& wk = FourstepWork<T>{}) {
  LevelDev<T> d = c->lv[l].template dev<T>();
  if (wk.scal) d.scal = wk.scal;
  cplx<T>* buf = wk.buf ? wk.buf : buf_of<T>(c);
  T* dp = wk.part ? wk.part : dpart_of<T>(c);
  const Twiddles<T>& tw = tw_of<T>(c);
  Profiler& P = c->prof;
  const bool prof = P.on && l == 0 && !wk.buf;  // caller-provided work memory: no events
  // events around the whole sweep only: events between its passes would add
  // their own gaps to it (the passes' durations come from a kernel trace)
  const size_t e0 = prof ? P.mark(s) : SIZE_MAX;
  HIP_TRY(launch_col_fwd<T>(cmode, d, in, buf, tw, dp, s));
  if (d.bmain) {
    // the band's product with the matvec input (as formed by the first pass)
    const T* xb = cmode == COL_MV ? in.x
                : cmode == COL_OUTER_UPDATE ? reinterpret_cast<const T*>(in.xo) : d.u;
    HIP_TRY(launch_band_mv<T>(d, xb, s));
  }
  HIP_TRY(launch_row<T>(1, d, buf, tw, dp, col_blocks(d.logL1, d.tcols), out.xin, s));
  HIP_TRY(launch_col_inv<T>(emode, d, out, buf, tw, c->npart, s));
  if (prof) {
    const size_t e3 = P.mark(s);
    const int off = sizeof(T) == 4 ? PK_COL_FWD32 : PK_COL_FWD;
    P.span(off + 3, e0, e3);
  }
  return AMG_OK;
}

template <typename T>
int wcycle_visit(amg_ctx* c, int l, bool first, hipStream_t s);

template <typename T>
int vcycle_dev(amg_ctx* c, hipStream_t s) {
  // input: level 0's b; output: level 0's u (precision T)
  if (c->opts.cycle == 2) return wcycle_visit<T>(c, 0, true, s);
  const amg_opts_t& o = c->opts;
  const int nl = (int)c->lv.size();
  const int ft = c->first_tail;
  const T wpre = (T)o.omega_pre, wpost = (T)o.omega_post;
  for (int l = 0; l < ft; ++l) {
    const LevelDev<T> d = c->lv[l].template dev<T>();
    ColIn<T> in{};
    in.omega = wpre;
    int cmode = COL_PRE;
    if (l > 0) {
      cmode = COL_PRE_RESTRICT;
      in.x = c->lv[l - 1].template dev<T>().r;
    }
    EpiOut<T> out{};
    out.xin = d.u;
    out.omega = wpre;
    for (int sweep = 1; sweep <= o.m1; ++sweep) {
      const int em = (sweep == o.m1) ? EPI_RESID : EPI_SMOOTH;
      AMG_TRY(fourstep<T>(c, l, cmode, in, em, out, s));
      cmode = COL_MV;
      in = ColIn<T>{};
      in.x = d.u;
    }
  }
  {
    const T* rf = (ft > 0) ? c->lv[ft - 1].template dev<T>().r : nullptr;
    const size_t t0 = c->prof.mark(s);
    if (c->deep_m) {
      T* u = c->lv[ft].template dev<T>().u;
      const hipError_t e = launch_fold_gemv<T, T>(rf, c->deep_m, deep_of<T>(c), u, s);
      if (e != hipSuccess) return hip_fail(e, "launch_fold_gemv", __LINE__);
    } else
      HIP_TRY(launch_tail_vcycle<T>(lvdev_of<T>(c), ft, c->vc_last, rf, o.m1, o.m2, wpre, wpost,
                                    c->lu_vc, tw_of<T>(c), c->maxL_tail, c->tail_variant, s));
    c->prof.span(PK_TAIL, t0, c->prof.mark(s));
  }
  for (int l = ft - 1; l >= 0; --l) {
    const LevelDev<T> d = c->lv[l].template dev<T>();
    ColIn<T> in{};
    in.x = c->lv[l + 1].template dev<T>().u;
    int cmode = COL_PROLONG;
    EpiOut<T> out{};
    out.xin = d.u;
    out.omega = wpost;
    for (int sweep = 0; sweep < o.m2; ++sweep) {
      AMG_TRY(fourstep<T>(c, l, cmode, in, EPI_SMOOTH, out, s));
      cmode = COL_MV;
      in = ColIn<T>{};
      in.x = d.u;
    }
  }
  return AMG_OK;
}

// The small-level part of a W-cycle visit of level l (first visit: smoothing
// from zero as in the V-cycle; later visits: m1 sweeps from the current
// iterate, then the residual); every level above the coarsest visits the
// next level `gamma` times, the level above the coarsest visits it once.
void tail_visit(std::vector<TailOp>& ops, int l, bool first, int ft, int last, int m1, int m2,
                int gamma, bool has_rf) {
  if (l == last) {
    ops.push_back({last, 0, 0, TAILOP_COARSE});
    return;
  }
  if (first) {
    for (int sw = 0; sw < m1; ++sw) {
      const int pro = sw > 0 ? TP_USE_U : ((l == ft && !has_rf) ? TP_PRE_B : TP_PRE_RESTRICT);
      ops.push_back({l, pro, sw == m1 - 1 ? TE_RESID : TE_SMOOTH, 0});
    }
  } else {
    for (int sw = 0; sw < m1; ++sw) ops.push_back({l, TP_USE_U, TE_SMOOTH, 0});
    ops.push_back({l, TP_USE_U, TE_RESID, 0});
  }
  const int visits = (l + 1 == last) ? 1 : gamma;
  for (int v = 0; v < visits; ++v) tail_visit(ops, l + 1, v == 0, ft, last, m1, m2, gamma, has_rf);
  for (int sw = 0; sw < m2; ++sw)
    ops.push_back({l, sw == 0 ? TP_PROLONG : TP_USE_U, TE_SMOOTH, TAILOP_UP});
}

// Level l of a W-cycle on the four-step levels (the small levels run as one
// program per visit).
template <typename T>
int wcycle_visit(amg_ctx* c, int l, bool first, hipStream_t s) {
  const amg_opts_t& o = c->opts;
  const int nl = (int)c->lv.size();
  const int ft = c->first_tail;
  const T wpre = (T)o.omega_pre, wpost = (T)o.omega_post;
  if (l == ft) {
    const T* rf = (ft > 0) ? c->lv[ft - 1].template dev<T>().r : nullptr;
    const int k = first ? 0 : 1;
    HIP_TRY(launch_tail_program<T>(lvdev_of<T>(c), ft, c->w_last, rf, c->tail_prog[k],
                                   c->tail_prog_n[k], wpre, wpost, c->lu_w, tw_of<T>(c),
                                   c->maxL_tail, c->tail_variant, s));
    return AMG_OK;
  }
  const LevelDev<T> d = c->lv[l].template dev<T>();
  EpiOut<T> out{};
  out.xin = d.u;
  out.omega = wpre;
  ColIn<T> mv{};
  mv.x = d.u;
  if (first) {
    ColIn<T> in{};
    in.omega = wpre;
    int cmode = COL_PRE;
    if (l > 0) {
      cmode = COL_PRE_RESTRICT;
      in.x = c->lv[l - 1].template dev<T>().r;
    }
    for (int sweep = 1; sweep <= o.m1; ++sweep) {
      AMG_TRY(fourstep<T>(c, l, cmode, in, sweep == o.m1 ? EPI_RESID : EPI_SMOOTH, out, s));
      cmode = COL_MV;
      in = mv;
    }
  } else {
    for (int sweep = 0; sweep < o.m1; ++sweep) AMG_TRY(fourstep<T>(c, l, COL_MV, mv, EPI_SMOOTH, out, s));
    AMG_TRY(fourstep<T>(c, l, COL_MV, mv, EPI_RESID, out, s));
  }
  const int visits = (l + 1 == nl - 1) ? 1 : o.cycle;
  for (int v = 0; v < visits; ++v) AMG_TRY(wcycle_visit<T>(c, l + 1, v == 0, s));
  ColIn<T> in{};
  in.x = c->lv[l + 1].template dev<T>().u;
  int cmode = COL_PROLONG;
  out.omega = wpost;
  for (int sweep = 0; sweep < o.m2; ++sweep) {
    AMG_TRY(fourstep<T>(c, l, cmode, in, EPI_SMOOTH, out, s));
    cmode = COL_MV;
    in = mv;
  }
  return AMG_OK;
}

constexpr int kGraphMinLevels = 2;

// One V-cycle in the handle's precision (level 0's b in, level 0's u out):
// the first runs eagerly (it also raises the kernels' LDS limits), the second
// is captured into a graph, and from then on the graph is replayed on s.
int vcycle_run(amg_ctx* c, hipStream_t s) {
  auto eager = [c](hipStream_t st) {
    return c->mixed ? vcycle_dev<float>(c, st) : vcycle_dev<double>(c, st);
  };
  // a graph pays off only over many launches: at least two four-step levels
  // (a V-cycle of only the small-level kernel launches it directly)
  if (c->prof.on || (c->opts.flags & AMG_FLAG_EAGER) || c->first_tail < kGraphMinLevels)
    return eager(s);
  if (!c->vgraph && c->vcycles_eager >= 1) {
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const int st = eager(c->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
    if (st != AMG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    HIP_TRY(ec);
    const hipError_t ei = hipGraphInstantiate(&c->vgraph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) c->vgraph = nullptr;
    HIP_TRY(ei);
  }
  if (c->vgraph) {
    HIP_TRY(hipGraphLaunch(c->vgraph, s));
    return AMG_OK;
  }
  ++c->vcycles_eager;
  return eager(s);
}

// The passes of r = b - A x on the finest level (FP64; split form under
// AMG_FLAG_ACCURATE_RESIDUAL), optionally with x += e fused in front, into
// ro (and its FP32 copy r32, if set); the block partials of ||r||^2 go to
// c->npart.  Returns the number of partials through *npart_out.
int residual_passes(amg_ctx* c, const double* b, double* x, const void* e, double* ro,
                    float* r32, hipStream_t s, int* npart_out) {
  const LevelRes& L0 = c->lv[0];
  const LevelDev<double> d = L0.dev<double>();
  ColIn<double> in{};
  EpiOut<double> out{};
  out.xin = x;
  out.bo = b;
  out.ro = ro;
  out.r32 = r32;
  int cmode = COL_MV;
  if (e) {
    cmode = COL_OUTER_UPDATE;
    in.xo = x;
    in.e = e;
    in.e_is_float = c->mixed ? 1 : 0;
  } else {
    in.x = x;
  }
  int npart = 1;
  if (c->split) {
    // far field through the FFT passes (pass 1 also applies x += e), the near
    // field in difference form from the updated x, added in the epilogue
    const LevelDev<double> df = c->far0.dev<double>();
    HIP_TRY(launch_col_fwd<double>(cmode, df, in, c->buf64, c->tw64, c->dpart64, s));
    HIP_TRY(launch_near(x, c->ynear, c->N, c->near_w, c->near_rl, c->near_rr, c->near_rin[0],
                        c->near_rin[1], s));
    HIP_TRY(launch_row<double>(1, df, c->buf64, c->tw64, c->dpart64,
                               col_blocks(df.logL1, df.tcols), x, s));
    out.ynear = c->ynear;
    HIP_TRY(launch_col_inv<double>(EPI_OUTER, df, out, c->buf64, c->tw64, c->npart, s));
    npart = col_blocks(df.logL1, df.tcols);
  } else if (L0.plan.tail) {
    HIP_TRY(launch_tail_matvec<double>(cmode, EPI_OUTER, d, in, out, c->tw64, c->npart, s));
  } else {
    AMG_TRY(fourstep<double>(c, 0, cmode, in, EPI_OUTER, out, s));
    npart = col_blocks(d.logL1, d.tcols);
  }
  *npart_out = npart;
  return AMG_OK;
}

// r = b - A x (residual_passes into the solver's residual buffers), then the
// stopping test; publish != null: the stop test also writes the state to
// that pinned host copy (the round ends there).
int outer_residual(amg_ctx* c, const double* b, double* x, const void* e, double tol,
                   hipStream_t s, bool gm_check = false, bool stall = false,
                   SolveState* publish = nullptr) {
  const LevelRes& L0 = c->lv[0];
  int npart = 1;
  AMG_TRY(residual_passes(c, b, x, e, c->mixed ? c->rout : L0.bd, c->mixed ? L0.bf : nullptr, s,
                          &npart));
  if (gm_check)
    HIP_TRY(launch_gm_check(c->st_dev, c->npart, npart, tol, c->opts.max_iter, c->hist_dev, s,
                            stall ? 1 : 0));
  else
    HIP_TRY(launch_finish(c->st_dev, c->npart, npart, tol, c->opts.max_iter, c->hist_dev, s, 0,
                          publish));
  return AMG_OK;
}

template <typename T>
int level_matvec(amg_ctx* c, int l, const T* x, T* y, hipStream_t s,
                 const FourstepWork<T>& wk = FourstepWork<T>{}) {
  const LevelRes& R = c->lv[l];
  const LevelDev<T> d = R.template dev<T>();
  ColIn<T> in{};
  in.x = x;
  EpiOut<T> out{};
  out.xin = x;
  out.y = y;
  if (R.plan.tail) {
    // the tail kernel's work lives in LDS (no partials are written for EPI_MV)
    HIP_TRY(launch_tail_matvec<T>(COL_MV, EPI_MV, d, in, out, tw_of<T>(c), nullptr, s));
    return AMG_OK;
  }
  return fourstep<T>(c, l, COL_MV, in, EPI_MV, out, s, wk);
}

int level_matvec64(amg_ctx* c, int l, const double* x, double* y, hipStream_t s) {
  return level_matvec<double>(c, l, x, y, s);
}

// The V-cycle below and including level k (pre-smoothing from zero, the
// recursion, post-smoothing) is a linear map of level k's right-hand side.
// For the largest level k above the coarsest with at most kSubDenseMax
// unknowns, its matrix is formed column by column by running the FP64
// small-level kernel on the unit vectors; the V-cycle's small-level kernel
// then stops at level k and applies it as it applies the coarsest inverse.
// One dense product of m^2 entries replaces that level's and the levels
// below's steps (a few microseconds of one workgroup each, whatever their
// size) and the coarsest solve.
int form_sub_vcycle(amg_ctx* c, hipStream_t s) {
  const int nl = (int)c->lv.size();
  const int ft = c->first_tail;
  int k = -1;
  for (int l = ft; l < nl - 1; ++l)
    if (2 * c->lv[l].n + 1 <= kSubDenseMax) {
      k = l;
      break;
    }
  if (k < 0) return AMG_OK;
  const amg_opts_t& o = c->opts;
  const int m = (int)(2 * c->lv[k].n + 1);
  double* M = nullptr;
  AMG_TRY(dalloc(c, &M, (size_t)m * m));
  // all m unit vectors at once: one small-level kernel block per column, each
  // with its own copies of the level vectors (b, u, r, scal) of levels k..last
  // in a setup scratch block and its own level table
  const int last = nl - 1;
  int64_t col = 0;  // doubles per column
  std::vector<int64_t> off(nl, 0);
  for (int l = k; l <= last; ++l) {
    off[l] = col;
    col += 3 * (2 * c->lv[l].n + 1) + 4;
  }
  col = (col + 31) & ~int64_t(31);
  double* scr = nullptr;  // setup temporary
  AMG_TRY(dalloc_temp(c, &scr, (size_t)(col * m)));
  std::vector<LevelDev<double>> tables((size_t)m * nl);
  for (int j = 0; j < m; ++j)
    for (int l = k; l <= last; ++l) {
      LevelDev<double> d = c->lv[l].dev<double>();
      const int64_t sz = 2 * c->lv[l].n + 1;
      double* base = scr + (int64_t)j * col + off[l];
      d.b = base;
      d.u = base + sz;
      d.r = base + 2 * sz;
      d.scal = base + 3 * sz;
      tables[(size_t)j * nl + l] = d;
    }
  LevelDev<double>* tdev = nullptr;
  AMG_TRY(upload_temp(c, &tdev, tables, s));
  std::vector<TailArgs<double>> args((size_t)m);
  for (int j = 0; j < m; ++j) {
    TailArgs<double>& a = args[(size_t)j];
    a.levels = tdev + (size_t)j * nl;
    a.first = k;
    a.last = last;
    a.rf = nullptr;
    a.m1 = o.m1;
    a.m2 = o.m2;
    a.wpre = o.omega_pre;
    a.wpost = o.omega_post;
    a.lu = c->lu;
    a.st = nullptr;
    a.gate = GATE_ACTIVE;
  }
  TailArgs<double>* adev = nullptr;
  AMG_TRY(upload_temp(c, &adev, args, s));
  HIP_TRY(hipMemsetAsync(scr, 0, (size_t)(col * m) * sizeof(double), s));
  HIP_TRY(launch_basis_batch(scr + off[k], col, m, s));
  HIP_TRY(launch_tail_vcycle_batch<double>(adev, m, c->tail_variant, c->tw64, s));
  HIP_TRY(launch_gather_columns(M, scr + off[k] + (2 * c->lv[k].n + 1), col, m, s));
  float* M32 = nullptr;  // the FP32 V-cycle reads the operator's FP32 rounding
  if (c->mixed) {
    AMG_TRY(dalloc(c, &M32, (size_t)m * m));
    HIP_TRY(launch_copy_d2f(M, M32, (int64_t)m * m, s));
  }
  c->vc_last = k;
  c->lu_vc = {m, M, M32};
  return AMG_OK;
}

// AMG_FLAG_DEEP_FOLD: the V-cycle below the four-step levels (the small-
// level kernel's levels first_tail .. vc_last and the operator it applies
// there) is a linear map of level first_tail's right-hand side; its matrix
// is formed from the unit vectors (the FP64 small-level kernel, in chunks of
// columns) and stored row-major for the multi-workgroup product.
int form_deep_fold(amg_ctx* c, hipStream_t s) {
  const int nl = (int)c->lv.size();
  const int k = c->first_tail;
  const int64_t md = deep_fold_size(c->N, &c->opts);
  if (md == 0 || k < 1 || k >= nl || 2 * c->lv[k].n + 1 != md || c->vc_last <= k) return AMG_OK;
  const amg_opts_t& o = c->opts;
  const int m = (int)md;
  const int last = c->vc_last;
  double* M = nullptr;
  AMG_TRY(dalloc(c, &M, (size_t)m * m));
  int64_t col = 0;
  std::vector<int64_t> off(nl, 0);
  for (int l = k; l <= last; ++l) {
    off[l] = col;
    col += 3 * (2 * c->lv[l].n + 1) + 4;
  }
  col = (col + 31) & ~int64_t(31);
  constexpr int kChunk = 1024;
  double* scr = nullptr;
  AMG_TRY(dalloc_temp(c, &scr, (size_t)(col * std::min(m, kChunk))));
  for (int j0 = 0; j0 < m; j0 += kChunk) {
    const int cnt = std::min(kChunk, m - j0);
    std::vector<LevelDev<double>> tables((size_t)cnt * nl);
    for (int j = 0; j < cnt; ++j)
      for (int l = 0; l < nl; ++l) {
        LevelDev<double> d = c->lv[l].dev<double>();
        if (l >= k && l <= last) {
          const int64_t sz = 2 * c->lv[l].n + 1;
          double* base = scr + (int64_t)j * col + off[l];
          d.b = base;
          d.u = base + sz;
          d.r = base + 2 * sz;
          d.scal = base + 3 * sz;
        }
        tables[(size_t)j * nl + l] = d;
      }
    LevelDev<double>* tdev = nullptr;
    AMG_TRY(upload_temp(c, &tdev, tables, s));
    std::vector<TailArgs<double>> args((size_t)cnt);
    for (int j = 0; j < cnt; ++j) {
      TailArgs<double>& a = args[(size_t)j];
      a.levels = tdev + (size_t)j * nl;
      a.first = k;
      a.last = last;
      a.rf = nullptr;
      a.m1 = o.m1;
      a.m2 = o.m2;
      a.wpre = o.omega_pre;
      a.wpost = o.omega_post;
      a.lu = c->lu_vc;
      a.st = nullptr;
      a.gate = GATE_ACTIVE;
    }
    TailArgs<double>* adev = nullptr;
    AMG_TRY(upload_temp(c, &adev, args, s));
    HIP_TRY(hipMemsetAsync(scr, 0, (size_t)(col * cnt) * sizeof(double), s));
    HIP_TRY(launch_basis_batch(scr + off[k], col, m, s, cnt, j0));
    HIP_TRY(launch_tail_vcycle_batch<double>(adev, cnt, c->tail_variant, c->tw64, s));
    HIP_TRY(launch_gather_rows(M, scr + off[k] + m, col, m, j0, cnt, s));
  }
  float* M32 = nullptr;
  if (c->mixed) {
    AMG_TRY(dalloc(c, &M32, (size_t)m * m));
    HIP_TRY(launch_copy_d2f(M, M32, (int64_t)m * m, s));
  }
  c->deep_m = m;
  c->deep64 = M;
  c->deep32 = M32;
  return AMG_OK;
}

// W-cycles: each time a level descends, the level below receives gamma visits
// (the first from zero, the others from the current iterate with the same
// right-hand side), which together are a linear map of that right-hand
// side.  For the largest level strictly below the small-level kernel's first
// one with at most kSubDenseMax unknowns, setup forms the matrix of those
// visits from the unit vectors (the FP64 step-program kernel on a program of
// just those visits), and the small-level programs stop there and apply it:
// 2^d visits of that level and everything below become 2^d dense products.
int form_sub_wcycle(amg_ctx* c, hipStream_t s) {
  const int nl = (int)c->lv.size();
  const int ft = c->first_tail, last = nl - 1;
  int k = -1;
  for (int l = ft + 1; l < last; ++l)
    if (2 * c->lv[l].n + 1 <= kSubDenseMaxW) {
      k = l;
      break;
    }
  if (k < 0) return AMG_OK;
  const amg_opts_t& o = c->opts;
  std::vector<TailOp> ops;
  for (int v = 0; v < o.cycle; ++v) tail_visit(ops, k, v == 0, k, last, o.m1, o.m2, o.cycle, false);
  std::vector<int> raw(ops.size() * 4);
  std::memcpy(raw.data(), ops.data(), raw.size() * sizeof(int));
  int* prog = nullptr;
  AMG_TRY(upload(c, &prog, raw, s));
  const int m = (int)(2 * c->lv[k].n + 1);
  double* M = nullptr;
  AMG_TRY(dalloc(c, &M, (size_t)m * m));
  double* bk = c->lv[k].bd;
  const double* uk = c->lv[k].ud;
  for (int j = 0; j < m; ++j) {
    HIP_TRY(launch_basis(bk, m, j, s));
    HIP_TRY(launch_tail_program<double>(c->lvdev64, k, last, nullptr,
                                        reinterpret_cast<const TailOp*>(prog), (int)ops.size(),
                                        o.omega_pre, o.omega_post, c->lu, c->tw64, c->maxL_tail,
                                        c->tail_variant, s));
    HIP_TRY(hipMemcpyAsync(M + (size_t)j * m, uk, (size_t)m * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  }
  float* M32 = nullptr;
  if (c->mixed) {
    AMG_TRY(dalloc(c, &M32, (size_t)m * m));
    HIP_TRY(launch_copy_d2f(M, M32, (int64_t)m * m, s));
  }
  c->w_last = k;
  c->lu_w = {m, M, M32};
  return AMG_OK;
}

// Spectra G1, G2 of a level (eq. (ccs3.4)) in FP64 (and their FP32 rounding
// when `f32`): the circulant columns of its four Toeplitz generators through
// the level's forward FFT, combined into the packed product's form.
int level_spectra_dev(amg_ctx* c, const double* ga, const double* gb, const double* gc,
                      const double* gd, LevelRes& R, bool f32, cplx<double>* zscratch,
                      hipStream_t s);

int level_spectra(amg_ctx* c, const TpxLevel& H, LevelRes& R, bool f32, cplx<double>* zscratch,
                  hipStream_t s) {
  // generators: setup temporaries, freed when setup has synchronised
  double *ga, *gb, *gc, *gd;
  AMG_TRY(upload_temp(c, &ga, H.a, s));
  AMG_TRY(upload_temp(c, &gb, H.b, s));
  AMG_TRY(upload_temp(c, &gc, H.c, s));
  AMG_TRY(upload_temp(c, &gd, H.d, s));
  return level_spectra_dev(c, ga, gb, gc, gd, R, f32, zscratch, s);
}

int level_spectra_dev(amg_ctx* c, const double* ga, const double* gb, const double* gc,
                      const double* gd, LevelRes& R, bool f32, cplx<double>* zscratch,
                      hipStream_t s) {
  const int64_t L = int64_t(1) << R.plan.logL;
  const size_t nspec = (size_t)(R.sym ? L : 2 * L);
  AMG_TRY(dalloc(c, &R.g1d, nspec));
  AMG_TRY(dalloc(c, &R.g2d, nspec));
  if (f32) {
    AMG_TRY(dalloc(c, &R.g1f, nspec));
    AMG_TRY(dalloc(c, &R.g2f, nspec));
  }
  const LevelDev<double> d = R.dev<double>();
  if (R.plan.tail) {
    HIP_TRY(launch_tail_fft_setup(d, ga, gb, c->buf64, c->tw64, s));
    HIP_TRY(launch_tail_fft_setup(d, gc, gd, zscratch, c->tw64, s));
  } else {
    ColIn<double> in{};
    double* dummy = nullptr;
    AMG_TRY(dalloc_temp(c, &dummy, (size_t)col_blocks(d.logL1, d.tcols)));
    in.gx = const_cast<double*>(ga);
    in.gy = const_cast<double*>(gb);
    HIP_TRY(launch_col_fwd<double>(COL_SETUP, d, in, c->buf64, c->tw64, dummy, s));
    HIP_TRY(launch_row<double>(0, d, c->buf64, c->tw64, dummy, 0, nullptr, s));
    in.gx = const_cast<double*>(gc);
    in.gy = const_cast<double*>(gd);
    HIP_TRY(launch_col_fwd<double>(COL_SETUP, d, in, zscratch, c->tw64, dummy, s));
    HIP_TRY(launch_row<double>(0, d, zscratch, c->tw64, dummy, 0, nullptr, s));
  }
  HIP_TRY(launch_combine(R.plan.logL, R.plan.logL1, R.plan.logL2, c->buf64, zscratch, R.sym,
                         R.g1d, R.g2d, f32 ? R.g1f : nullptr, f32 ? R.g2f : nullptr, s));
  return AMG_OK;
}

struct DevTwiddles {
  Twiddles<double> t64{};
  Twiddles<float> t32{};
  bool ready = false;
};
std::mutex g_tw_mu;
std::unordered_map<int, DevTwiddles> g_tw;

int device_twiddles(int dev, hipStream_t s, Twiddles<double>* t64, Twiddles<float>* t32) {
  std::lock_guard<std::mutex> g(g_tw_mu);
  DevTwiddles& D = g_tw[dev];
  if (!D.ready) {
    const std::vector<double> base = twiddles(kTwM, kTwM);
    const std::vector<double> lo = twiddles(int64_t(1) << kTw4Log, kTw4Lo);
    const std::vector<double> hi = twiddles(int64_t(1) << kTw4Log, kTw4Hi, kTw4Lo);
    const std::vector<float> basef = to_float(base), lof = to_float(lo), hif = to_float(hi);
    const std::vector<const void*> src = {base.data(), lo.data(), hi.data(),
                                          basef.data(), lof.data(), hif.data()};
    const size_t bytes[6] = {base.size() * 8, lo.size() * 8, hi.size() * 8,
                             basef.size() * 4, lof.size() * 4, hif.size() * 4};
    void* p[6] = {};
    for (int i = 0; i < 6; ++i) {
      if (hipMalloc(&p[i], bytes[i]) != hipSuccess) {
        for (int k = 0; k < i; ++k) (void)hipFree(p[k]);
        return AMG_ENOMEM;
      }
      HIP_TRY(hipMemcpyAsync(p[i], src[i], bytes[i], hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    D.t64 = {static_cast<cplx<double>*>(p[0]), static_cast<cplx<double>*>(p[1]),
             static_cast<cplx<double>*>(p[2])};
    D.t32 = {static_cast<cplx<float>*>(p[3]), static_cast<cplx<float>*>(p[4]),
             static_cast<cplx<float>*>(p[5])};
    D.ready = true;
  }
  *t64 = D.t64;
  *t32 = D.t32;
  return AMG_OK;
}

int setup_device(amg_ctx* c, hipStream_t s) {
  const bool mixed = c->mixed;
  const int nl = (int)c->host.size();
  // twiddle tables (long double, rounded once): one copy per device, shared
  // by every handle on it and kept until the process ends
  AMG_TRY(device_twiddles(c->device, s, &c->tw64, &c->tw32));
  const int64_t L0 = 2 * c->N;
  AMG_TRY(dalloc(c, &c->buf64, (size_t)L0));
  if (mixed) AMG_TRY(dalloc(c, &c->buf32, (size_t)L0));
  cplx<double>* zscratch = nullptr;  // second setup transform
  AMG_TRY(dalloc(c, &zscratch, (size_t)L0));
  int maxblocks = 1;
  c->lv.resize(nl);
  c->first_tail = nl - 1;
  c->maxL_tail = 0;
  // device-built hierarchy (stencil kernels): every level's generators and
  // Cross data formed on the device; the host receives the diagonal scalars
  // and the coarsest level (for its LU)
  std::vector<DevTpx> dt;
  if (c->gpu_setup) {
    dt.resize(nl);
    // per-thread host buffers: a set-up thread's later hierarchies reuse
    // their pages (the copies are staged when hipMemcpyAsync returns)
    static thread_local std::vector<double> Wn, Wm;
    int64_t Sn = 0, Sm = 0;
    const bool same = row_stencils_reuse(c->kspec, c->N, Wn, Sn, Wm, Sm);
    double *wn, *wm, *scratch, *dscal;
    int* bad;
    AMG_TRY(upload_temp(c, &wn, Wn, s));
    if (same) wm = wn;
    else AMG_TRY(upload_temp(c, &wm, Wm, s));
    AMG_TRY(dalloc_temp(c, &scratch, (size_t)(4 * c->host[0].n)));
    AMG_TRY(dalloc_temp(c, &dscal, (size_t)(3 * nl)));
    AMG_TRY(dalloc_temp(c, &bad, 1));
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), s));
    for (int l = 0; l < nl; ++l) {
      const int64_t n = c->host[l].n;
      LevelRes& R = c->lv[l];
      DevTpx& T = dt[l];
      AMG_TRY(dalloc_temp(c, &T.a, (size_t)(2 * n - 1)));
      AMG_TRY(dalloc_temp(c, &T.b, (size_t)(2 * n - 1)));
      AMG_TRY(dalloc_temp(c, &T.c, (size_t)(2 * n - 1)));
      AMG_TRY(dalloc_temp(c, &T.d, (size_t)(2 * n - 1)));
      AMG_TRY(dalloc_temp(c, &T.o, 1));
      AMG_TRY(dalloc(c, &R.pd, (size_t)n));
      AMG_TRY(dalloc(c, &R.qd, (size_t)n));
      AMG_TRY(dalloc(c, &R.xid, (size_t)n));
      AMG_TRY(dalloc(c, &R.zetad, (size_t)n));
      T.p = R.pd;
      T.q = R.qd;
      T.xi = R.xid;
      T.zeta = R.zetad;
      if (l == 0)
        HIP_TRY(launch_finest_level(wn, Sn, wm, Sm, n, c->opts.scale, c->opts.shift, T, bad, s));
      else
        HIP_TRY(launch_coarsen(dt[l - 1], c->host[l - 1].n, T, scratch, c->gpu_sym, bad, s));
      HIP_TRY(launch_level_scalars(T, n, dscal + 3 * l, s));
    }
    std::vector<double> sc((size_t)(3 * nl));
    int hbad = 0;
    HIP_TRY(hipMemcpyAsync(sc.data(), dscal, sc.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    // the coarsest level on the host, for its LU
    TpxLevel& Hc = c->host[nl - 1];
    const int64_t nc = Hc.n;
    for (auto* v : {&Hc.a, &Hc.b, &Hc.c, &Hc.d}) v->assign((size_t)(2 * nc - 1), 0.0);
    for (auto* v : {&Hc.p, &Hc.q, &Hc.xi, &Hc.zeta}) v->assign((size_t)nc, 0.0);
    const DevTpx& Tc = dt[nl - 1];
    const std::pair<std::vector<double>*, const double*> cp[8] = {
        {&Hc.a, Tc.a}, {&Hc.b, Tc.b}, {&Hc.c, Tc.c}, {&Hc.d, Tc.d},
        {&Hc.p, Tc.p}, {&Hc.q, Tc.q}, {&Hc.xi, Tc.xi}, {&Hc.zeta, Tc.zeta}};
    for (const auto& pr : cp)
      HIP_TRY(hipMemcpyAsync(pr.first->data(), pr.second, pr.first->size() * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hbad) return AMG_EINVAL;
    for (int l = 0; l < nl; ++l) {
      c->host[l].o = sc[(size_t)(3 * l)];
      c->lv[l].o = sc[(size_t)(3 * l)];
      c->lv[l].dv = sc[(size_t)(3 * l + 1)];
      c->lv[l].dw = sc[(size_t)(3 * l + 2)];
      if (!(c->lv[l].dv != 0.0 && c->lv[l].dw != 0.0 && c->lv[l].o != 0.0))
        return AMG_EINVAL;  // Jacobi needs a nonzero diagonal
    }
    Hc.o = sc[(size_t)(3 * (nl - 1))];
  }
  for (int l = 0; l < nl; ++l) {
    const TpxLevel& H = c->host[l];
    LevelRes& R = c->lv[l];
    R.n = H.n;
    R.plan = plan_level(H.n);
    if (l == nl - 1) R.plan.tail = true;  // the coarsest level always lives in the tail kernel
    if (R.plan.tail) {
      c->first_tail = std::min(c->first_tail, l);
      c->maxL_tail = std::max(c->maxL_tail, 1 << R.plan.logL);
      R.plan.logL1 = R.plan.logL;
      R.plan.logL2 = 0;
      R.plan.tcols = 1;
    } else {
      maxblocks = std::max(maxblocks, col_blocks(R.plan.logL1, R.plan.tcols));
      maxblocks = std::max(maxblocks, (1 << R.plan.logL2) / 2);
    }
    const int64_t n = H.n, m = 2 * n + 1, L = int64_t(1) << R.plan.logL;
    if (c->gpu_setup) {
      R.sym = c->gpu_sym;
    } else {
      R.sym = H.symmetric();
      R.o = H.o;
      R.dv = H.a[H.n - 1];
      R.dw = H.d[H.n - 1];
      AMG_TRY(upload(c, &R.pd, H.p, s));
      AMG_TRY(upload(c, &R.qd, H.q, s));
      AMG_TRY(upload(c, &R.xid, H.xi, s));
      AMG_TRY(upload(c, &R.zetad, H.zeta, s));
    }
    (void)L;
    AMG_TRY(dalloc(c, &R.bd, m));
    AMG_TRY(dalloc(c, &R.ud, m));
    AMG_TRY(dalloc(c, &R.rd, m));
    AMG_TRY(dalloc(c, &R.scald, 4));
    HIP_TRY(hipMemsetAsync(R.bd, 0, m * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(R.ud, 0, m * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(R.rd, 0, m * sizeof(double), s));
    if (H.has_band()) {
      std::vector<double> dinv((size_t)m);
      for (int64_t i = 0; i < m; ++i) {
        const double dt = i < n ? H.a[n - 1] : (i == n ? H.o : H.d[n - 1]);
        dinv[(size_t)i] = 1.0 / (dt + H.bmain[(size_t)i]);
      }
      AMG_TRY(upload(c, &R.bsubd, H.bsub, s));
      AMG_TRY(upload(c, &R.bmaind, H.bmain, s));
      AMG_TRY(upload(c, &R.bsupd, H.bsup, s));
      AMG_TRY(upload(c, &R.dinvd, dinv, s));
      AMG_TRY(dalloc(c, &R.bcd, m));
      if (mixed) {
        AMG_TRY(upload(c, &R.bsubf, to_float(H.bsub), s));
        AMG_TRY(upload(c, &R.bmainf, to_float(H.bmain), s));
        AMG_TRY(upload(c, &R.bsupf, to_float(H.bsup), s));
        AMG_TRY(upload(c, &R.dinvf, to_float(dinv), s));
        AMG_TRY(dalloc(c, &R.bcf, m));
      }
    }
    if (mixed) {
      if (c->gpu_setup) {
        AMG_TRY(dalloc(c, &R.pf, (size_t)n));
        AMG_TRY(dalloc(c, &R.qf, (size_t)n));
        AMG_TRY(dalloc(c, &R.xif, (size_t)n));
        AMG_TRY(dalloc(c, &R.zetaf, (size_t)n));
        HIP_TRY(launch_copy_d2f(R.pd, R.pf, n, s));
        HIP_TRY(launch_copy_d2f(R.qd, R.qf, n, s));
        HIP_TRY(launch_copy_d2f(R.xid, R.xif, n, s));
        HIP_TRY(launch_copy_d2f(R.zetad, R.zetaf, n, s));
      } else {
        AMG_TRY(upload(c, &R.pf, to_float(H.p), s));
        AMG_TRY(upload(c, &R.qf, to_float(H.q), s));
        AMG_TRY(upload(c, &R.xif, to_float(H.xi), s));
        AMG_TRY(upload(c, &R.zetaf, to_float(H.zeta), s));
      }
      AMG_TRY(dalloc(c, &R.bf, m));
      AMG_TRY(dalloc(c, &R.uf, m));
      AMG_TRY(dalloc(c, &R.rf, m));
      AMG_TRY(dalloc(c, &R.scalf, 4));
      HIP_TRY(hipMemsetAsync(R.bf, 0, m * sizeof(float), s));
      HIP_TRY(hipMemsetAsync(R.uf, 0, m * sizeof(float), s));
      HIP_TRY(hipMemsetAsync(R.rf, 0, m * sizeof(float), s));
    }
    if (c->gpu_setup)
      AMG_TRY(level_spectra_dev(c, dt[l].a, dt[l].b, dt[l].c, dt[l].d, R, mixed, zscratch, s));
    else
      AMG_TRY(level_spectra(c, H, R, mixed, zscratch, s));
  }
  if (c->split) {
    // the far field of the finest level: same geometry and work vectors,
    // its own spectra (FP64 only) and Cross data
    const KernelSpec ks = c->kspec;
    TpxLevel far = finest_level(ks, c->N, kNearM);
    if (c->opts.scale != 1.0) shift_level(far, 0.0, c->opts.scale);
    LevelRes& F = c->far0;
    F = c->lv[0];
    F.sym = far.symmetric() && c->lv[0].sym;
    F.o = far.o;
    F.g1f = F.g2f = nullptr;
    F.pf = F.qf = F.xif = F.zetaf = nullptr;
    AMG_TRY(upload(c, &F.pd, far.p, s));
    AMG_TRY(upload(c, &F.qd, far.q, s));
    AMG_TRY(upload(c, &F.xid, far.xi, s));
    AMG_TRY(upload(c, &F.zetad, far.zeta, s));
    AMG_TRY(level_spectra(c, far, F, false, zscratch, s));
    NearField nf;
    near_field(ks, c->N, kNearM, c->opts.shift, c->opts.scale, nf);
    std::vector<double> w(nf.wn);
    w.insert(w.end(), nf.wm.begin(), nf.wm.end());
    AMG_TRY(upload(c, &c->near_w, w, s));
    AMG_TRY(upload(c, &c->near_rl, nf.rsum_left, s));
    AMG_TRY(upload(c, &c->near_rr, nf.rsum_right, s));
    c->near_rin[0] = nf.rsum_in[0];
    c->near_rin[1] = nf.rsum_in[1];
    AMG_TRY(dalloc(c, &c->ynear, (size_t)(2 * c->N - 1)));
  }
  // coarsest level: LU with partial pivoting (host, FP64), then A_c^{-1} by
  // solving against the identity with those factors; stored column-major
  {
    const TpxLevel& Hc = c->host.back();
    const int m = (int)(2 * Hc.n + 1);
    std::vector<double> A = densify(Hc);
    std::vector<int> piv;
    if (!lu_factor(A, m, piv)) return AMG_EINVAL;
    std::vector<double> inv;
    lu_inverse(A, m, piv, inv);
    double* ai;
    AMG_TRY(upload(c, &ai, inv, s));
    c->lu = {m, ai, nullptr};
  }
  {
    const int ft = c->first_tail;
    const bool band = c->host[ft].has_band(), sym = c->lv[ft].sym;
    for (int l = ft; l < nl; ++l)
      if (c->host[l].has_band() != band || c->lv[l].sym != sym) return AMG_EINVAL;
    c->tail_variant = (band ? TAIL_BAND : 0) | (sym ? TAIL_SYM : 0);
  }
  AMG_TRY(dalloc(c, &c->dpart64, (size_t)maxblocks));
  AMG_TRY(dalloc(c, &c->dpart32, (size_t)maxblocks));
  // residual-norm partials: column blocks of the finest four-step level or
  // the vector chunks of the conjugate-gradient update
  AMG_TRY(dalloc(c, &c->npart,
                 (size_t)std::max(maxblocks, vec_blocks((int64_t)(2 * c->N - 1)))));
  {
    std::vector<LevelDev<double>> v64(nl);
    for (int l = 0; l < nl; ++l) v64[l] = c->lv[l].dev<double>();
    AMG_TRY(dalloc(c, &c->lvdev64, nl));
    HIP_TRY(hipMemcpyAsync(c->lvdev64, v64.data(), nl * sizeof(LevelDev<double>),
                           hipMemcpyHostToDevice, s));
    if (mixed) {
      std::vector<LevelDev<float>> v32(nl);
      for (int l = 0; l < nl; ++l) v32[l] = c->lv[l].dev<float>();
      AMG_TRY(dalloc(c, &c->lvdev32, nl));
      HIP_TRY(hipMemcpyAsync(c->lvdev32, v32.data(), nl * sizeof(LevelDev<float>),
                             hipMemcpyHostToDevice, s));
    }
  }
  c->vc_last = nl - 1;
  c->lu_vc = c->lu;
  if (c->opts.cycle != 2) AMG_TRY(form_sub_vcycle(c, s));
  if (c->opts.cycle == 1 && (c->opts.flags & AMG_FLAG_DEEP_FOLD)) AMG_TRY(form_deep_fold(c, s));
  if (c->opts.cycle == 2) {
    const int ft = c->first_tail;
    c->w_last = nl - 1;
    c->lu_w = c->lu;
    AMG_TRY(form_sub_wcycle(c, s));
    for (int k = 0; k < 2; ++k) {
      std::vector<TailOp> ops;
      tail_visit(ops, ft, k == 0, ft, c->w_last, c->opts.m1, c->opts.m2, c->opts.cycle, ft > 0);
      std::vector<int> raw(ops.size() * 4);
      std::memcpy(raw.data(), ops.data(), raw.size() * sizeof(int));
      int* dev = nullptr;
      AMG_TRY(upload(c, &dev, raw, s));
      c->tail_prog[k] = reinterpret_cast<TailOp*>(dev);
      c->tail_prog_n[k] = (int)ops.size();
    }
  }
  AMG_TRY(dalloc(c, &c->st_dev, 1));
  AMG_TRY(dalloc(c, &c->hist_dev, (size_t)c->opts.max_iter + 2));
  if (mixed) AMG_TRY(dalloc(c, &c->rout, (size_t)(2 * c->N - 1)));
  if (c->opts.inner == AMG_INNER_PCG) {
    const size_t m = (size_t)(2 * c->N - 1);
    AMG_TRY(dalloc(c, &c->cg_p, m));
    AMG_TRY(dalloc(c, &c->cg_q, m));
    AMG_TRY(dalloc(c, &c->cg_rold, m));
    AMG_TRY(dalloc(c, &c->cg_part, (size_t)(2 * vec_blocks((int64_t)m))));
  }
  if (c->opts.inner == AMG_INNER_GMRES) {
    const size_t m = (size_t)(2 * c->N - 1);
    const size_t R = (size_t)c->opts.restart;
    AMG_TRY(dalloc(c, &c->gm_V, (R + 1) * m));
    AMG_TRY(dalloc(c, &c->gm_Z, R * m));
    AMG_TRY(dalloc(c, &c->gm_H, (size_t)(kGmMax + 1) * kGmMax));
    AMG_TRY(dalloc(c, &c->gm_small, (size_t)(kGmMax + 1) * 6));
    AMG_TRY(dalloc(c, &c->gm_part, (size_t)(kGmMax + 1) * vec_blocks((int64_t)m)));
  }
  void* ph = nullptr;
  HIP_TRY(hipHostMalloc(&ph, sizeof(SolveState), hipHostMallocDefault));
  c->st_host = static_cast<SolveState*>(ph);
  HIP_TRY(hipStreamSynchronize(s));
  free_setup_temps(c);
  return AMG_OK;
}

void release(amg_ctx* c) {
  if (!c) return;
  if (c->vgraph) (void)hipGraphExecDestroy(c->vgraph);
  c->vgraph = nullptr;
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->cap_stream = nullptr;
  for (const auto& p : c->dev_allocs) (void)hipFree(p.first);
  c->dev_allocs.clear();
  for (const auto& p : c->spare) (void)hipFree(p.first);
  c->spare.clear();
  c->bump = nullptr;
  // a setup that failed part-way: its stream may still use the temporaries
  // (hipFree waits for the device; the pool would not)
  for (const auto& t : c->setup_temps) (void)hipFree(t.first);
  c->setup_temps.clear();
  if (c->st_host) (void)hipHostFree(c->st_host);
  c->st_host = nullptr;
}

// Static work memory of amg_matvec_noalloc: the FFT buffer of a finest level
// of up to 2^18 intervals (2N complex doubles), its block partials and the
// w_o scalars.  Each device holds its own copy for the life of the process;
// host code must use the per-device address from hipGetSymbolAddress (the
// array's name on the host is only a stand-in).
constexpr size_t kScratchFftBytes = size_t(8) << 20;
constexpr size_t kScratchPartBytes = size_t(32) << 10;
constexpr size_t kScratchBytes = kScratchFftBytes + kScratchPartBytes + 256;
constexpr int64_t kScratchMaxN = int64_t(1) << 18;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device `dev` (current), looked up once.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return AMG_EINVAL;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __LINE__);
    if (!p) return AMG_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return AMG_OK;
}

}  // namespace

namespace {
int setup_impl(const amg_kernel_t* kernel, double delta, int64_t N, const amg_opts_t* opts,
               void* stream, amg_ctx* donor, amg_t* out);
}  // namespace

extern "C" {

void amg_default_opts(amg_opts_t* o) {
  if (!o) return;
  o->m1 = 1;
  o->m2 = 1;
  o->omega_pre = 2.0 / 3.0;
  o->omega_post = 2.0 / 3.0;
  o->coarsest_log2 = 5;
  o->precision = AMG_FP64;
  o->max_iter = 200;
  o->flags = 0;
  o->inner = AMG_INNER_VCYCLE;
  o->shift = 0.0;
  o->scale = 1.0;
  o->restart = 30;
  o->cycle = 1;
}

const char* amg_strerror(int st) {
  switch (st) {
    case AMG_OK: return "ok";
    case AMG_NOT_CONVERGED: return "not converged within max_iter";
    case AMG_DIVERGED: return "diverged (NaN/Inf or residual growth)";
    case AMG_EINVAL: return "invalid argument";
    case AMG_ENOMEM: return "out of memory";
    case AMG_EHIP: return "HIP runtime error";
    case AMG_ENOTSUP: return "not supported by this library";
    default: return "unknown status";
  }
}

int amg_setup(const amg_kernel_t* kernel, double delta, int64_t N, const amg_opts_t* opts,
              void* stream, amg_t* out) {
  return setup_impl(kernel, delta, N, opts, stream, nullptr, out);
}

}  // extern "C"

namespace {

// amg_setup; donor (may be NULL): a handle that is no longer used, on the
// current device, whose device chunks the new hierarchy reuses where they are
// large enough (no hipMalloc / hipFree for a hierarchy of the same shape);
// the donor is destroyed in every case.
int setup_impl(const amg_kernel_t* kernel, double delta, int64_t N, const amg_opts_t* opts,
               void* stream, amg_ctx* donor, amg_t* out) {
  struct DonorGuard {
    amg_ctx* d;
    ~DonorGuard() {
      if (d) (void)amg_destroy(d);
    }
  } dg{donor};
  if (!kernel || !out) return AMG_EINVAL;
  *out = nullptr;
  amg_opts_t o;
  if (opts) o = *opts;
  else amg_default_opts(&o);
  int st = check_opts(&o);
  if (st != AMG_OK) return st;
  const KernelSpec ks = spec_of(kernel, ignores_delta(kernel) ? 0.25 : delta);
  if (!validate(ks, N, o.coarsest_log2).empty()) return AMG_EINVAL;
  if (!ignores_delta(kernel) && !(std::isfinite(delta))) return AMG_EINVAL;
  if (!ks.supported()) return AMG_ENOTSUP;
  amg_ctx* c = new (std::nothrow) amg_ctx();
  if (!c) return AMG_ENOMEM;
  c->N = N;
  c->opts = o;
  c->host_only = (o.flags & AMG_FLAG_HOST_ONLY) != 0;
  c->prof.on = (o.flags & AMG_FLAG_PROFILE) != 0 && !c->host_only;
  c->mixed = o.precision == AMG_MIXED;
  c->kspec = ks;
  if (o.flags & AMG_FLAG_ACCURATE_RESIDUAL) {
    if (kernel->kind != AMG_K_CONST && kernel->kind != AMG_K_WEIGHTED &&
        !is_fractional(kernel->kind)) {
      delete c;
      return AMG_ENOTSUP;
    }
    // finest levels in the small-level kernels keep the plain residual
    c->split = !plan_level(N - 1).tail;
  }
  // Stencil kernels on a device handle form their hierarchy on the device
  // (the same arithmetic, amg_setup.hip); the host keeps the level sizes
  c->gpu_setup = !c->host_only && (kernel->kind == AMG_K_CONST ||
                                    kernel->kind == AMG_K_WEIGHTED ||
                                    is_fractional(kernel->kind));
  // symmetric levels: a symmetric kernel under the shifted rule (the stencil
  // is then exactly symmetric, and Lemma 3.1 keeps it so)
  c->gpu_sym = ks.scheme == SCHEME_SHIFTED &&
               (kernel->kind != AMG_K_WEIGHTED || kernel->wl == kernel->wr);
  try {
    if (c->gpu_setup) {
      const int64_t nc = (int64_t(1) << o.coarsest_log2) - 1;
      for (int64_t n = N - 1;; n = (n - 1) / 2) {
        TpxLevel t;
        t.n = n;
        c->host.push_back(t);
        if (n <= nc) break;
      }
    } else {
      c->host.push_back(finest_level(ks, N));
      if (o.shift != 0.0 || o.scale != 1.0) shift_level(c->host[0], o.shift, o.scale);
      const int64_t nc = (int64_t(1) << o.coarsest_log2) - 1;
      while (c->host.back().n > nc) c->host.push_back(coarsen(c->host.back()));
    }
  } catch (const std::bad_alloc&) {
    delete c;
    return AMG_ENOMEM;
  }
  if (!c->gpu_setup) {
    for (const TpxLevel& t : c->host) {
      for (const auto* v : {&t.a, &t.b, &t.c, &t.d, &t.p, &t.q, &t.xi, &t.zeta})
        for (double x : *v)
          if (!std::isfinite(x)) {
            delete c;
            return AMG_EINVAL;
          }
      if (!(t.a[t.n - 1] != 0.0 && t.d[t.n - 1] != 0.0 && t.o != 0.0)) {
        delete c;
        return AMG_EINVAL;  // Jacobi needs a nonzero diagonal
      }
    }
  }
  if (o.inner == AMG_INNER_PCG && !(c->gpu_setup ? c->gpu_sym : c->host[0].symmetric())) {
    delete c;
    return AMG_EINVAL;  // conjugate gradients needs a symmetric operator
  }
  if (!c->host_only) {
    const hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "hipGetDevice", __LINE__);
    }
    void* sp = nullptr;
    // the first device chunk holds the whole persistent footprint
    c->arena_hint = (size_t)footprint(N, &o,
                                      (kernel->kind == AMG_K_CONST ||
                                       is_fractional(kernel->kind)) &&
                                          ks.scheme == SCHEME_SHIFTED,
                                      kernel->kind == AMG_K_WEAKLY_SINGULAR);
    c->arena_hint += c->arena_hint / 32 + (size_t(2) << 20);
    if (dg.d && dg.d->device == c->device) {
      c->spare = std::move(dg.d->dev_allocs);
      dg.d->dev_allocs.clear();
      dg.d->bump = nullptr;
    }
    st = scratch_address(c->device, &sp);
    if (st == AMG_OK) st = setup_device(c, (hipStream_t)stream);
    if (st != AMG_OK) {
      release(c);
      delete c;
      return st;
    }
    for (const auto& p : c->spare) (void)hipFree(p.first);  // chunks left over
    c->spare.clear();
  }
  *out = c;
  return AMG_OK;
}

}  // namespace

extern "C" {

int amg_destroy(amg_t h) {
  if (!h) return AMG_OK;
  if (!h->host_only) (void)hipSetDevice(h->device);
  release(h);
  delete h;
  return AMG_OK;
}

int amg_num_levels(amg_t h) { return h ? (int)h->host.size() : AMG_EINVAL; }

int64_t amg_level_size(amg_t h, int level) {
  if (!h || level < 0 || level >= (int)h->host.size()) return AMG_EINVAL;
  return 2 * h->host[level].n + 1;
}

int amg_level_band(amg_t h, int level, double* sub, double* main, double* sup) {
  if (!h || level < 0 || level >= (int)h->host.size()) return AMG_EINVAL;
  const TpxLevel& t = h->host[level];
  if (!t.has_band()) return 0;
  for (auto pr : {std::make_pair(sub, &t.bsub), std::make_pair(main, &t.bmain),
                  std::make_pair(sup, &t.bsup)})
    if (pr.first) std::memcpy(pr.first, pr.second->data(), pr.second->size() * sizeof(double));
  return 1;
}

int amg_level_tpx(amg_t h, int level, double* a, double* b, double* c, double* d, double* p,
                  double* q, double* xi, double* zeta, double* o) {
  if (!h || level < 0 || level >= (int)h->host.size()) return AMG_EINVAL;
  const TpxLevel& t = h->host[level];
  if (t.a.empty()) return AMG_ENOTSUP;  // formed on the device (see amg.h)
  auto cp = [](double* dst, const std::vector<double>& v) {
    if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(double));
  };
  cp(a, t.a);
  cp(b, t.b);
  cp(c, t.c);
  cp(d, t.d);
  cp(p, t.p);
  cp(q, t.q);
  cp(xi, t.xi);
  cp(zeta, t.zeta);
  if (o) *o = t.o;
  return AMG_OK;
}

int amg_matvec(amg_t h, const double* x, double* y, void* stream) {
  return amg_level_matvec(h, 0, x, y, stream);
}

int amg_level_matvec(amg_t h, int level, const double* x, double* y, void* stream) {
  if (!h || !x || !y || h->host_only || level < 0 || level >= (int)h->lv.size()) return AMG_EINVAL;
  if (x == y) return AMG_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  return level_matvec64(h, level, x, y, (hipStream_t)stream);
}

int amg_residual(amg_t h, const double* b, const double* x, double* r, void* stream) {
  if (!h || !b || !x || !r || h->host_only || r == b || r == x) return AMG_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  int npart = 1;
  // COL_MV does not write x (x += e is not requested)
  return residual_passes(h, b, const_cast<double*>(x), nullptr, r, nullptr, (hipStream_t)stream,
                         &npart);
}

int amg_matvec_noalloc(amg_t h, const double* x, double* y, void* stream) {
  if (!h || !x || !y || h->host_only || x == y) return AMG_EINVAL;
  if (h->N > kScratchMaxN) {
    if (std::getenv("AMG_DEBUG"))
      std::fprintf(stderr, "amg: amg_matvec_noalloc: N = %lld exceeds the static scratch (N <= %lld)\n",
                   (long long)h->N, (long long)kScratchMaxN);
    return AMG_EINVAL;
  }
  {
    // the block partials of the level's geometry must fit their slot
    const Plan& q = h->lv[0].plan;
    const size_t nb = (size_t)std::max(col_blocks(q.logL1, q.tcols), (1 << q.logL2) / 2);
    if (!q.tail && nb * sizeof(double) > kScratchPartBytes) return AMG_EINVAL;
  }
  HIP_TRY(hipSetDevice(h->device));
  void* sp = nullptr;
  AMG_TRY(scratch_address(h->device, &sp));
  unsigned char* base = static_cast<unsigned char*>(sp);
  FourstepWork<double> wk;
  wk.buf = reinterpret_cast<cplx<double>*>(base);
  wk.part = reinterpret_cast<double*>(base + kScratchFftBytes);
  wk.scal = reinterpret_cast<double*>(base + kScratchFftBytes + kScratchPartBytes);
  return level_matvec<double>(h, 0, x, y, (hipStream_t)stream, wk);
}

int amg_level_matvec_f32(amg_t h, int level, const float* x, float* y, void* stream) {
  if (!h || !x || !y || h->host_only || !h->mixed || level < 0 || level >= (int)h->lv.size())
    return AMG_EINVAL;
  if ((const void*)x == (const void*)y) return AMG_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  return level_matvec<float>(h, level, x, y, (hipStream_t)stream);
}

int amg_vcycle(amg_t h, const void* r, void* e, void* stream) {
  if (!h || !r || !e || h->host_only || r == e) return AMG_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  const LevelRes& L0 = h->lv[0];
  const size_t m = (size_t)(2 * L0.n + 1);
  if (h->mixed) {
    HIP_TRY(hipMemcpyAsync(L0.bf, r, m * sizeof(float), hipMemcpyDeviceToDevice, s));
    AMG_TRY(vcycle_run(h, s));
    HIP_TRY(hipMemcpyAsync(e, L0.uf, m * sizeof(float), hipMemcpyDeviceToDevice, s));
  } else {
    HIP_TRY(hipMemcpyAsync(L0.bd, r, m * sizeof(double), hipMemcpyDeviceToDevice, s));
    AMG_TRY(vcycle_run(h, s));
    HIP_TRY(hipMemcpyAsync(e, L0.ud, m * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return AMG_OK;
}

namespace {

// One solve is: begin (reset the stop state, r_0 = b - A x_0, stop test), then
// rounds of (V-cycle, x += e fused into r = b - A x, stop test) until the
// device-side state says done; every enqueue ends with an asynchronous copy of
// the 40-byte state to pinned host memory.
int solve_begin(amg_t h, const double* b, double* x, double tol, hipStream_t s) {
  SolveState init{};
  init.cg_first = 1;
  *h->st_host = init;
  HIP_TRY(hipMemcpyAsync(h->st_dev, h->st_host, sizeof(SolveState), hipMemcpyHostToDevice, s));
  AMG_TRY(outer_residual(h, b, x, nullptr, tol, s));
  HIP_TRY(hipMemcpyAsync(h->st_host, h->st_dev, sizeof(SolveState), hipMemcpyDeviceToHost, s));
  h->gm_j = 0;
  h->cg_restart = false;
  return AMG_OK;
}

// Conjugate gradients preconditioned by the V-cycle.  The residual r lives
// where the V-cycle reads its right-hand side (level 0's b; in the mixed form
// r is FP64 in `rout` with its FP32 copy in level 0's b), z = B r is level 0's
// u, and every scalar stays on the device.
// z = B r, then the new direction (first: p = z; otherwise Polak-Ribiere).
int pcg_precondition(amg_t h, int first, hipStream_t s) {
  const LevelRes& L0 = h->lv[0];
  const int64_t m = 2 * h->N - 1;
  const int nb = vec_blocks(m);
  const size_t v0 = h->prof.mark(s);
  AMG_TRY(vcycle_run(h, s));
  h->prof.span(PK_VCYCLE, v0, h->prof.mark(s));
  const double* rold = first ? nullptr : h->cg_rold;
  if (h->mixed)
    HIP_TRY(launch_vdot<float>(h->rout, L0.uf, rold, m, h->cg_part, s));
  else
    HIP_TRY(launch_vdot<double>(L0.bd, L0.ud, rold, m, h->cg_part, s));
  HIP_TRY(launch_cg_scalar(h->st_dev, h->cg_part, nb, first ? CG_INIT : CG_BETA, s));
  if (h->mixed)
    HIP_TRY(launch_cg_dir<float>(h->st_dev, h->cg_p, L0.uf, m, first, s));
  else
    HIP_TRY(launch_cg_dir<double>(h->st_dev, h->cg_p, L0.ud, m, first, s));
  return AMG_OK;
}

// q = A p, alpha, x += alpha p, r -= alpha q (and its FP32 copy), stop test.
int pcg_step(amg_t h, double* x, double tol, hipStream_t s) {
  const LevelRes& L0 = h->lv[0];
  const int64_t m = 2 * h->N - 1;
  const size_t v0 = h->prof.mark(s);
  AMG_TRY(level_matvec64(h, 0, h->cg_p, h->cg_q, s));
  HIP_TRY(launch_vdot<double>(h->cg_p, h->cg_q, nullptr, m, h->cg_part, s));
  HIP_TRY(launch_cg_scalar(h->st_dev, h->cg_part, vec_blocks(m), CG_ALPHA, s));
  double* r = h->mixed ? h->rout : L0.bd;
  HIP_TRY(launch_cg_update(h->st_dev, x, h->cg_p, r, h->cg_rold, h->cg_q, h->mixed ? L0.bf : nullptr,
                           m, h->npart, s));
  HIP_TRY(launch_finish(h->st_dev, h->npart, vec_blocks(m), tol, h->opts.max_iter, h->hist_dev, s,
                        1));
  h->prof.span(PK_OUTER, v0, h->prof.mark(s));
  return AMG_OK;
}

// Restarted flexible GMRES, one Arnoldi step per round (one V-cycle):
// z_j = B v_j, w = A z_j, two classical Gram-Schmidt passes against v_0..v_j,
// Givens rotation and residual estimate; v_{j+1} = w / h_{j+1,j}.  The round
// after a cycle ended (estimate below tol, restart length, max_iter) forms
// x += Z y and the true residual b - A x with its stop test; the next round
// starts a new cycle from that residual.  The residual r lives where the
// V-cycle reads its right-hand side (level 0's b; mixed: `rout`).
int gmres_round(amg_t h, const double* b, double* x, double tol, hipStream_t s) {
  const LevelRes& L0 = h->lv[0];
  const int64_t m = 2 * h->N - 1;
  const int nb = vec_blocks(m);
  double* g = h->gm_small;
  double* cs = g + (kGmMax + 1);
  double* sn = cs + (kGmMax + 1);
  double* hcur = sn + (kGmMax + 1);
  double* y = hcur + (kGmMax + 1);
  double* hn = y + (kGmMax + 1);
  double* vin64 = h->mixed ? nullptr : L0.bd;
  float* vin32 = h->mixed ? L0.bf : nullptr;
  const size_t v0 = h->prof.mark(s);
  if (h->st_host->cycle_end) {
    HIP_TRY(launch_gm_update(h->st_dev, h->gm_H, g, h->gm_j, y, x, h->gm_Z, m, s));
    AMG_TRY(outer_residual(h, b, x, nullptr, tol, s, true));
    h->gm_j = 0;
    h->prof.span(PK_OUTER, v0, h->prof.mark(s));
    return AMG_OK;
  }
  const int j = h->gm_j;
  if (j == 0)
    HIP_TRY(launch_gm_start(h->st_dev, h->mixed ? h->rout : L0.bd, h->gm_V, g, m, vin64, vin32, s));
  AMG_TRY(vcycle_run(h, s));
  const size_t v1 = h->prof.mark(s);
  double* z = h->gm_Z + (int64_t)j * m;
  if (h->mixed)
    HIP_TRY(launch_copy_f2d(L0.uf, z, m, s));
  else
    HIP_TRY(hipMemcpyAsync(z, L0.ud, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, s));
  double* w = h->gm_V + (int64_t)(j + 1) * m;
  AMG_TRY(level_matvec64(h, 0, z, w, s));
  double* Hj = h->gm_H + (int64_t)j * (kGmMax + 1);
  for (int pass = 0; pass < 2; ++pass) {
    HIP_TRY(launch_gm_dot(h->gm_V, j + 1, w, m, h->gm_part, s));
    HIP_TRY(launch_gm_reduce(h->st_dev, h->gm_part, nb, j + 1, hcur, Hj, pass, s));
    HIP_TRY(launch_gm_axpy(h->st_dev, w, h->gm_V, hcur, j + 1, m, pass ? h->npart : nullptr, s));
  }
  HIP_TRY(launch_gm_givens(h->st_dev, h->gm_H, j, cs, sn, g, hn, h->npart, nb, tol,
                           h->opts.max_iter, h->opts.restart, h->hist_dev, s));
  HIP_TRY(launch_gm_scale(h->st_dev, w, hn, m, vin64, vin32, s));
  h->gm_j = j + 1;
  h->prof.span(PK_VCYCLE, v0, v1);
  h->prof.span(PK_OUTER, v1, h->prof.mark(s));
  return AMG_OK;
}

// Waits for a round's stop test by polling the stream instead of a blocking
// synchronise (whose wake-up latency is of the order of a small level's whole
// V-cycle): the calling thread spins while the round runs.
hipError_t round_wait(hipStream_t s) {
  for (;;) {
    const hipError_t e = hipStreamQuery(s);
    if (e != hipErrorNotReady) return e;
  }
}

// The stationary iteration's round ends with the stop test writing the state
// to pinned host memory, so the host can watch that copy (the iteration count
// advanced, or done) and queue the next round before the stream has reported
// completion; the stream is still queried every so often, so that a failure
// ends the wait.  Words are written whole, and iter advances only when done
// stays 0, so either change is a consistent signal.
hipError_t state_wait(const SolveState* host, int prev_iter, hipStream_t s) {
  const volatile SolveState* hs = host;
  for (unsigned k = 1;; ++k) {
    if (hs->done || hs->iter != prev_iter) return hipSuccess;
    if ((k & 255) == 0) {
      const hipError_t e = hipStreamQuery(s);
      if (e != hipErrorNotReady) return e;
    }
  }
}

// Enqueues the work up to the next stop test; round counts the calls since
// solve_begin (whose residual and stop test come first).
int solve_round(amg_t h, const double* b, double* x, double tol, hipStream_t s, int round) {
  if (h->opts.inner == AMG_INNER_PCG) {
    if (h->st_host->cycle_end) {
      // the recurrence's residual passed the test: b - A x decides; if it has
      // not passed, CG restarts from it
      const size_t v0 = h->prof.mark(s);
      AMG_TRY(outer_residual(h, b, x, nullptr, tol, s, true, true));
      h->prof.span(PK_OUTER, v0, h->prof.mark(s));
      h->cg_restart = true;
    } else {
      AMG_TRY(pcg_precondition(h, round == 0 || h->cg_restart, s));
      AMG_TRY(pcg_step(h, x, tol, s));
      h->cg_restart = false;
    }
  } else if (h->opts.inner == AMG_INNER_GMRES) {
    AMG_TRY(gmres_round(h, b, x, tol, s));
  } else {
    const void* e = h->mixed ? (const void*)h->lv[0].uf : (const void*)h->lv[0].ud;
    const size_t v0 = h->prof.mark(s);
    AMG_TRY(vcycle_run(h, s));
    const size_t v1 = h->prof.mark(s);
    AMG_TRY(outer_residual(h, b, x, e, tol, s, false, false, h->st_host));
    const size_t v2 = h->prof.mark(s);
    h->prof.span(PK_VCYCLE, v0, v1);
    h->prof.span(PK_OUTER, v1, v2);
    return AMG_OK;  // the stop test published the state
  }
  HIP_TRY(launch_publish(h->st_dev, h->st_host, s));
  return AMG_OK;
}

// After the stream has been synchronised: residual history and results.
int solve_end(amg_t h, hipStream_t s, int* iters, double* relres) {
  h->prof.collect();
  const SolveState st = *h->st_host;
  h->last_iters = st.iter;
  h->hist.assign((size_t)st.iter + 1, 0.0);
  HIP_TRY(hipMemcpyAsync(h->hist.data(), h->hist_dev, h->hist.size() * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (iters) *iters = st.iter;
  if (relres) *relres = st.relres;
  return st.status;
}

// Internal streams (default priority) for amg_solve_batch, one pool per device.
struct StreamPool {
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;  // one per stream (join) + one (fork)
};
std::mutex g_pool_mu;
std::unordered_map<int, StreamPool> g_pools;
constexpr int kBatchStreams = 8;

int get_pool(int device, StreamPool** out) {
  std::lock_guard<std::mutex> g(g_pool_mu);
  StreamPool& p = g_pools[device];
  if (p.streams.empty()) {
    for (int i = 0; i < kBatchStreams; ++i) {
      hipStream_t st;
      HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      p.streams.push_back(st);
    }
    for (int i = 0; i <= kBatchStreams; ++i) {
      hipEvent_t ev;
      HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      p.events.push_back(ev);
    }
  }
  *out = &p;
  return AMG_OK;
}

}  // namespace

int amg_solve(amg_t h, const double* b, double* x, double tol, void* stream, int* iters,
              double* relres) {
  if (!h || !b || !x || h->host_only || b == x) return AMG_EINVAL;
  if (!(tol > 0.0) || !std::isfinite(tol)) return AMG_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  AMG_TRY(solve_begin(h, b, x, tol, s));
  const bool watch = h->opts.inner == AMG_INNER_VCYCLE;  // its rounds publish their own state
  int prev_iter = 0;
  for (int round = 0;; ++round) {
    if (watch && round > 0)
      HIP_TRY(state_wait(h->st_host, prev_iter, s));
    else
      HIP_TRY(round_wait(s));
    if (h->st_host->done) break;
    prev_iter = h->st_host->iter;
    AMG_TRY(solve_round(h, b, x, tol, s, round));
  }
  HIP_TRY(round_wait(s));  // the last round complete before its state is read
  return solve_end(h, s, iters, relres);
}

int amg_bdf4_step(amg_t h, const double* u1, const double* u2, const double* u3,
                  const double* u4, const double* src, double* x, double tol, void* stream,
                  int* iters, double* relres) {
  if (!h || h->host_only || !u1 || !u2 || !u3 || !u4 || !x || x == src) return AMG_EINVAL;
  if (!(tol > 0.0) || !std::isfinite(tol)) return AMG_EINVAL;
  HIP_TRY(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t m = 2 * h->N - 1;
  if (!h->step_b) AMG_TRY(dalloc(h, &h->step_b, (size_t)m));
  HIP_TRY(launch_bdf4_rhs(u1, u2, u3, u4, src, h->step_b, m, s));
  if (x != u1) HIP_TRY(hipMemcpyAsync(x, u1, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, s));
  return amg_solve(h, h->step_b, x, tol, stream, iters, relres);
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Batched rounds (amg_solve_batch): every launch covers all instances of one
// (precision, level size, pass, mode) group, one block row per instance, with
// that instance's own arguments and buffers; gates in the instances' solve
// states decide who takes part (finished instances, and the CG step vs the
// check of b - A x).  A round is: the CG checks, one V-cycle over every
// instance (descending level sizes, the small levels of all instances in one
// launch, ascending sizes), the stationary instances' x += e with b - A x and
// stop test, and the CG instances' step (direction, A p, update, stop test).
// Per instance it is the same sequence of kernels and arithmetic as its solo
// solve, so results are bitwise those of amg_solve.
// ---------------------------------------------------------------------------
bool batchable(const amg_ctx* c) {
  if (c->opts.cycle != 1 || c->split || c->prof.on) return false;
  if (c->opts.inner != AMG_INNER_VCYCLE && c->opts.inner != AMG_INNER_PCG) return false;
  for (const LevelRes& R : c->lv)
    if (R.bmaind) return false;  // band levels (weakly singular model)
  return true;
}

// A growing host-side list of argument records, uploaded as one block.
struct ArgArena {
  std::vector<unsigned char> host;
  size_t put(const void* p, size_t bytes) {
    const size_t off = (host.size() + 255) & ~size_t(255);
    host.resize(off + bytes);
    std::memcpy(host.data() + off, p, bytes);
    return off;
  }
};

using Launch = std::function<hipError_t(unsigned char* dev, hipStream_t)>;

struct BatchPlan {
  std::vector<Launch> round;   // launches of one round, in order
  ArgArena arena;
  void* dev = nullptr;
  size_t dev_bytes = 0;
};

template <typename T>
struct PrecTag {};

template <typename T>
void add_pass_group(BatchPlan& P, int pass, int mode, const LevelDev<T>& geom,
                    const std::vector<PassArgs<T>>& args, const Twiddles<T>& tw) {
  if (args.empty()) return;
  const size_t off = P.arena.put(args.data(), args.size() * sizeof(PassArgs<T>));
  const int count = (int)args.size();
  const LevelDev<T> g = geom;
  const Twiddles<T> t = tw;
  P.round.push_back([=](unsigned char* dev, hipStream_t s) {
    const PassArgs<T>* a = reinterpret_cast<const PassArgs<T>*>(dev + off);
    if (pass == 0) return launch_col_fwd_batch<T>(mode, g, a, count, t, s);
    if (pass == 1) return launch_row_batch<T>(g, a, count, t, s);
    return launch_col_inv_batch<T>(mode, g, a, count, t, s);
  });
}

template <typename T>
void add_tail_matvec_group(BatchPlan& P, int cmode, int emode, const std::vector<PassArgs<T>>& args,
                           const Twiddles<T>& tw) {
  if (args.empty()) return;
  const size_t off = P.arena.put(args.data(), args.size() * sizeof(PassArgs<T>));
  const int count = (int)args.size();
  const Twiddles<T> t = tw;
  P.round.push_back([=](unsigned char* dev, hipStream_t s) {
    return launch_tail_matvec_batch<T>(cmode, emode,
                                       reinterpret_cast<const PassArgs<T>*>(dev + off), count, t, s);
  });
}

template <typename T>
PassArgs<T> pass_args(amg_ctx* c, int l, const ColIn<T>& in, const EpiOut<T>& out, int gate,
                      bool fp64_outer) {
  PassArgs<T> a{};
  a.lv = c->lv[l].template dev<T>();
  a.in = in;
  a.out = out;
  a.buf = buf_of<T>(c);
  a.part = dpart_of<T>(c);
  a.npart = col_blocks(a.lv.logL1, a.lv.tcols);
  a.xin = out.xin;
  a.npart_out = c->npart;
  a.st = c->st_dev;
  a.gate = gate;
  (void)fp64_outer;
  return a;
}

// Four-step matvec sweeps of one level size for a set of (instance, level)
// pairs of one precision: groups by pass-1 mode and by symmetry (row pass).
template <typename T>
struct SweepItem {
  amg_ctx* c;
  int l;
  int cmode, emode;
  ColIn<T> in;
  EpiOut<T> out;
  int gate;
};
template <typename T>
void add_sweep_geom(BatchPlan& P, const std::vector<SweepItem<T>>& items);

// Items of one level size may differ in geometry (hierarchies set up before
// and after a change of plan): one set of launches per geometry.
template <typename T>
void add_sweep(BatchPlan& P, const std::vector<SweepItem<T>>& items) {
  std::vector<std::pair<int, int>> geoms;
  for (const auto& it : items) {
    const Plan& q = it.c->lv[it.l].plan;
    if (std::find(geoms.begin(), geoms.end(), std::make_pair(q.logL1, q.tcols)) == geoms.end())
      geoms.push_back({q.logL1, q.tcols});
  }
  for (const auto& g : geoms) {
    std::vector<SweepItem<T>> part;
    for (const auto& it : items) {
      const Plan& q = it.c->lv[it.l].plan;
      if (q.logL1 == g.first && q.tcols == g.second) part.push_back(it);
    }
    add_sweep_geom<T>(P, part);
  }
}

template <typename T>
void add_sweep_geom(BatchPlan& P, const std::vector<SweepItem<T>>& items) {
  if (items.empty()) return;
  const Twiddles<T>& tw = tw_of<T>(items[0].c);
  // pass 1 by prologue mode
  for (int cm : {COL_MV, COL_PRE, COL_PRE_RESTRICT, COL_PROLONG, COL_OUTER_UPDATE}) {
    std::vector<PassArgs<T>> v;
    LevelDev<T> geom{};
    for (const auto& it : items)
      if (it.cmode == cm) {
        v.push_back(pass_args<T>(it.c, it.l, it.in, it.out, it.gate, false));
        geom = v.back().lv;
      }
    add_pass_group<T>(P, 0, cm, geom, v, tw);
  }
  for (int sy : {0, 1}) {
    std::vector<PassArgs<T>> v;
    LevelDev<T> geom{};
    for (const auto& it : items) {
      PassArgs<T> a = pass_args<T>(it.c, it.l, it.in, it.out, it.gate, false);
      if ((a.lv.sym != 0) == (sy != 0)) {
        v.push_back(a);
        geom = a.lv;
      }
    }
    add_pass_group<T>(P, 1, 1, geom, v, tw);
  }
  for (int em : {EPI_MV, EPI_RESID, EPI_SMOOTH, EPI_OUTER}) {
    std::vector<PassArgs<T>> v;
    LevelDev<T> geom{};
    for (const auto& it : items)
      if (it.emode == em) {
        v.push_back(pass_args<T>(it.c, it.l, it.in, it.out, it.gate, false));
        geom = v.back().lv;
      }
    add_pass_group<T>(P, 2, em, geom, v, tw);
  }
}

// One V-cycle (Algorithm 2, as vcycle_dev) of every instance of precision T.
template <typename T>
void plan_vcycle(BatchPlan& P, const std::vector<amg_ctx*>& cs, const std::vector<int>& gates) {
  std::vector<int> idx;
  for (size_t i = 0; i < cs.size(); ++i)
    if ((sizeof(T) == 4) == cs[i]->mixed) idx.push_back((int)i);
  if (idx.empty()) return;
  int maxlog = 0;
  for (int i : idx) maxlog = std::max(maxlog, cs[i]->lv[0].plan.logL);
  const int m1 = cs[idx[0]]->opts.m1, m2 = cs[idx[0]]->opts.m2;
  // descent: level sizes from the largest down to the four-step range's end
  for (int lg = maxlog; lg > kTailLog; --lg) {
    for (int sweep = 1; sweep <= m1; ++sweep) {
      std::vector<SweepItem<T>> items;
      for (int i : idx) {
        amg_ctx* c = cs[i];
        for (int l = 0; l < c->first_tail; ++l) {
          if (c->lv[l].plan.logL != lg) continue;
          const LevelDev<T> d = c->lv[l].template dev<T>();
          SweepItem<T> it{};
          it.c = c;
          it.l = l;
          it.gate = gates[i];
          it.out.xin = d.u;
          it.out.omega = (T)c->opts.omega_pre;
          it.emode = sweep == m1 ? EPI_RESID : EPI_SMOOTH;
          if (sweep == 1) {
            it.in.omega = (T)c->opts.omega_pre;
            it.cmode = l == 0 ? COL_PRE : COL_PRE_RESTRICT;
            if (l > 0) it.in.x = c->lv[l - 1].template dev<T>().r;
          } else {
            it.cmode = COL_MV;
            it.in.x = d.u;
          }
          items.push_back(it);
        }
      }
      add_sweep<T>(P, items);
    }
  }
  // the small levels and the coarsest solve, one block per instance
  {
    // instances with the deep fold: one product per instance, one launch
    std::vector<FoldArgs<T>> v;
    int mmax = 0;
    for (int i : idx) {
      amg_ctx* c = cs[i];
      if (!c->deep_m) continue;
      FoldArgs<T> a{};
      a.rf = c->lv[c->first_tail - 1].template dev<T>().r;
      a.M = deep_of<T>(c);
      a.u = c->lv[c->first_tail].template dev<T>().u;
      a.m = c->deep_m;
      a.st = c->st_dev;
      a.gate = gates[i];
      v.push_back(a);
      mmax = std::max(mmax, a.m);
    }
    if (!v.empty()) {
      const size_t off = P.arena.put(v.data(), v.size() * sizeof(FoldArgs<T>));
      const int count = (int)v.size();
      P.round.push_back([=](unsigned char* dev, hipStream_t s) {
        return launch_fold_gemv_batch<T>(reinterpret_cast<const FoldArgs<T>*>(dev + off), count,
                                         mmax, s);
      });
    }
  }
  for (int variant = 0; variant < 4; ++variant) {
    std::vector<TailArgs<T>> v;
    for (int i : idx) {
      amg_ctx* c = cs[i];
      if (c->deep_m || c->tail_variant != variant) continue;
      TailArgs<T> a{};
      a.levels = lvdev_of<T>(c);
      a.first = c->first_tail;
      a.last = c->vc_last;
      a.rf = c->first_tail > 0 ? c->lv[c->first_tail - 1].template dev<T>().r : nullptr;
      a.m1 = c->opts.m1;
      a.m2 = c->opts.m2;
      a.wpre = (T)c->opts.omega_pre;
      a.wpost = (T)c->opts.omega_post;
      a.lu = c->lu_vc;
      a.st = c->st_dev;
      a.gate = gates[i];
      v.push_back(a);
    }
    if (v.empty()) continue;
    const size_t off = P.arena.put(v.data(), v.size() * sizeof(TailArgs<T>));
    const int count = (int)v.size();
    const Twiddles<T> tw = tw_of<T>(cs[idx[0]]);
    P.round.push_back([=](unsigned char* dev, hipStream_t s) {
      return launch_tail_vcycle_batch<T>(reinterpret_cast<const TailArgs<T>*>(dev + off), count,
                                         variant, tw, s);
    });
  }
  // ascent
  for (int lg = kTailLog + 1; lg <= maxlog; ++lg) {
    for (int sweep = 0; sweep < m2; ++sweep) {
      std::vector<SweepItem<T>> items;
      for (int i : idx) {
        amg_ctx* c = cs[i];
        for (int l = 0; l < c->first_tail; ++l) {
          if (c->lv[l].plan.logL != lg) continue;
          const LevelDev<T> d = c->lv[l].template dev<T>();
          SweepItem<T> it{};
          it.c = c;
          it.l = l;
          it.gate = gates[i];
          it.out.xin = d.u;
          it.out.omega = (T)c->opts.omega_post;
          it.emode = EPI_SMOOTH;
          if (sweep == 0) {
            it.cmode = COL_PROLONG;
            it.in.x = c->lv[l + 1].template dev<T>().u;
          } else {
            it.cmode = COL_MV;
            it.in.x = d.u;
          }
          items.push_back(it);
        }
      }
      add_sweep<T>(P, items);
    }
  }
}

// FP64 finest-level products of the instances in `sel`: four-step ones by
// level size, tail-size ones in one launch.  mk(c, i) gives (cmode, emode,
// in, out) of instance i.
template <typename F>
void plan_fp64_finest(BatchPlan& P, const std::vector<amg_ctx*>& cs, const std::vector<int>& sel,
                      int gate, F&& mk) {
  if (sel.empty()) return;
  int maxlog = 0;
  for (int i : sel) maxlog = std::max(maxlog, cs[i]->lv[0].plan.logL);
  for (int lg = maxlog; lg > kTailLog; --lg) {
    std::vector<SweepItem<double>> items;
    for (int i : sel) {
      amg_ctx* c = cs[i];
      if (c->lv[0].plan.tail || c->lv[0].plan.logL != lg) continue;
      SweepItem<double> it{};
      it.c = c;
      it.l = 0;
      it.gate = gate;
      mk(c, i, it.cmode, it.emode, it.in, it.out);
      items.push_back(it);
    }
    add_sweep<double>(P, items);
  }
  for (int cm : {COL_MV, COL_OUTER_UPDATE})
    for (int em : {EPI_MV, EPI_OUTER}) {
      std::vector<PassArgs<double>> v;
      for (int i : sel) {
        amg_ctx* c = cs[i];
        if (!c->lv[0].plan.tail) continue;
        int cmode, emode;
        ColIn<double> in{};
        EpiOut<double> out{};
        mk(c, i, cmode, emode, in, out);
        if (cmode != cm || emode != em) continue;
        PassArgs<double> a = pass_args<double>(c, 0, in, out, gate, true);
        v.push_back(a);
      }
      if (!v.empty()) add_tail_matvec_group<double>(P, cm, em, v, cs[sel[0]]->tw64);
    }
}

int build_batch_plan(BatchPlan& P, const std::vector<amg_ctx*>& cs,
                     const std::vector<const double*>& bs, const std::vector<double*>& xs,
                     const std::vector<double>& tols) {
  P.round.clear();
  P.arena.host.clear();
  const int n = (int)cs.size();
  std::vector<int> stat, cg;
  for (int i = 0; i < n; ++i) (cs[i]->opts.inner == AMG_INNER_PCG ? cg : stat).push_back(i);
  auto outer_in = [&](amg_ctx* c, int i, bool update, ColIn<double>& in, EpiOut<double>& out) {
    const LevelRes& L0 = c->lv[0];
    out.xin = xs[i];
    out.bo = bs[i];
    out.ro = c->mixed ? c->rout : L0.bd;
    out.r32 = c->mixed ? L0.bf : nullptr;
    if (update) {
      in.xo = xs[i];
      in.e = c->mixed ? (const void*)L0.uf : (const void*)L0.ud;
      in.e_is_float = c->mixed ? 1 : 0;
    } else {
      in.x = xs[i];
    }
  };
  // 1. CG: the check of b - A x where the recurrence passed
  plan_fp64_finest(P, cs, cg, GATE_CG_CHECK,
                   [&](amg_ctx* c, int i, int& cm, int& em, ColIn<double>& in, EpiOut<double>& out) {
                     cm = COL_MV;
                     em = EPI_OUTER;
                     outer_in(c, i, false, in, out);
                   });
  {
    std::vector<FinishArgs> v;
    for (int i : cg) {
      amg_ctx* c = cs[i];
      FinishArgs a{};
      a.st = c->st_dev;
      a.gate = GATE_CG_CHECK;
      a.part = c->npart;
      a.npart = c->lv[0].plan.tail ? 1 : col_blocks(c->lv[0].plan.logL1, c->lv[0].plan.tcols);
      a.tol = tols[i];
      a.max_iter = c->opts.max_iter;
      a.hist = c->hist_dev;
      a.verify = 1;  // the stall rule
      a.host = c->st_host;
      v.push_back(a);
    }
    if (!v.empty()) {
      const size_t off = P.arena.put(v.data(), v.size() * sizeof(FinishArgs));
      const int count = (int)v.size();
      P.round.push_back([=](unsigned char* dev, hipStream_t s) {
        return launch_gm_check_batch(reinterpret_cast<const FinishArgs*>(dev + off), count, s);
      });
    }
  }
  // 2. one V-cycle per instance (stationary: every round; CG: in its step)
  std::vector<int> gates(n);
  for (int i = 0; i < n; ++i) gates[i] = cs[i]->opts.inner == AMG_INNER_PCG ? GATE_CG_STEP : GATE_ACTIVE;
  plan_vcycle<float>(P, cs, gates);
  plan_vcycle<double>(P, cs, gates);
  // 3. stationary: x += e, r = b - A x, stop test
  plan_fp64_finest(P, cs, stat, GATE_ACTIVE,
                   [&](amg_ctx* c, int i, int& cm, int& em, ColIn<double>& in, EpiOut<double>& out) {
                     cm = COL_OUTER_UPDATE;
                     em = EPI_OUTER;
                     outer_in(c, i, true, in, out);
                   });
  auto add_finish = [&](const std::vector<int>& sel, int gate, int verify, bool vecparts) {
    std::vector<FinishArgs> v;
    for (int i : sel) {
      amg_ctx* c = cs[i];
      FinishArgs a{};
      a.st = c->st_dev;
      a.gate = gate;
      a.part = c->npart;
      a.npart = vecparts ? vec_blocks(2 * c->N - 1)
                         : (c->lv[0].plan.tail ? 1
                                               : col_blocks(c->lv[0].plan.logL1, c->lv[0].plan.tcols));
      a.tol = tols[i];
      a.max_iter = c->opts.max_iter;
      a.hist = c->hist_dev;
      a.verify = verify;
      a.host = c->st_host;
      v.push_back(a);
    }
    if (v.empty()) return;
    const size_t off = P.arena.put(v.data(), v.size() * sizeof(FinishArgs));
    const int count = (int)v.size();
    P.round.push_back([=](unsigned char* dev, hipStream_t s) {
      return launch_finish_batch(reinterpret_cast<const FinishArgs*>(dev + off), count, s);
    });
  };
  add_finish(stat, GATE_ACTIVE, 0, false);
  // 4. CG step: z = B r was formed above; direction, A p, update, stop test
  if (!cg.empty()) {
    int64_t mmax = 0;
    for (int i : cg) mmax = std::max<int64_t>(mmax, 2 * cs[i]->N - 1);
    for (int prec = 0; prec < 2; ++prec) {  // 0: FP64 z, 1: FP32 z
      std::vector<VdotArgs> vd;
      std::vector<CgArgs> cga;
      for (int i : cg) {
        amg_ctx* c = cs[i];
        if ((prec == 1) != c->mixed) continue;
        const LevelRes& L0 = c->lv[0];
        VdotArgs a{};
        a.st = c->st_dev;
        a.gate = GATE_CG_STEP;
        a.a = c->mixed ? c->rout : L0.bd;
        a.z = c->mixed ? (const void*)L0.uf : (const void*)L0.ud;
        a.c = c->cg_rold;
        a.m = 2 * c->N - 1;
        a.part = c->cg_part;
        vd.push_back(a);
        CgArgs g{};
        g.st = c->st_dev;
        g.gate = GATE_CG_STEP;
        g.part = c->cg_part;
        g.nb = vec_blocks(a.m);
        g.p = c->cg_p;
        g.z = a.z;
        g.m = a.m;
        cga.push_back(g);
      }
      if (vd.empty()) continue;
      const size_t ov = P.arena.put(vd.data(), vd.size() * sizeof(VdotArgs));
      const size_t og = P.arena.put(cga.data(), cga.size() * sizeof(CgArgs));
      const int count = (int)vd.size();
      P.round.push_back([=](unsigned char* dev, hipStream_t s) {
        const VdotArgs* a = reinterpret_cast<const VdotArgs*>(dev + ov);
        return prec ? launch_vdot_batch<float>(a, count, mmax, s)
                    : launch_vdot_batch<double>(a, count, mmax, s);
      });
      P.round.push_back([=](unsigned char* dev, hipStream_t s) {
        return launch_cg_scalar_batch(reinterpret_cast<const CgArgs*>(dev + og), count, CG_AUTO, s);
      });
      P.round.push_back([=](unsigned char* dev, hipStream_t s) {
        const CgArgs* g = reinterpret_cast<const CgArgs*>(dev + og);
        return prec ? launch_cg_dir_batch<float>(g, count, mmax, s)
                    : launch_cg_dir_batch<double>(g, count, mmax, s);
      });
    }
    // q = A p (FP64)
    plan_fp64_finest(P, cs, cg, GATE_CG_STEP,
                     [&](amg_ctx* c, int i, int& cm, int& em, ColIn<double>& in, EpiOut<double>& out) {
                       (void)i;
                       cm = COL_MV;
                       em = EPI_MV;
                       in.x = c->cg_p;
                       out.xin = c->cg_p;
                       out.y = c->cg_q;
                     });
    std::vector<VdotArgs> vd;
    std::vector<CgArgs> cga;
    for (int i : cg) {
      amg_ctx* c = cs[i];
      const LevelRes& L0 = c->lv[0];
      VdotArgs a{};
      a.st = c->st_dev;
      a.gate = GATE_CG_STEP;
      a.a = c->cg_p;
      a.z = c->cg_q;
      a.c = nullptr;
      a.m = 2 * c->N - 1;
      a.part = c->cg_part;
      vd.push_back(a);
      CgArgs g{};
      g.st = c->st_dev;
      g.gate = GATE_CG_STEP;
      g.part = c->cg_part;
      g.nb = vec_blocks(a.m);
      g.x = xs[i];
      g.p = c->cg_p;
      g.r = c->mixed ? c->rout : L0.bd;
      g.r_old = c->cg_rold;
      g.q = c->cg_q;
      g.r32 = c->mixed ? L0.bf : nullptr;
      g.m = a.m;
      g.npart = c->npart;
      cga.push_back(g);
    }
    const size_t ov = P.arena.put(vd.data(), vd.size() * sizeof(VdotArgs));
    const size_t og = P.arena.put(cga.data(), cga.size() * sizeof(CgArgs));
    const int count = (int)vd.size();
    P.round.push_back([=](unsigned char* dev, hipStream_t s) {
      return launch_vdot_batch<double>(reinterpret_cast<const VdotArgs*>(dev + ov), count, mmax, s);
    });
    P.round.push_back([=](unsigned char* dev, hipStream_t s) {
      return launch_cg_scalar_batch(reinterpret_cast<const CgArgs*>(dev + og), count, CG_ALPHA, s);
    });
    P.round.push_back([=](unsigned char* dev, hipStream_t s) {
      return launch_cg_update_batch(reinterpret_cast<const CgArgs*>(dev + og), count, mmax, s);
    });
    add_finish(cg, GATE_CG_STEP, 1, true);
  }
  return AMG_OK;
}

int run_batch_plan(BatchPlan& P, hipStream_t s) {
  const size_t need = P.arena.host.size();
  if (need > P.dev_bytes) {
    if (P.dev) (void)hipFree(P.dev);
    P.dev = nullptr;
    P.dev_bytes = 0;
    const size_t grow = need + need / 2;  // rebuilt plans of a server vary in size
    if (hipMalloc(&P.dev, grow) != hipSuccess) return AMG_ENOMEM;
    P.dev_bytes = grow;
  }
  HIP_TRY(hipMemcpyAsync(P.dev, P.arena.host.data(), need, hipMemcpyHostToDevice, s));
  // the tables must be in place before the round reads them; pageable source
  // memory: the copy has been staged when the call returns
  return AMG_OK;
}

// The round's launches captured into a graph on an internal stream (the
// tables stay in place until the next rebuild); replayed on the caller's
// stream.
int capture_round(BatchPlan& P, hipGraphExec_t* out) {
  *out = nullptr;
  hipStream_t cap = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  int st = AMG_OK;
  if (e == hipSuccess) {
    for (const Launch& L : P.round) {
      const hipError_t le = L(static_cast<unsigned char*>(P.dev), cap);
      if (le != hipSuccess) {
        st = hip_fail(le, "batched launch (capture)", __LINE__);
        break;
      }
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    if (st == AMG_OK && e == hipSuccess) {
      e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
      if (e != hipSuccess) *out = nullptr;
    }
    if (g) (void)hipGraphDestroy(g);
  }
  (void)hipStreamDestroy(cap);
  if (st != AMG_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "round capture", __LINE__);
  return AMG_OK;
}

// Rounds queued per wait for the instances' states: finished instances sit
// out by their gates, so the rounds after the last instance finishes are
// near-empty launches.
constexpr int kRoundsPerWait = 4;

int batch_solve(const std::vector<amg_ctx*>& cs, const std::vector<const double*>& bs,
                const std::vector<double*>& xs, const std::vector<double>& tols, hipStream_t s) {
  const int n = (int)cs.size();
  for (int i = 0; i < n; ++i) AMG_TRY(solve_begin(cs[i], bs[i], xs[i], tols[i], s));
  HIP_TRY(round_wait(s));
  BatchPlan P;
  hipGraphExec_t gexec = nullptr;
  std::vector<int> active;
  for (int i = 0; i < n; ++i)
    if (!cs[i]->st_host->done) active.push_back(i);
  size_t built_for = 0;
  bool eager = false;
  int st = AMG_OK;
  while (!active.empty()) {
    if (built_for == 0 || active.size() * 4 <= built_for * 3) {
      // (re)build the round over the active instances only
      HIP_TRY(round_wait(s));  // the previous tables are no longer read
      if (gexec) (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
      std::vector<amg_ctx*> c2;
      std::vector<const double*> b2;
      std::vector<double*> x2;
      std::vector<double> t2;
      for (int i : active) {
        c2.push_back(cs[i]);
        b2.push_back(bs[i]);
        x2.push_back(xs[i]);
        t2.push_back(tols[i]);
      }
      st = build_batch_plan(P, c2, b2, x2, t2);
      if (st == AMG_OK) st = run_batch_plan(P, s);
      if (st != AMG_OK) break;
      built_for = active.size();
      eager = true;
    }
    if (eager) {
      // the first round of a plan runs directly (it also raises the kernels'
      // LDS limits); the next ones replay its captured graph
      for (const Launch& L : P.round) {
        const hipError_t e = L(static_cast<unsigned char*>(P.dev), s);
        if (e != hipSuccess) {
          st = hip_fail(e, "batched launch", __LINE__);
          break;
        }
      }
      if (st != AMG_OK) break;
      eager = false;
    } else {
      if (!gexec) {
        st = capture_round(P, &gexec);
        if (st != AMG_OK) break;
      }
      for (int r = 0; r < kRoundsPerWait; ++r) {
        const hipError_t e = hipGraphLaunch(gexec, s);
        if (e != hipSuccess) {
          st = hip_fail(e, "hipGraphLaunch", __LINE__);
          break;
        }
      }
      if (st != AMG_OK) break;
    }
    HIP_TRY(round_wait(s));
    std::vector<int> still;
    for (int i : active)
      if (!cs[i]->st_host->done) still.push_back(i);
    active.swap(still);
  }
  (void)round_wait(s);
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (P.dev) (void)hipFree(P.dev);
  return st;
}

}  // namespace

extern "C" {

int amg_solve_batch(int count, amg_t* hs, const double* const* b, double* const* x,
                    const double* tol, void* stream, int* iters, double* relres) {
  if (count < 0 || (count > 0 && (!hs || !b || !x || !tol))) return AMG_EINVAL;
  if (count == 0) return AMG_OK;
  const int dev = hs[0] ? hs[0]->device : -1;
  for (int i = 0; i < count; ++i) {
    amg_t h = hs[i];
    if (!h || h->host_only || h->device != dev || !b[i] || !x[i] || b[i] == x[i]) return AMG_EINVAL;
    if (!(tol[i] > 0.0) || !std::isfinite(tol[i])) return AMG_EINVAL;
    for (int j = 0; j < i; ++j)
      if (hs[j] == h) return AMG_EINVAL;  // a handle's buffers serve one solve at a time
  }
  HIP_TRY(hipSetDevice(dev));
  hipStream_t s = (hipStream_t)stream;
  bool batched = true;
  for (int i = 0; i < count; ++i)
    if (!batchable(hs[i]) || hs[i]->opts.m1 != hs[0]->opts.m1 || hs[i]->opts.m2 != hs[0]->opts.m2)
      batched = false;
  if (batched) {
    std::vector<amg_ctx*> cs(hs, hs + count);
    std::vector<const double*> bs(b, b + count);
    std::vector<double*> xs(x, x + count);
    std::vector<double> ts(tol, tol + count);
    AMG_TRY(batch_solve(cs, bs, xs, ts, s));
    // results: every history copy queued, one wait
    for (int i = 0; i < count; ++i) {
      amg_t h = hs[i];
      h->prof.collect();
      const SolveState st = *h->st_host;
      h->last_iters = st.iter;
      h->hist.assign((size_t)st.iter + 1, 0.0);
      HIP_TRY(hipMemcpyAsync(h->hist.data(), h->hist_dev, h->hist.size() * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    int worst = AMG_OK;
    for (int i = 0; i < count; ++i) {
      const SolveState st = *hs[i]->st_host;
      if (iters) iters[i] = st.iter;
      if (relres) relres[i] = st.relres;
      worst = std::max(worst, st.status);
    }
    return worst;
  }
  StreamPool* pool = nullptr;
  AMG_TRY(get_pool(dev, &pool));
  const int S = std::min(count, kBatchStreams);
  // fork: the internal streams start after the caller's stream
  HIP_TRY(hipEventRecord(pool->events[kBatchStreams], s));
  for (int k = 0; k < S; ++k) HIP_TRY(hipStreamWaitEvent(pool->streams[k], pool->events[kBatchStreams], 0));
  for (int i = 0; i < count; ++i)
    AMG_TRY(solve_begin(hs[i], b[i], x[i], tol[i], pool->streams[i % S]));
  std::vector<char> done(count, 0);
  for (int round = 0;; ++round) {
    for (int k = 0; k < S; ++k) HIP_TRY(round_wait(pool->streams[k]));
    int active = 0;
    for (int i = 0; i < count; ++i) {
      if (done[i]) continue;
      if (hs[i]->st_host->done) {
        done[i] = 1;
        continue;
      }
      ++active;
      AMG_TRY(solve_round(hs[i], b[i], x[i], tol[i], pool->streams[i % S], round));
    }
    if (!active) break;
  }
  int worst = AMG_OK;
  for (int i = 0; i < count; ++i) {
    const int st = solve_end(hs[i], pool->streams[i % S], iters ? &iters[i] : nullptr,
                             relres ? &relres[i] : nullptr);
    if (st < 0) return st;
    worst = std::max(worst, st);
  }
  // join: the caller's stream continues after every internal stream
  for (int k = 0; k < S; ++k) {
    HIP_TRY(hipEventRecord(pool->events[k], pool->streams[k]));
    HIP_TRY(hipStreamWaitEvent(s, pool->events[k], 0));
  }
  return worst;
}

int amg_profile_stats(amg_t h, amg_stat_t* out, int cap, int reset) {
  if (!h || cap < 0 || (!out && cap > 0)) return AMG_EINVAL;
  const int k = std::min<int>(cap, PK_COUNT);
  for (int i = 0; i < k; ++i) {
    std::memset(&out[i], 0, sizeof(amg_stat_t));
    std::snprintf(out[i].name, sizeof(out[i].name), "%s", kProfNames[i]);
    out[i].launches = h->prof.launches[i];
    out[i].total_ms = h->prof.total_ms[i];
  }
  if (reset) {
    for (int i = 0; i < PK_COUNT; ++i) {
      h->prof.launches[i] = 0;
      h->prof.total_ms[i] = 0.0;
    }
  }
  return k;
}

int amg_residual_history(amg_t h, double* hist, int cap) {
  if (!h || (!hist && cap > 0) || cap < 0) return AMG_EINVAL;
  const int k = std::min<int>(cap, (int)h->hist.size());
  for (int i = 0; i < k; ++i) hist[i] = h->hist[i];
  return k;
}

int amg_manufactured_rhs(const amg_kernel_t* kernel, double delta, int64_t N, double* b_host) {
  if (!kernel || !b_host || kernel->kind == AMG_K_GENERATORS) return AMG_EINVAL;
  if (kernel->kind == AMG_K_WEAKLY_SINGULAR) return AMG_ENOTSUP;
  const KernelSpec ks = spec_of(kernel, delta);
  if (!validate(ks, N, 2).empty() || !std::isfinite(delta)) return AMG_EINVAL;
  if (!ks.supported()) return AMG_ENOTSUP;
  manufactured_rhs(ks, N, b_host);
  return AMG_OK;
}

int64_t amg_volume_reach(const amg_kernel_t* kernel, double delta, int64_t N) {
  if (!kernel || kernel->kind == AMG_K_GENERATORS) return AMG_EINVAL;
  const KernelSpec ks = spec_of(kernel, ignores_delta(kernel) ? 0.25 : delta);
  if (!validate(ks, N, 2).empty() || !std::isfinite(ks.delta)) return AMG_EINVAL;
  if (!ks.supported()) return AMG_ENOTSUP;
  try {
    return volume_reach(ks, N);
  } catch (const std::bad_alloc&) {
    return AMG_ENOMEM;
  }
}

int amg_volume_rhs(const amg_kernel_t* kernel, double delta, int64_t N, const double* g_left,
                   const double* g_right, double* b) {
  if (!kernel || !g_left || !g_right || !b || kernel->kind == AMG_K_GENERATORS) return AMG_EINVAL;
  const KernelSpec ks = spec_of(kernel, ignores_delta(kernel) ? 0.25 : delta);
  if (!validate(ks, N, 2).empty() || !std::isfinite(ks.delta)) return AMG_EINVAL;
  if (!ks.supported()) return AMG_ENOTSUP;
  try {
    volume_correction(ks, N, g_left, g_right, b);
  } catch (const std::bad_alloc&) {
    return AMG_ENOMEM;
  }
  return AMG_OK;
}

int64_t amg_footprint_bytes(const amg_kernel_t* kernel, double delta, int64_t N,
                            const amg_opts_t* opts) {
  if (!kernel) return AMG_EINVAL;
  amg_opts_t o;
  if (opts) o = *opts;
  else amg_default_opts(&o);
  if (check_opts(&o) != AMG_OK) return AMG_EINVAL;
  const KernelSpec ks = spec_of(kernel, ignores_delta(kernel) ? 0.25 : delta);
  if (!validate(ks, N, o.coarsest_log2).empty()) return AMG_EINVAL;
  if (!ks.supported()) return AMG_ENOTSUP;
  return footprint(N, &o, (kernel->kind == AMG_K_CONST || is_fractional(kernel->kind)) &&
                              ks.scheme == SCHEME_SHIFTED,
                   kernel->kind == AMG_K_WEAKLY_SINGULAR);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Geometry autotuner: per four-step size, the (row length, column tile) of
// the level matvec that runs fastest on this GPU among the candidates.
// ---------------------------------------------------------------------------
namespace {

template <typename F>
int time_median(hipStream_t s, int reps, F&& f, double* us) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return AMG_EHIP;
  }
  std::vector<float> t;
  int st = AMG_OK;
  for (int r = 0; r < reps && st == AMG_OK; ++r) {
    float ms = 0;
    if (hipEventRecord(e0, s) != hipSuccess) st = AMG_EHIP;
    if (st == AMG_OK) st = f();
    if (st == AMG_OK && (hipEventRecord(e1, s) != hipSuccess ||
                         hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = AMG_EHIP;
    t.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != AMG_OK) return st;
  std::sort(t.begin(), t.end());
  *us = 1e3 * (double)t[t.size() / 2];
  return AMG_OK;
}

// One size: a level of general blocks (random generators and Cross data)
// with each candidate geometry; the FP64 product of every candidate must
// agree with the default geometry's to 1e-11 of its largest entry, else the
// candidate is rejected; cost = median FP32 + median FP64 matvec time.
int tune_size(int dev, int logL, hipStream_t s, PlanChoice* out) {
  const std::vector<Plan> cands = plan_candidates(logL);
  *out = PlanChoice{};
  out->p = cands[0];
  out->candidates = (int)cands.size();
  if (cands[0].tail) return AMG_OK;
  const int64_t L = int64_t(1) << logL, n = L / 2 - 1, m = 2 * n + 1;
  amg_ctx t;
  t.device = dev;
  t.mixed = true;
  struct Guard {
    amg_ctx* c;
    hipStream_t s;
    ~Guard() {
      (void)hipStreamSynchronize(s);
      free_setup_temps(c);
      release(c);
    }
  } guard{&t, s};
  AMG_TRY(device_twiddles(dev, s, &t.tw64, &t.tw32));
  AMG_TRY(dalloc(&t, &t.buf64, (size_t)L));
  AMG_TRY(dalloc(&t, &t.buf32, (size_t)L));
  cplx<double>* zs = nullptr;
  AMG_TRY(dalloc(&t, &zs, (size_t)L));
  double *ga, *gb, *gc, *gd, *cx, *x, *y;
  float *cxf, *xf, *yf;
  for (double** g : {&ga, &gb, &gc, &gd}) AMG_TRY(dalloc(&t, g, (size_t)(2 * n - 1)));
  AMG_TRY(dalloc(&t, &cx, (size_t)(4 * n)));
  AMG_TRY(dalloc(&t, &x, (size_t)m));
  AMG_TRY(dalloc(&t, &y, (size_t)m));
  AMG_TRY(dalloc(&t, &cxf, (size_t)(4 * n)));
  AMG_TRY(dalloc(&t, &xf, (size_t)m));
  AMG_TRY(dalloc(&t, &yf, (size_t)m));
  unsigned seed = 1;
  for (double* g : {ga, gb, gc, gd}) HIP_TRY(launch_fill_hash(g, 2 * n - 1, seed++, s));
  HIP_TRY(launch_fill_hash(cx, 4 * n, seed++, s));
  HIP_TRY(launch_fill_hash(x, m, seed++, s));
  HIP_TRY(launch_copy_d2f(cx, cxf, 4 * n, s));
  HIP_TRY(launch_copy_d2f(x, xf, m, s));
  int maxb = 1;
  for (const Plan& q : cands)
    maxb = std::max({maxb, col_blocks(q.logL1, q.tcols), (1 << q.logL2) / 2});
  AMG_TRY(dalloc(&t, &t.dpart64, (size_t)maxb));
  AMG_TRY(dalloc(&t, &t.dpart32, (size_t)maxb));
  AMG_TRY(dalloc(&t, &t.npart, (size_t)std::max(maxb, vec_blocks(m))));
  t.lv.resize(1);
  LevelRes& R = t.lv[0];
  R.n = n;
  R.sym = false;
  R.o = R.dv = R.dw = 1.0;
  R.pd = cx;
  R.qd = cx + n;
  R.xid = cx + 2 * n;
  R.zetad = cx + 3 * n;
  R.pf = cxf;
  R.qf = cxf + n;
  R.xif = cxf + 2 * n;
  R.zetaf = cxf + 3 * n;
  AMG_TRY(dalloc(&t, &R.scald, 4));
  AMG_TRY(dalloc(&t, &R.scalf, 4));
  std::vector<double> yref((size_t)m), ycur((size_t)m);
  double best = 0;
  for (size_t k = 0; k < cands.size(); ++k) {
    R.plan = cands[k];
    AMG_TRY(level_spectra_dev(&t, ga, gb, gc, gd, R, true, zs, s));
    AMG_TRY(level_matvec<double>(&t, 0, x, y, s));
    std::vector<double>& h = k == 0 ? yref : ycur;
    HIP_TRY(hipMemcpyAsync(h.data(), y, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (k > 0) {
      double dmax = 0, ymax = 0;
      bool fin = true;
      for (int64_t i = 0; i < m; ++i) {
        fin = fin && std::isfinite(ycur[(size_t)i]);
        dmax = std::max(dmax, std::fabs(ycur[(size_t)i] - yref[(size_t)i]));
        ymax = std::max(ymax, std::fabs(yref[(size_t)i]));
      }
      if (!fin || !(dmax <= 1e-11 * ymax)) {
        out->rejected += 1;
        continue;
      }
    }
    double us32 = 0, us64 = 0;
    AMG_TRY(level_matvec<float>(&t, 0, xf, yf, s));  // warm-up
    AMG_TRY(time_median(s, 7, [&] { return level_matvec<float>(&t, 0, xf, yf, s); }, &us32));
    AMG_TRY(time_median(s, 7, [&] { return level_matvec<double>(&t, 0, x, y, s); }, &us64));
    const double cost = us32 + us64;
    if (k == 0) out->us_default = cost;
    if (k == 0 || cost < best) {
      best = cost;
      out->p = cands[k];
    }
  }
  out->us_best = best;
  out->set = true;
  return AMG_OK;
}

bool plan_size_ok(int logL) { return logL > kTailLog && logL <= 23; }

}  // namespace

extern "C" {

int amg_autotune(int logL_min, int logL_max, void* stream) {
  if (logL_min > logL_max) return AMG_EINVAL;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipStream_t s = (hipStream_t)stream;
  for (int lg = std::max(logL_min, kTailLog + 1); lg <= std::min(logL_max, 23); ++lg) {
    PlanChoice pc;
    AMG_TRY(tune_size(dev, lg, s, &pc));
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_plan[lg] = pc;
  }
  return AMG_OK;
}

int amg_plan_get(int logL, int* logL1, int* tcols, double* us_default, double* us_best,
                 int* candidates, int* rejected) {
  if (!plan_size_ok(logL)) return AMG_EINVAL;
  std::lock_guard<std::mutex> g(g_plan_mu);
  const PlanChoice& c = g_plan[logL];
  const Plan p = c.set ? c.p : default_plan(logL);
  if (logL1) *logL1 = p.logL1;
  if (tcols) *tcols = p.tcols;
  if (us_default) *us_default = c.us_default;
  if (us_best) *us_best = c.us_best;
  if (candidates) *candidates = c.set ? c.candidates : (int)plan_candidates(logL).size();
  if (rejected) *rejected = c.rejected;
  return AMG_OK;
}

int amg_plan_set(int logL, int logL1, int tcols) {
  if (!plan_size_ok(logL)) return AMG_EINVAL;
  std::lock_guard<std::mutex> g(g_plan_mu);
  if (logL1 == 0) {
    g_plan[logL] = PlanChoice{};
    return AMG_OK;
  }
  const std::vector<Plan> cands = plan_candidates(logL);
  for (const Plan& p : cands)
    if (p.logL1 == logL1 && p.tcols == tcols) {
      g_plan[logL] = PlanChoice{};
      g_plan[logL].set = true;
      g_plan[logL].p = p;
      g_plan[logL].candidates = (int)cands.size();
      return AMG_OK;
    }
  return AMG_EINVAL;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: a request loop over the batched rounds (amg_server_*).  Requests
// are admitted by device footprint, set up by worker threads on their own
// streams (or taken from a cache of idle hierarchies with the same problem
// key), started between rounds, and advanced together: every round runs one
// iteration of every request in flight, whatever it arrived; finished ones
// leave, new ones join (continuous batching at iteration granularity).
// ---------------------------------------------------------------------------
namespace {

struct ServerKey {
  int kind, scheme, precision, inner, m1, m2, coarsest, max_iter, flags;
  double alpha, wl, wr, delta, omega_pre, omega_post, shift, scale;
  int64_t N;
  bool operator<(const ServerKey& o) const {
    return std::memcmp(this, &o, sizeof(ServerKey)) < 0;
  }
};

ServerKey server_key(const amg_kernel_t& k, double delta, int64_t N, const amg_opts_t& o) {
  ServerKey key;
  std::memset(&key, 0, sizeof key);  // padding compares equal
  key.kind = k.kind;
  key.scheme = k.scheme;
  key.precision = o.precision;
  key.inner = o.inner;
  key.m1 = o.m1;
  key.m2 = o.m2;
  key.coarsest = o.coarsest_log2;
  key.max_iter = o.max_iter;
  key.flags = o.flags;
  key.alpha = is_fractional(k.kind) ? k.alpha : 0.0;
  key.wl = k.kind == AMG_K_WEIGHTED ? k.wl : 0.0;
  key.wr = k.kind == AMG_K_WEIGHTED ? k.wr : 0.0;
  key.delta = delta;
  key.omega_pre = o.omega_pre;
  key.omega_post = o.omega_post;
  key.shift = o.shift;
  key.scale = o.scale;
  key.N = N;
  return key;
}

struct ServerReq {
  int64_t id = 0;
  amg_kernel_t kernel{};
  double delta = 0;
  int64_t N = 0;
  amg_opts_t opts{};
  const double* b = nullptr;
  double* x = nullptr;
  double tol = 0;
  int64_t bytes = 0;
  ServerKey key{};
  amg_t h = nullptr;
  amg_t donor = nullptr;  // an evicted hierarchy whose memory the set-up reuses
  int setup_status = AMG_OK;
  bool cached = false;
};

}  // namespace

struct amg_server {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t budget = 0, reserved = 0, peak_reserved = 0;
  int m1 = -1, m2 = -1;
  int64_t next_id = 1;
  std::mutex mu;
  std::condition_variable cv;       // work for the set-up threads
  std::condition_variable cv_done;  // a set-up finished
  int setting_up = 0;               // set-ups a worker has taken
  bool stop = false;
  std::deque<ServerReq*> pending;   // submitted, not admitted
  std::deque<ServerReq*> setup_q;   // admitted (memory reserved), for a worker
  std::vector<std::pair<amg_t, int64_t>> release_q;  // evicted, for a worker to free
  int64_t releasing = 0;                              // their bytes, until freed
  std::vector<ServerReq*> ready;    // hierarchy ready, starts at the next step
  // requests in the rounds (step thread only): lane 0 on the server's
  // stream, lane 1 (the small requests, when amg_server_lanes set it up) on
  // a stream of its own, so that the two lanes' rounds overlap on the device
  struct Lane {
    std::vector<ServerReq*> active;
    BatchPlan plan;
    bool dirty = true;
    bool running = false;  // its last rounds are still on the stream
    hipStream_t s = nullptr;
  };
  Lane lane[2];
  bool own_small_stream = false;
  int64_t small_max_N = 0;  // 0: one lane
  int small_rounds = 1;     // rounds of lane 1 per round of lane 0
  std::vector<ServerReq*> failed;   // setup failed, reported by the next poll
  std::vector<amg_server_result_t> finished;
  std::multimap<ServerKey, std::pair<amg_t, int64_t>> idle;  // cached hierarchies
  std::deque<std::pair<ServerKey, amg_t>> idle_order;       // oldest first
  std::vector<std::thread> workers;
  amg_server_stats_t stats{};
};

namespace {

// Take a cached hierarchy for the key, if one is idle (caller holds mu).
amg_t cache_take(amg_server* sv, const ServerKey& key, int64_t* bytes) {
  auto it = sv->idle.find(key);
  if (it == sv->idle.end()) return nullptr;
  amg_t h = it->second.first;
  *bytes = it->second.second;
  sv->idle.erase(it);
  for (auto o = sv->idle_order.begin(); o != sv->idle_order.end(); ++o)
    if (o->second == h) {
      sv->idle_order.erase(o);
      break;
    }
  return h;
}

// Evict the oldest cached hierarchy (caller holds mu); false if none.  A
// set-up thread releases it (hipFree waits for the device, which neither the
// rounds nor a submitting thread should do); its bytes stay reserved until
// then, so the reservation never exceeds the budget.
bool cache_evict_one(amg_server* sv) {
  if (sv->idle_order.empty()) return false;
  const auto victim = sv->idle_order.front();
  sv->idle_order.pop_front();
  auto range = sv->idle.equal_range(victim.first);
  for (auto it = range.first; it != range.second; ++it)
    if (it->second.first == victim.second) {
      sv->release_q.push_back(it->second);
      sv->releasing += it->second.second;
      sv->idle.erase(it);
      break;
    }
  sv->stats.evictions += 1;
  sv->cv.notify_one();
  return true;
}

// Admit pending requests in order while their footprint fits (caller holds
// mu): a cached hierarchy with the same key is taken at once; otherwise the
// memory is reserved (evicting idle hierarchies if needed) and a worker sets
// the request up.
void admit(amg_server* sv) {
  while (!sv->pending.empty()) {
    ServerReq* r = sv->pending.front();
    int64_t cbytes = 0;
    amg_t h = cache_take(sv, r->key, &cbytes);
    if (h) {
      r->h = h;
      r->bytes = cbytes;
      r->cached = true;
      sv->stats.cache_hits += 1;
      sv->pending.pop_front();
      sv->ready.push_back(r);
      continue;
    }
    if (sv->reserved + r->bytes > sv->budget) {
      // an idle hierarchy of the same footprint (the same shape: N, options,
      // kernel symmetry) hands its device memory to this set-up
      amg_t victim = nullptr;
      for (auto o = sv->idle_order.begin(); o != sv->idle_order.end() && !victim; ++o) {
        auto range = sv->idle.equal_range(o->first);
        for (auto it = range.first; it != range.second; ++it)
          if (it->second.first == o->second && it->second.second == r->bytes) {
            victim = o->second;
            sv->idle.erase(it);
            sv->idle_order.erase(o);
            break;
          }
      }
      if (victim) {
        r->donor = victim;
        sv->stats.evictions += 1;
        sv->stats.cache_misses += 1;
        sv->pending.pop_front();
        sv->setup_q.push_back(r);
        sv->cv.notify_one();
        continue;
      }
    }
    while (sv->reserved - sv->releasing + r->bytes > sv->budget && cache_evict_one(sv)) {
    }
    if (sv->reserved + r->bytes > sv->budget) break;  // waits for memory
    sv->reserved += r->bytes;
    sv->peak_reserved = std::max(sv->peak_reserved, sv->reserved);
    sv->stats.cache_misses += 1;
    sv->pending.pop_front();
    sv->setup_q.push_back(r);
    sv->cv.notify_one();
  }
}

int64_t usec_since(std::chrono::steady_clock::time_point t0) {
  return (int64_t)std::chrono::duration_cast<std::chrono::microseconds>(
             std::chrono::steady_clock::now() - t0)
      .count();
}

void server_worker(amg_server* sv) {
  (void)hipSetDevice(sv->device);
  hipStream_t ws = nullptr;
  (void)hipStreamCreateWithFlags(&ws, hipStreamNonBlocking);
  for (;;) {
    ServerReq* r = nullptr;
    std::pair<amg_t, int64_t> victim{nullptr, 0};
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait(lk, [&] {
        return sv->stop || !sv->setup_q.empty() || !sv->release_q.empty();
      });
      if (!sv->release_q.empty()) {
        victim = sv->release_q.back();
        sv->release_q.pop_back();
      } else if (sv->stop) {
        break;  // queued set-ups are dropped by amg_server_destroy
      } else {
        r = sv->setup_q.front();
        sv->setup_q.pop_front();
        sv->setting_up += 1;
      }
    }
    if (victim.first) {
      (void)amg_destroy(victim.first);
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->reserved -= victim.second;
        sv->releasing -= victim.second;
        admit(sv);
      }
      sv->cv_done.notify_all();
      continue;
    }
    amg_t h = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    const int st = setup_impl(&r->kernel, r->delta, r->N, &r->opts, ws, r->donor, &h);
    r->donor = nullptr;  // destroyed or taken over by the set-up
    const int64_t us = usec_since(t0);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stats.setup_us += us;
      r->setup_status = st;
      r->h = h;
      if (st == AMG_OK) {
        sv->ready.push_back(r);
      } else {
        sv->reserved -= r->bytes;
        sv->failed.push_back(r);
        admit(sv);
      }
      sv->setting_up -= 1;
    }
    sv->cv_done.notify_all();
  }
  if (ws) (void)hipStreamDestroy(ws);
}

// Wait for the server stream with short sleeps between queries: the set-up
// threads keep making runtime calls meanwhile, and a query loop without
// pauses contends with them.
hipError_t server_wait(hipStream_t s) {
  for (;;) {
    const hipError_t e = hipStreamQuery(s);
    if (e != hipErrorNotReady) return e;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

void retire(amg_server* sv, ServerReq* r, const SolveState& st) {
  amg_server_result_t res{};
  res.id = r->id;
  res.status = st.status;
  res.iters = st.iter;
  res.relres = st.relres;
  res.cached = r->cached ? 1 : 0;
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->finished.push_back(res);
  sv->stats.finished += 1;
  // the hierarchy stays on the device for a later request with the same key
  sv->idle.insert({r->key, {r->h, r->bytes}});
  sv->idle_order.push_back({r->key, r->h});
  delete r;
  admit(sv);
}

}  // namespace

extern "C" {

int amg_server_create(int64_t mem_budget_bytes, int workers, void* stream, amg_server_t* out) {
  if (!out || mem_budget_bytes <= 0 || workers < 1 || workers > 64) return AMG_EINVAL;
  *out = nullptr;
  amg_server* sv = new (std::nothrow) amg_server();
  if (!sv) return AMG_ENOMEM;
  const hipError_t e = hipGetDevice(&sv->device);
  if (e != hipSuccess) {
    delete sv;
    return hip_fail(e, "hipGetDevice", __LINE__);
  }
  sv->budget = mem_budget_bytes;
  sv->stream = (hipStream_t)stream;
  if (!sv->stream) {
    // an own stream: the legacy default stream would also wait for the
    // set-up threads' work whenever the rounds are waited for
    const hipError_t es = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (es != hipSuccess) {
      delete sv;
      return hip_fail(es, "hipStreamCreateWithFlags", __LINE__);
    }
    sv->own_stream = true;
  }
  try {
    for (int i = 0; i < workers; ++i) sv->workers.emplace_back(server_worker, sv);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
    }
    sv->cv.notify_all();
    for (auto& t : sv->workers) t.join();
    delete sv;
    return AMG_ENOMEM;
  }
  *out = sv;
  return AMG_OK;
}

int amg_server_submit(amg_server_t sv, const amg_kernel_t* kernel, double delta, int64_t N,
                      const amg_opts_t* opts, const double* b, double* x, double tol,
                      int64_t* id) {
  if (!sv || !kernel || !b || !x || b == x || !(tol > 0.0) || !std::isfinite(tol)) return AMG_EINVAL;
  if (kernel->kind != AMG_K_CONST && kernel->kind != AMG_K_WEIGHTED &&
      !is_fractional(kernel->kind))
    return AMG_ENOTSUP;
  amg_opts_t o;
  if (opts) o = *opts;
  else amg_default_opts(&o);
  if (o.cycle != 1 || (o.inner != AMG_INNER_VCYCLE && o.inner != AMG_INNER_PCG) ||
      (o.flags & (AMG_FLAG_ACCURATE_RESIDUAL | AMG_FLAG_PROFILE | AMG_FLAG_HOST_ONLY)))
    return AMG_ENOTSUP;
  const int64_t bytes = amg_footprint_bytes(kernel, delta, N, &o);
  if (bytes < 0) return (int)bytes;
  ServerReq* r = new (std::nothrow) ServerReq();
  if (!r) return AMG_ENOMEM;
  r->kernel = *kernel;
  r->kernel.gen = nullptr;
  r->delta = delta;
  r->N = N;
  r->opts = o;
  r->b = b;
  r->x = x;
  r->tol = tol;
  r->bytes = bytes;
  r->key = server_key(*kernel, delta, N, o);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->m1 < 0) {
    sv->m1 = o.m1;
    sv->m2 = o.m2;
  }
  if (o.m1 != sv->m1 || o.m2 != sv->m2 || bytes > sv->budget) {
    delete r;
    return AMG_ENOTSUP;  // one sweep count per server; larger than the budget
  }
  r->id = sv->next_id++;
  if (id) *id = r->id;
  sv->pending.push_back(r);
  sv->stats.submitted += 1;
  admit(sv);
  return AMG_OK;
}

int amg_server_step(amg_server_t sv, int rounds, int* in_flight, int* waiting) {
  if (!sv || rounds < 0) return AMG_EINVAL;
  HIP_TRY(hipSetDevice(sv->device));
  sv->lane[0].s = sv->stream;
  auto idle = [&]() {
    return sv->lane[0].active.empty() && sv->lane[1].active.empty() && !sv->lane[0].running &&
           !sv->lane[1].running;
  };
  std::vector<ServerReq*> start;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    admit(sv);
    // nothing to run yet: wait for the first set-up to end
    if (idle() && rounds > 0)
      sv->cv_done.wait(lk, [&] {
        return !sv->ready.empty() || !sv->failed.empty() ||
               (sv->setup_q.empty() && sv->setting_up == 0 && sv->releasing == 0);
      });
    start.swap(sv->ready);
  }
  auto t0 = std::chrono::steady_clock::now();
  for (ServerReq* r : start) {
    // on a running lane the request's start queues behind its rounds
    amg_server::Lane& ln = sv->lane[(sv->small_max_N > 0 && r->N <= sv->small_max_N) ? 1 : 0];
    AMG_TRY(solve_begin(r->h, r->b, r->x, r->tol, ln.s));
    ln.active.push_back(r);
    ln.dirty = true;
  }
  auto retire_done = [&](amg_server::Lane& ln) {
    for (size_t i = 0; i < ln.active.size();) {
      ServerReq* r = ln.active[i];
      if (r->h->st_host->done) {
        const SolveState st = *r->h->st_host;
        ln.active.erase(ln.active.begin() + (long)i);
        retire(sv, r, st);
        ln.dirty = true;
      } else {
        ++i;
      }
    }
  };
  int64_t t_start = usec_since(t0), t_rebuild = 0, t_rounds = 0;
  if (rounds == 0) {
    // start only: wait for every lane, retire what the starts finished
    for (amg_server::Lane& ln : sv->lane)
      if (!ln.active.empty() || ln.running) HIP_TRY(server_wait(ln.s));
    for (amg_server::Lane& ln : sv->lane) {
      ln.running = false;
      retire_done(ln);
    }
  } else {
    // The lanes advance independently: a lane whose rounds have completed
    // retires its finished requests and queues its next rounds (rebuilding
    // its tables if its members changed); the call returns once a lane has
    // completed and been queued again, so neither lane waits for the other.
    t0 = std::chrono::steady_clock::now();
    bool progressed = false;
    for (;;) {
      for (int li = 0; li < 2; ++li) {
        amg_server::Lane& ln = sv->lane[li];
        if (ln.running) {
          const hipError_t e = hipStreamQuery(ln.s);
          if (e == hipErrorNotReady) continue;
          if (e != hipSuccess) return hip_fail(e, "server lane", __LINE__);
          ln.running = false;
          retire_done(ln);
          progressed = true;
        }
        if (ln.active.empty()) continue;
        if (ln.dirty) {
          const auto tb = std::chrono::steady_clock::now();
          std::vector<amg_ctx*> cs;
          std::vector<const double*> bs;
          std::vector<double*> xs;
          std::vector<double> ts;
          for (ServerReq* r : ln.active) {
            cs.push_back(r->h);
            bs.push_back(r->b);
            xs.push_back(r->x);
            ts.push_back(r->tol);
          }
          AMG_TRY(build_batch_plan(ln.plan, cs, bs, xs, ts));
          AMG_TRY(run_batch_plan(ln.plan, ln.s));
          ln.dirty = false;
          sv->stats.rebuilds += 1;
          t_rebuild += usec_since(tb);
        }
        const int nr = li == 0 ? rounds : rounds * sv->small_rounds;
        for (int k = 0; k < nr; ++k)
          for (const Launch& L : ln.plan.round) {
            const hipError_t e = L(static_cast<unsigned char*>(ln.plan.dev), ln.s);
            if (e != hipSuccess) return hip_fail(e, "server round", __LINE__);
          }
        sv->stats.rounds += nr;
        ln.running = true;
      }
      if (progressed || (!sv->lane[0].running && !sv->lane[1].running)) break;
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    t_rounds = usec_since(t0) - t_rebuild;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->stats.start_us += t_start;
  sv->stats.rebuild_us += t_rebuild;
  sv->stats.rounds_us += t_rounds;
  if (in_flight)
    *in_flight = (int)(sv->lane[0].active.size() + sv->lane[1].active.size() + sv->ready.size() +
                       sv->setup_q.size()) +
                 sv->setting_up;
  if (waiting) *waiting = (int)sv->pending.size();
  return AMG_OK;
}

int amg_server_lanes(amg_server_t sv, int64_t small_max_N, int small_rounds) {
  if (!sv || small_max_N < 0 || small_rounds < 1 || small_rounds > 16) return AMG_EINVAL;
  if (!sv->lane[0].active.empty() || !sv->lane[1].active.empty() || sv->lane[0].running ||
      sv->lane[1].running)
    return AMG_EINVAL;
  if (small_max_N > 0 && !sv->lane[1].s) {
    HIP_TRY(hipSetDevice(sv->device));
    HIP_TRY(hipStreamCreateWithFlags(&sv->lane[1].s, hipStreamNonBlocking));
    sv->own_small_stream = true;
  }
  sv->small_max_N = small_max_N;
  sv->small_rounds = small_rounds;
  return AMG_OK;
}

int amg_server_poll(amg_server_t sv, amg_server_result_t* out, int cap) {
  if (!sv || cap < 0 || (!out && cap > 0)) return AMG_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  for (ServerReq* r : sv->failed) {
    amg_server_result_t res{};
    res.id = r->id;
    res.status = r->setup_status;
    sv->finished.push_back(res);
    delete r;
  }
  sv->failed.clear();
  const int k = std::min<int>(cap, (int)sv->finished.size());
  for (int i = 0; i < k; ++i) out[i] = sv->finished[(size_t)i];
  sv->finished.erase(sv->finished.begin(), sv->finished.begin() + k);
  return k;
}

int amg_server_stats(amg_server_t sv, amg_server_stats_t* out) {
  if (!sv || !out) return AMG_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->stats;
  out->reserved_bytes = sv->reserved;
  out->peak_reserved_bytes = sv->peak_reserved;
  out->cached_hierarchies = (int64_t)sv->idle.size();
  return AMG_OK;
}

int amg_server_destroy(amg_server_t sv) {
  if (!sv) return AMG_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  for (auto& t : sv->workers) t.join();
  (void)hipSetDevice(sv->device);
  if (sv->stream) (void)round_wait(sv->stream);
  if (sv->lane[1].s) (void)round_wait(sv->lane[1].s);
  for (amg_server::Lane& ln : sv->lane)
    for (ServerReq* r : ln.active) {
      (void)amg_destroy(r->h);
      delete r;
    }
  for (ServerReq* r : sv->ready) {
    (void)amg_destroy(r->h);
    delete r;
  }
  for (ServerReq* r : sv->pending) delete r;
  for (ServerReq* r : sv->setup_q) {
    if (r->donor) (void)amg_destroy(r->donor);
    delete r;
  }
  for (ServerReq* r : sv->failed) delete r;
  for (auto& kv : sv->idle) (void)amg_destroy(kv.second.first);
  for (amg_server::Lane& ln : sv->lane)
    if (ln.plan.dev) (void)hipFree(ln.plan.dev);
  if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
  if (sv->own_small_stream) (void)hipStreamDestroy(sv->lane[1].s);
  delete sv;
  return AMG_OK;
}

}  // extern "C"
