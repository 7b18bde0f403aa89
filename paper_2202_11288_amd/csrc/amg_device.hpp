// Device-side data views and kernel launchers shared by the HIP kernels
// (amg_kernels.hip) and the C-ABI orchestration (amg_api.cpp).  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amg {

template <typename T>
struct cplx;

// Constants of the FFT machinery.
constexpr int kTwLog = 14;
constexpr int kTwM = 1 << kTwLog;  // base twiddle table: e^{-2 pi i m / kTwM}
constexpr int kTw4Log = 23;        // four-step twiddles resolved on 2^23 points
constexpr int kTw4Lo = 4096;       // low table: e^{-2 pi i m / 2^23}, m < 4096
constexpr int kTw4Hi = 2048;       // high table: e^{-2 pi i m 4096 / 2^23}, m < 2048
constexpr int kNT4 = 256;          // threads of a four-step pass workgroup
constexpr int kCap4 = 4096;        // complex values per four-step workgroup (tile or row pair)
constexpr int kCapWide = 2 * kCap4;  // wide column tiles (2 kNT4 threads) of the largest levels
constexpr int kNTT = 512;          // threads of the single-workgroup tail kernels
constexpr int kTailLog = 12;       // levels with L <= 2^12 run in the tail kernels
constexpr int kTailMaxLev = 16;    // levels one tail kernel call may span (first..last)

template <typename T>
struct Twiddles {
  const cplx<T>* base;  // kTwM entries
  const cplx<T>* lo;    // kTw4Lo entries
  const cplx<T>* hi;    // kTw4Hi entries
};

// One Toeplitz-plus-Cross level (eq. (split01)) as the kernels see it.
// n = v-size; the packed FFT signal z = v + i w_bar has L = 2(n+1) points.
// Four-step levels: L = L1 * L2 (L1 = row length), column tiles of T columns.
// Tail levels (whole FFT in one workgroup's LDS): logL2 = 0.
// Spectra: G1, G2 with Y[f] = G1[f] Z[f] + G2[f] conj(Z[-f]), already divided
// by L; stored at the position the row pass holds bin f (k1 + L1 k2 for
// f = k2 + L2 k1; natural order for tail levels).  sym: G1 real, G2 = i*g2
// (one real array each); otherwise interleaved complex arrays.
template <typename T>
struct LevelDev {
  int n;
  int logL, logL1, logL2, tcols;
  int sym;
  const T* g1;
  const T* g2;
  const T* p;
  const T* q;
  const T* xi;
  const T* zeta;
  T o, dv, dw;  // diagonal: a_0 (v rows), o (w_o row), d_0 (w_bar rows)
  T* b;         // level right-hand side (2n+1)
  T* u;         // level iterate (2n+1)
  T* r;         // level residual (2n+1)
  T* scal;      // scal[0]: y_o of the matvec in flight
  // tridiagonal band (weakly singular model; all null otherwise): couplings
  // of unknown i to i-1, i, i+1 on the block-ordered vector; dinv = 1 / the
  // full diagonal (Toeplitz part + band); bc = band product B x of the matvec
  // in flight (four-step levels)
  const T* bsub;
  const T* bmain;
  const T* bsup;
  const T* dinv;
  T* bc;
};

// Prologue of the forward column pass: how the FFT input vector is formed.
enum ColMode { COL_MV = 0, COL_PRE = 1, COL_PRE_RESTRICT = 2, COL_PROLONG = 3,
               COL_OUTER_UPDATE = 4, COL_SETUP = 5 };
// Epilogue of the inverse column pass.
enum EpiMode { EPI_MV = 0, EPI_RESID = 1, EPI_SMOOTH = 2, EPI_OUTER = 3 };

template <typename T>
struct ColIn {
  const T* x;          // COL_MV: input; COL_PRE_RESTRICT: fine residual; COL_PROLONG: coarse iterate
  T omega;             // COL_PRE / COL_PRE_RESTRICT
  double* xo;          // COL_OUTER_UPDATE: solution (updated in place)
  const void* e;       // COL_OUTER_UPDATE: correction (float or double)
  int e_is_float;
  const double* gx;    // COL_SETUP: generator of the real part's block
  const double* gy;    // COL_SETUP: generator of the imaginary part's block
};

template <typename T>
struct EpiOut {
  const T* xin;        // matvec input (its w_o feeds the Cross terms)
  T* y;                // EPI_MV output
  T omega;             // EPI_SMOOTH
  const double* bo;    // EPI_OUTER: right-hand side
  double* ro;          // EPI_OUTER: residual (FP64)
  float* r32;          // EPI_OUTER: FP32 copy of the residual (may be null)
  const double* ynear; // EPI_OUTER: near-field part of A x added to the FFT's
                       // far-field product (split residual; null: none)
};

// Steps of the small-level kernel: how a step forms its iterate (prologue)
// and what its epilogue writes.
enum TailPro { TP_PRE_B = 0, TP_PRE_RESTRICT, TP_USE_U, TP_PROLONG };
enum TailEpi { TE_RESID = 0, TE_SMOOTH };
// One step of a small-level program (W-cycles): a matvec step of `level`
// (pro, epi; post-smoothing damping when TAILOP_UP) or the coarsest solve.
enum TailOpFlags { TAILOP_COARSE = 1, TAILOP_UP = 2 };
struct TailOp {
  int level, pro, epi, flags;
};

// Coarsest level: A_c^{-1} (column-major m x m), formed at setup from the
// LU factors with partial pivoting; or the matrix of the V-cycle below a
// level folded into one operator.  ainv32: its FP32 rounding for the FP32
// V-cycle (null: the FP32 V-cycle reads ainv).
struct CoarseLU {
  int m;
  const double* ainv;
  const float* ainv32;
};

struct SolveState {
  double r0;
  double relres;
  double best;
  int iter;
  int status;
  int done;
  int cycle_end;  // GMRES: the current Arnoldi cycle has ended (update x next)
  // conjugate-gradient scalars (inner = AMG_INNER_PCG)
  double rz;     // <r, z> of the current direction
  double alpha;  // step length
  double beta;   // direction update
  double vtrue;  // last true residual formed to confirm a recurrence's (0: none yet)
  int cg_first;  // the next CG step starts a new direction sequence (p = z)
  int pad_;
};

// Arguments of one instance of a batched pass (block row blockIdx.y of a
// batched launch; the *_b kernels): the level, the prologue / epilogue
// operands, the FFT buffer and the partial-sum buffers of that instance's
// own launch, and its solve state with the gate that decides whether the
// instance takes part in this round.
enum PassGate { GATE_ACTIVE = 0, GATE_CG_STEP = 1, GATE_CG_CHECK = 2 };
template <typename T>
struct PassArgs {
  LevelDev<T> lv;
  ColIn<T> in;         // pass 1
  EpiOut<T> out;       // pass 3
  cplx<T>* buf;        // L complex
  T* part;             // pass 1 writes the w_o row's block partials, pass 2 reads them
  int npart;           // their count
  const T* xin;        // pass 2: the matvec input (its w_o)
  double* npart_out;   // pass 3 (EPI_OUTER): residual-norm block partials
  const SolveState* st;
  int gate;            // PassGate
};
// Whether an instance sits out a batched launch: solved, or (CG) in the other
// half of its round (a step of the recurrence vs the check of b - A x).  Read
// from state written by an earlier launch, so every thread of a block agrees.
__device__ __forceinline__ bool gate_skip(const SolveState* st, int gate) {
  if (!st) return false;
  if (st->done) return true;
  if (gate == GATE_CG_STEP) return st->cycle_end != 0;
  if (gate == GATE_CG_CHECK) return st->cycle_end == 0;
  return false;
}

// Stages of the conjugate-gradient scalar kernel (CG_AUTO: CG_INIT when the
// state's cg_first is set, else CG_BETA).
enum CgStage { CG_INIT = 0, CG_ALPHA = 1, CG_BETA = 2, CG_AUTO = 3 };

// Per-instance arguments of the batched small-level V-cycle and of the
// batched solver kernels (one block row per instance).
template <typename T>
struct TailArgs {
  const LevelDev<T>* levels;  // the handle's device level table
  int first, last;
  const T* rf;
  int m1, m2;
  T wpre, wpost;
  CoarseLU lu;
  const SolveState* st;
  int gate;
};
// The folded V-cycle below the four-step levels as one dense product (see
// launch_fold_gemv): per instance of a batch.
template <typename T>
struct FoldArgs {
  const T* rf;   // fine residual (2m + 1)
  const T* M;    // row-major m x m
  T* u;          // output (m)
  int m;
  const SolveState* st;
  int gate;
};
struct VdotArgs {           // part[2b] = a.z, part[2b+1] = c.z over chunk b
  const SolveState* st;
  int gate;
  const double* a;
  const void* z;            // float or double (one type per launch)
  const double* c;
  int64_t m;
  double* part;
};
struct CgArgs {             // scalar stage, direction, update of one instance
  SolveState* st;
  int gate;
  const double* part;       // cg_scalar: the vdot partials
  int nb;
  double* p;                // cg_dir, cg_update
  const void* z;            // cg_dir
  double* x;                // cg_update
  double* r;
  double* r_old;
  const double* q;
  float* r32;
  int64_t m;
  double* npart;            // cg_update: ||r||^2 partials
};
struct FinishArgs {         // stop test (k_finish / k_gm_check) of one instance
  SolveState* st;
  int gate;
  const double* part;
  int npart;
  double tol;
  int max_iter;
  double* hist;
  int verify;               // k_finish: recurrence residual; k_gm_check: stall rule
  SolveState* host;         // pinned copy of the state (may be null)
};

template <typename T>
hipError_t launch_tail_vcycle_batch(const TailArgs<T>* args, int count, int variant,
                                    const Twiddles<T>& tw, hipStream_t s);
template <typename T>
hipError_t launch_tail_matvec_batch(int colmode, int epimode, const PassArgs<T>* args, int count,
                                    const Twiddles<T>& tw, hipStream_t s);
template <typename TZ>
hipError_t launch_vdot_batch(const VdotArgs* args, int count, int64_t mmax, hipStream_t s);
hipError_t launch_cg_scalar_batch(const CgArgs* args, int count, int stage, hipStream_t s);
template <typename TZ>
hipError_t launch_cg_dir_batch(const CgArgs* args, int count, int64_t mmax, hipStream_t s);
hipError_t launch_cg_update_batch(const CgArgs* args, int count, int64_t mmax, hipStream_t s);
hipError_t launch_finish_batch(const FinishArgs* args, int count, hipStream_t s);
hipError_t launch_gm_check_batch(const FinishArgs* args, int count, hipStream_t s);

// Largest GMRES restart length (Krylov basis vectors per cycle).
constexpr int kGmMax = 64;
// Vectors per block row of the GMRES multi-dot kernel.
constexpr int kGmGroup = 8;

// Vector kernels: fixed contiguous chunks, one per block of kVecNT threads.
constexpr int kVecNT = 256;
__host__ __device__ inline int vec_blocks(int64_t m) {
  const int64_t b = (m + 2047) / 2048;
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}
__host__ __device__ inline int64_t vec_chunk(int64_t m) {
  const int nb = vec_blocks(m);
  return (m + nb - 1) / nb;
}

// ---- launchers (all asynchronous on `s`) ------------------------------------
template <typename T>
hipError_t launch_col_fwd(int mode, const LevelDev<T>& lv, const ColIn<T>& in, cplx<T>* buf,
                          const Twiddles<T>& tw, T* part, hipStream_t s);
template <typename T>
hipError_t launch_row(int spectral, const LevelDev<T>& lv, cplx<T>* buf, const Twiddles<T>& tw,
                      const T* part, int npart, const T* xin, hipStream_t s);
template <typename T>
hipError_t launch_col_inv(int mode, const LevelDev<T>& lv, const EpiOut<T>& out,
                          const cplx<T>* buf, const Twiddles<T>& tw, double* part, hipStream_t s);
// Batched forms of the three passes: `count` instances of the geometry of
// `geom`, per-instance arguments in the device table `args` (PassArgs).
template <typename T>
hipError_t launch_col_fwd_batch(int mode, const LevelDev<T>& geom, const PassArgs<T>* args,
                                int count, const Twiddles<T>& tw, hipStream_t s);
template <typename T>
hipError_t launch_row_batch(const LevelDev<T>& geom, const PassArgs<T>* args, int count,
                            const Twiddles<T>& tw, hipStream_t s);
template <typename T>
hipError_t launch_col_inv_batch(int mode, const LevelDev<T>& geom, const PassArgs<T>* args,
                                int count, const Twiddles<T>& tw, hipStream_t s);
template <typename T>
hipError_t launch_tail_matvec(int colmode, int epimode, const LevelDev<T>& lv, const ColIn<T>& in,
                              const EpiOut<T>& out, const Twiddles<T>& tw, double* part,
                              hipStream_t s);
// variant: TAIL_BAND if the levels carry a band, TAIL_SYM if their spectra
// are of the symmetric form (every tail level alike).
enum TailVariant { TAIL_BAND = 1, TAIL_SYM = 2 };
template <typename T>
hipError_t launch_tail_vcycle(const LevelDev<T>* levels_dev, int first, int last, const T* rf,
                              int m1, int m2, T wpre, T wpost, const CoarseLU& lu,
                              const Twiddles<T>& tw, int maxL, int variant, hipStream_t s);
template <typename T>
hipError_t launch_tail_program(const LevelDev<T>* levels_dev, int first, int last, const T* rf,
                               const TailOp* ops, int nops, T wpre, T wpost, const CoarseLU& lu,
                               const Twiddles<T>& tw, int maxL, int variant, hipStream_t s);
hipError_t launch_tail_fft_setup(const LevelDev<double>& lv, const double* gx, const double* gy,
                                 cplx<double>* out, const Twiddles<double>& tw, hipStream_t s);
hipError_t launch_combine(int logL, int logL1, int logL2, const cplx<double>* z1,
                          const cplx<double>* z2, int sym, double* g1, double* g2, float* g1f,
                          float* g2f, hipStream_t s);
// Stop test on sqrt(sum part) / r0.  verify != 0 (a recurrence's residual):
// passing the test sets cycle_end instead of done, and the true residual's
// check (launch_gm_check) decides.
hipError_t launch_finish(SolveState* st, const double* part, int npart, double tol, int max_iter,
                         double* hist, hipStream_t s, int verify = 0,
                         SolveState* host = nullptr);
hipError_t launch_copy_d2f(const double* a, float* b, int64_t m, hipStream_t s);
hipError_t launch_fill_hash(double* p, int64_t n, unsigned seed, hipStream_t s);
// u = M (R rf): R the restriction 1/4 [1 2 1] of the fine residual rf
// (2m + 1 entries) to m entries, M row-major m x m (m <= kFoldMax); FP64
// accumulation, one wavefront per row, kFoldRows rows per block.
constexpr int kFoldMax = 4095;
template <typename T, typename MT>
hipError_t launch_fold_gemv(const T* rf, int m, const MT* M, T* u, hipStream_t s);
template <typename T>
hipError_t launch_fold_gemv_batch(const FoldArgs<T>* args, int count, int m, hipStream_t s);
// Columns j0 .. j0+count-1 of a row-major m x m matrix from the vectors at
// src + k * stride (k = 0 .. count-1, m entries each).
hipError_t launch_gather_rows(double* M, const double* src, int64_t stride, int m, int j0,
                              int count, hipStream_t s);
// part[2b] = a.z, part[2b+1] = c.z over chunk b (c may be null); z FP64 or FP32
template <typename TZ>
hipError_t launch_vdot(const double* a, const TZ* z, const double* c, int64_t m, double* part,
                       hipStream_t s);
hipError_t launch_cg_scalar(SolveState* st, const double* part, int nb, int stage, hipStream_t s);
// x += alpha p; r_old = r; r -= alpha q; r32 = (float) r (if set); npart = ||r||^2 partials
hipError_t launch_cg_update(const SolveState* st, double* x, const double* p, double* r,
                            double* r_old, const double* q, float* r32, int64_t m, double* npart,
                            hipStream_t s);
// p = z (first) or p = z + beta p
template <typename TZ>
hipError_t launch_cg_dir(const SolveState* st, double* p, const TZ* z, int64_t m, int first,
                         hipStream_t s);

// ---- restarted flexible GMRES (inner = AMG_INNER_GMRES) ------------------
// The basis V (ld = m) and the preconditioned vectors Z (ld = m) are FP64;
// the Hessenberg matrix H is column-major with leading dimension kGmMax + 1;
// g, cs, sn are the rotated right-hand side and the Givens rotations.
// v0 = r / beta with beta = relres * r0 of the last residual; also written to
// the V-cycle input (vin64 or vin32, either may be null); g[0] = beta.
hipError_t launch_gm_start(const SolveState* st, const double* r, double* v0, double* g, int64_t m,
                           double* vin64, float* vin32, hipStream_t s);
// part[i * nb + blk] = <V[i], w> over chunk blk, i < cnt
hipError_t launch_gm_dot(const double* V, int cnt, const double* w, int64_t m, double* part,
                         hipStream_t s);
// hcur[i] = sum_blk part[i * nb + blk]; hcol[i] = (accumulate ? hcol[i] : 0) + hcur[i]
hipError_t launch_gm_reduce(const SolveState* st, const double* part, int nb, int cnt,
                            double* hcur, double* hcol, int accumulate, hipStream_t s);
// w -= sum_i hcur[i] V[i]; npart (if set) = ||w||^2 partials
hipError_t launch_gm_axpy(const SolveState* st, double* w, const double* V, const double* hcur,
                          int cnt, int64_t m, double* npart, hipStream_t s);
// h_{j+1,j} = ||w|| (from npart), rotations, residual estimate, stop test
hipError_t launch_gm_givens(SolveState* st, double* H, int j, double* cs, double* sn, double* g,
                            double* hn, const double* npart, int nb, double tol, int max_iter,
                            int restart, double* hist, hipStream_t s);
// v_{j+1} = w / h_{j+1,j} in place, also into the V-cycle input (unless the cycle ended)
hipError_t launch_gm_scale(const SolveState* st, double* w, const double* hn, int64_t m,
                           double* vin64, float* vin32, hipStream_t s);
// y = R^{-1} g (R = leading k x k block of the rotated H), x += Z y
hipError_t launch_gm_update(const SolveState* st, const double* H, const double* g, int k,
                            double* y, double* x, const double* Z, int64_t m, hipStream_t s);
// true residual norm (npart) -> relres, stop test, next cycle.  stall != 0:
// a true residual that is not below 0.9 times the previous one ends the solve
// (AMG_NOT_CONVERGED): the residual has reached what FP64 can resolve.
hipError_t launch_gm_check(SolveState* st, const double* npart, int nb, double tol, int max_iter,
                           double* hist, hipStream_t s, int stall = 0);
hipError_t launch_copy_f2d(const float* a, double* b, int64_t m, hipStream_t s);
hipError_t launch_publish(const SolveState* st, SolveState* host, hipStream_t s);
hipError_t launch_basis(double* b, int m, int j, hipStream_t s);
// b_j = e_j for j < m, b_j at base + j * stride
// Unit vectors e_{j0 + k} (m entries) at base + k * stride, k < count
// (count < 0: m vectors from j0 = 0).
hipError_t launch_basis_batch(double* base, int64_t stride, int m, hipStream_t s, int count = -1,
                              int j0 = 0);
// M[:, j] = u_j (column-major m x m), u_j at base + j * stride
hipError_t launch_gather_columns(double* M, const double* base, int64_t stride, int m,
                                 hipStream_t s);

// bc = B x for the level's band (2n+1 entries)
template <typename T>
hipError_t launch_band_mv(const LevelDev<T>& lv, const T* x, hipStream_t s);

// b = 4 u1 - 3 u2 + (4/3) u3 - (1/4) u4 + src (src may be null): the BDF4
// right-hand side
hipError_t launch_bdf4_rhs(const double* u1, const double* u2, const double* u3,
                           const double* u4, const double* src, double* b, int64_t m,
                           hipStream_t s);

// Near field of the split residual (amg_host.hpp NearField): y (block order,
// 2N-1 doubles) = sum_{0<|k|<=M} W(k) (x_{s+k} - x_s) + R_s x_s at every
// collocation position s; w = [node-row W | midpoint-row W] (2 (2M+1)
// doubles), rl / rr = R_s of the first / last M positions, rin_n / rin_m =
// R_s of the other node / midpoint positions.
constexpr int kNearM = 64;  // near offsets |k| <= kNearM half-steps
hipError_t launch_near(const double* x, double* y, int64_t N, const double* w, const double* rl,
                       const double* rr, double rin_n, double rin_m, hipStream_t s);

// One Toeplitz-plus-Cross level in device memory (setup): generators a, b,
// c, d (2n - 1 entries, offsets -(n-1)..n-1), Cross vectors p, q, xi, zeta
// (n entries) and the scalar o (one entry).
struct DevTpx {
  double *a, *b, *c, *d;
  double *p, *q, *xi, *zeta;
  double* o;
};
// The finest level from the node- and midpoint-row stencils (Wn[s2 + Sn],
// Wm[s2 + Sm]), scaled by `scale`, `shift` added to the diagonal entries.
hipError_t launch_finest_level(const double* Wn, int64_t Sn, const double* Wm, int64_t Sm,
                               int64_t n, double scale, double shift, const DevTpx& f, int* bad,
                               hipStream_t s);
// The Galerkin coarse level of f (v-size n) by Lemma 3.1 into c (v-size
// (n-1)/2); scratch holds 4 n doubles; sym: average the mirror entries
// (symmetric levels).  *bad becomes nonzero if an entry is not finite.
hipError_t launch_coarsen(const DevTpx& f, int64_t n, const DevTpx& c, double* scratch, bool sym,
                          int* bad, hipStream_t s);
// out[0..2] = o, a_0, d_0 of the level
hipError_t launch_level_scalars(const DevTpx& t, int64_t n, double* out, hipStream_t s);

// Column tiles / grid sizes used by the launchers (host helpers).
inline int col_blocks(int logL1, int tcols) { return (1 << logL1) / tcols; }

}  // namespace amg
