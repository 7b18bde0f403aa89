// HIP kernels of the block-structured V-cycle (Algorithm 2) with FFT-based
// Toeplitz-plus-Cross matrix-vector products (Sec. 3.2, eq. (ccs3.4),
// eq. (split01)) for gfx950.
//
// Each level's matvec works on the packed complex signal z = v + i w_bar
// (zero-padded to L = 2(n+1)); one complex FFT replaces the two real ones,
// and the 2x2 block product becomes, bin by bin,
//     Y[f] = G1[f] Z[f] + G2[f] conj(Z[-f]),
//     G1 = (A^ + D^ + i(C^ - B^))/2,  G2 = (A^ - D^ + i(C^ + B^))/2,
// with A^..D^ the spectra of the four circulant embeddings.  The inverse FFT
// of Y gives A v + B_bar w_bar in its real part and C_bar v + D_bar w_bar in
// its imaginary part.  Large levels run the FFT as a four-step transform in
// three HBM passes (column FFTs, row FFT + spectral product + inverse row FFT,
// inverse column FFTs) with the vector formation (smoothing, restriction,
// prolongation, refinement update) fused into the first pass and the residual
// / Jacobi epilogue fused into the last.  Small levels run the whole V-cycle
// below them in one workgroup with the FFT and its twiddles in LDS.
#include "kernel_common.hpp"

#include <type_traits>

namespace amg {

constexpr int kET = (1 << kTailLog) / kNTT;  // elements per thread, tail kernels

// ---------------------------------------------------------------------------
// Tail levels: L <= 2^12, one workgroup of 512 threads, FFT and twiddles in LDS.
// ---------------------------------------------------------------------------
// Dynamic LDS starts after a kernel's static LDS; it is declared 16-byte
// aligned so that the complex FP64 accesses (16-byte LDS instructions) stay
// aligned whatever the static variables add up to (an 8-byte offset made the
// FP64 FFT passes 3.5 times slower).
template <typename T>
struct TailLds {
  Lds<T> z;     // lds_slots(2^kTailLog) complex
  cplx<T>* tw;  // 2^kTailLog twiddles e^{-2 pi i m / 2^kTailLog}
  T* red;       // kNTT/64 wave partials + 2 broadcast slots
};

template <typename T>
__device__ TailLds<T> tail_lds(unsigned char* smem, const cplx<T>* tw_base) {
  TailLds<T> s;
  s.z.p = reinterpret_cast<cplx<T>*>(smem);
  s.tw = s.z.p + lds_slots(1 << kTailLog);
  s.red = reinterpret_cast<T*>(s.tw + (1 << kTailLog));
  for (int m = threadIdx.x; m < (1 << kTailLog); m += kNTT)
    s.tw[m] = tw_base[m << (kTwLog - kTailLog)];
  __syncthreads();
  return s;
}
constexpr size_t tail_lds_bytes(size_t elem) {
  return 2 * elem * ((size_t)lds_slots(1 << kTailLog) + (1 << kTailLog)) + elem * (kNTT / 64 + 2);
}

// The level descriptors a tail call visits, copied to LDS once at kernel start
// (one round trip instead of a dependent scalar load at every step), and read
// back as wave-uniform values so that their pointers stay scalar.
template <typename T>
__device__ __forceinline__ void tail_levels_to_lds(const LevelDev<T>* levels, int first, int last,
                                                   LevelDev<T>* lvs) {
  static_assert(sizeof(LevelDev<T>) % 4 == 0, "descriptor copied as 32-bit words");
  constexpr int W = sizeof(LevelDev<T>) / 4;
  const int total = (last - first + 1) * W;
  const unsigned* src = reinterpret_cast<const unsigned*>(levels + first);
  unsigned* dst = reinterpret_cast<unsigned*>(lvs);
  for (int i = threadIdx.x; i < total; i += kNTT) dst[i] = src[i];
}
// (Pointers are rebuilt through the global address space so that accesses
// through them compile to global, not flat, memory instructions.)
template <typename T>
__device__ __forceinline__ T* ptr_uniform(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  using G = __attribute__((address_space(1))) T;
  return (T*)(G*)(((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T val_uniform(T x) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
  } else {
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}
template <typename T>
__device__ __forceinline__ LevelDev<T> lv_uniform(const LevelDev<T>& x) {
  LevelDev<T> o;
  o.n = __builtin_amdgcn_readfirstlane(x.n);
  o.logL = __builtin_amdgcn_readfirstlane(x.logL);
  o.logL1 = __builtin_amdgcn_readfirstlane(x.logL1);
  o.logL2 = __builtin_amdgcn_readfirstlane(x.logL2);
  o.tcols = __builtin_amdgcn_readfirstlane(x.tcols);
  o.sym = __builtin_amdgcn_readfirstlane(x.sym);
  o.g1 = ptr_uniform(x.g1);
  o.g2 = ptr_uniform(x.g2);
  o.p = ptr_uniform(x.p);
  o.q = ptr_uniform(x.q);
  o.xi = ptr_uniform(x.xi);
  o.zeta = ptr_uniform(x.zeta);
  o.o = val_uniform(x.o);
  o.dv = val_uniform(x.dv);
  o.dw = val_uniform(x.dw);
  o.b = ptr_uniform(x.b);
  o.u = ptr_uniform(x.u);
  o.r = ptr_uniform(x.r);
  o.scal = ptr_uniform(x.scal);
  o.bsub = ptr_uniform(x.bsub);
  o.bmain = ptr_uniform(x.bmain);
  o.bsup = ptr_uniform(x.bsup);
  o.dinv = ptr_uniform(x.dinv);
  o.bc = ptr_uniform(x.bc);
  return o;
}

constexpr int kTailP = (1 << (kTailLog - 1)) / kNTT + 1;  // spectral pairs per thread (f <= L/2)

// Spectra of the pairs (f, L-f), f = threadIdx.x + k*kNTT, loaded into
// registers before the forward FFT so their latency overlaps it.
template <typename T>
struct TailSpec {
  cplx<T> a1[kTailP], a2[kTailP], b1[kTailP], b2[kTailP];  // G1[f], G2[f], G1[-f], G2[-f]
};

// Waves whose pairs all lie past L/2 skip the loads (a wave-uniform branch:
// on small levels most waves have nothing to load, and the cost of a load
// instruction is paid per wave); within a loading wave the pairs past L/2
// read bin 0 and are not used.
template <typename T, bool SYM>
__device__ __forceinline__ void tail_spec_load(const LevelDev<T>& lv, TailSpec<T>& sp) {
  const int L = 1 << lv.logL;
  const int wave0 = threadIdx.x & ~63;
#pragma unroll
  for (int k = 0; k < kTailP; ++k) {
    if (wave0 + k * kNTT > L / 2) continue;
    const int f0 = threadIdx.x + k * kNTT;
    const int f = f0 <= L / 2 ? f0 : 0;
    const int fb = (L - f) & (L - 1);
    if constexpr (SYM) {
      sp.a1[k] = {lv.g1[f], T(0)};
      sp.a2[k] = {T(0), lv.g2[f]};
      sp.b1[k] = {lv.g1[fb], T(0)};
      sp.b2[k] = {T(0), lv.g2[fb]};
    } else {
      const cplx<T>* G1 = reinterpret_cast<const cplx<T>*>(lv.g1);
      const cplx<T>* G2 = reinterpret_cast<const cplx<T>*>(lv.g2);
      sp.a1[k] = G1[f];
      sp.a2[k] = G2[f];
      sp.b1[k] = G1[fb];
      sp.b2[k] = G2[fb];
    }
  }
}

// z holds the packed input (zero-padded); leaves y_v + i y_w_bar (without the
// Cross terms) in z[0..n).
template <typename T>
__device__ void tail_fft_spectral(const LevelDev<T>& lv, const TailLds<T>& s, const TailSpec<T>& sp) {
  const int L = 1 << lv.logL;
  const FftGeom g{lv.logL, 0, 0, 0, kTailLog, false};
  // FP32: the two largest tail levels (most of the small-level kernel's FFT
  // work) with the geometry as compile-time constants, so the Stockham index
  // arithmetic folds; the others share one runtime-geometry copy (FP64 keeps
  // the one copy: the specialised ones need more registers than it has left)
  auto fft = [&](auto inv) {
    constexpr bool INV = decltype(inv)::value;
    if (sizeof(T) == 8) {
      lds_fft<T, kET, kNTT, INV>(s.z, g, s.tw);
    } else if (lv.logL == kTailLog) {
      constexpr FftGeom gc{kTailLog, 0, 0, 0, kTailLog, false};
      lds_fft<T, kET, kNTT, INV>(s.z, gc, s.tw);
    } else if (lv.logL == kTailLog - 1) {
      constexpr FftGeom gc{kTailLog - 1, 0, 0, 0, kTailLog, false};
      lds_fft<T, kET, kNTT, INV>(s.z, gc, s.tw);
    } else {
      lds_fft<T, kET, kNTT, INV>(s.z, g, s.tw);
    }
  };
  fft(std::false_type{});
#pragma unroll
  for (int k = 0; k < kTailP; ++k) {
    const int f = threadIdx.x + k * kNTT;
    if (f <= L / 2) {
      const int fb = (L - f) & (L - 1);
      const cplx<T> za = s.z[f], zb = s.z[fb];
      const cplx<T> ya = cmul(sp.a1[k], za) + cmul(sp.a2[k], conj(zb));
      const cplx<T> yb = cmul(sp.b1[k], zb) + cmul(sp.b2[k], conj(za));
      s.z[f] = ya;
      if (fb != f) s.z[fb] = yb;
    }
  }
  __syncthreads();
  fft(std::true_type{});
}

constexpr int kTailJ = (1 << (kTailLog - 1)) / kNTT;  // v/w slots per thread (n < L/2)

// One matvec step of a tail level: form u (prologue), y = A u, then the
// residual or Jacobi epilogue; b and u stay in registers between the two.
// The prologue issues the global loads of the step (spectra, Cross vectors,
// the prologue's operands, the w_o entry's) as one batch.  A load
// instruction costs the same per wave however few of its lanes are in range,
// so only waves holding elements j < n load (wave-uniform branches), and only
// the operands the prologue kind needs.
template <typename T, bool BAND, bool SYM>
__device__ __forceinline__ void tail_step(const LevelDev<T>& lv, int pro, int epi, const T* src,
                                          T wpro, T wepi, const TailLds<T>& s) {
  constexpr int J = kTailJ;
  const int n = lv.n, L = 1 << lv.logL;
  const bool restr = pro == TP_PRE_RESTRICT, prol = pro == TP_PROLONG;
  TailSpec<T> sp;
  tail_spec_load<T, SYM>(lv, sp);
  const T* pa = restr ? src : lv.b;            // slots 0, 1
  const T* pb = restr ? src : lv.u;            // slots 2, 3
  const T* pc = (restr || prol) ? src : lv.b;  // slots 4..7
  int jj[J];
  bool ok[J], ml0[J], mh0[J], ml1[J], mh1[J];
  T pj[J], xj[J], qq[J], zz[J], r0[J], r1[J], r2[J], r3[J], r4[J], r5[J], r6[J], r7[J];
  T dv0[J], dv1[J];
  const int wave0 = threadIdx.x & ~63;
  const bool six = restr || prol;  // operands 4 and 5
#pragma unroll
  for (int k = 0; k < J; ++k) {
    const int j = threadIdx.x + k * kNTT;
    ok[k] = j < n;
    const int js = ok[k] ? j : 0, jw = n + 1 + js;
    jj[k] = js;
    int lo0, hi0, lo1, hi1;
    prolong_idx(js, n, lo0, hi0, ml0[k], mh0[k]);
    prolong_idx(jw, n, lo1, hi1, ml1[k], mh1[k]);
    pj[k] = xj[k] = qq[k] = zz[k] = T(0);
    r0[k] = r1[k] = r2[k] = r3[k] = r4[k] = r5[k] = r6[k] = r7[k] = T(0);
    dv0[k] = dv1[k] = T(0);
    if (wave0 + k * kNTT >= n) continue;
    pj[k] = lv.p[js];
    xj[k] = lv.xi[js];
    qq[k] = lv.q[js];
    zz[k] = lv.zeta[js];
    r0[k] = pa[restr ? 2 * js : js];
    r1[k] = pa[restr ? 2 * js + 1 : jw];
    r2[k] = pb[restr ? 2 * js + 2 : js];
    r3[k] = pb[restr ? 2 * jw : jw];
    if (six) {
      r4[k] = pc[restr ? 2 * jw + 1 : lo0];
      r5[k] = pc[restr ? 2 * jw + 2 : hi0];
    }
    if (prol) {
      r6[k] = pc[lo1];
      r7[k] = pc[hi1];
    }
    if constexpr (BAND) {
      dv0[k] = lv.dinv[js];
      dv1[k] = lv.dinv[jw];
    }
  }
  // the w_o entry's operands (wave 0 loads them, one request each)
  int wlo, whi;
  bool wml, wmh;
  prolong_idx(n, n, wlo, whi, wml, wmh);
  T wo0 = T(0), wo1 = T(0), wo2 = T(0), wo3 = T(0), wdo = T(0);
  if (wave0 == 0) {
    wo0 = pa[restr ? 2 * n : n];
    wo1 = pb[restr ? 2 * n + 1 : n];
    wo2 = pc[restr ? 2 * n + 2 : (prol ? wlo : n)];
    wo3 = pc[prol ? whi : n];
    if constexpr (BAND) wdo = lv.dinv[n];
  }
  const T wo_b = restr ? T(0.25) * (wo0 + T(2) * wo1 + wo2) : wo0;
  const T wo_u = wo1;
  const T wo_x = T(0.5) * ((wml ? wo2 : T(0)) + (wmh ? wo3 : T(0)));
  T bv[J], bw[J], uv[J], uw[J];
  T dot = 0;
  const T wdv = wpro / lv.dv, wdw = wpro / lv.dw;
#pragma unroll
  for (int k = 0; k < J; ++k) {
    if (restr) {
      bv[k] = T(0.25) * (r0[k] + T(2) * r1[k] + r2[k]);
      bw[k] = T(0.25) * (r3[k] + T(2) * r4[k] + r5[k]);
    } else {
      bv[k] = r0[k];
      bw[k] = r1[k];
    }
    if (pro == TP_PRE_B || restr) {
      if constexpr (BAND) {
        uv[k] = wpro * bv[k] * dv0[k];
        uw[k] = wpro * bw[k] * dv1[k];
      } else {
        uv[k] = wdv * bv[k];
        uw[k] = wdw * bw[k];
      }
    } else if (prol) {
      uv[k] = r2[k] + T(0.5) * ((ml0[k] ? r4[k] : T(0)) + (mh0[k] ? r5[k] : T(0)));
      uw[k] = r3[k] + T(0.5) * ((ml1[k] ? r6[k] : T(0)) + (mh1[k] ? r7[k] : T(0)));
    } else {
      uv[k] = r2[k];
      uw[k] = r3[k];
    }
    if (!ok[k]) bv[k] = bw[k] = uv[k] = uw[k] = T(0);
  }
#pragma unroll
  for (int k = 0; k < J; ++k) {
    if (ok[k]) {
      const int j = jj[k], jw = n + 1 + j;
      if (pro == TP_PRE_RESTRICT) {
        lv.b[j] = bv[k];
        lv.b[jw] = bw[k];
      }
      if (pro != TP_USE_U) {
        lv.u[j] = uv[k];
        lv.u[jw] = uw[k];
      }
      s.z[j] = {uv[k], uw[k]};
      dot += qq[k] * uv[k] + zz[k] * uw[k];
    }
  }
  for (int j = n + threadIdx.x; j < L; j += kNTT) s.z[j] = {T(0), T(0)};
  if (threadIdx.x == 0) {  // the w_o entry
    const T bo = wo_b;
    if (restr) lv.b[n] = bo;
    T uo;
    if (pro == TP_PRE_B || restr) uo = wpro * bo * (BAND ? wdo : T(1) / lv.o);
    else if (prol) uo = wo_u + wo_x;
    else uo = wo_u;
    if (pro != TP_USE_U) lv.u[n] = uo;
    s.red[kNTT / 64] = uo;
    s.red[kNTT / 64 + 1] = bo;
  }
  const T qdot = block_sum<T, kNTT>(dot, s.red);  // also publishes z and the w_o slots
  const T uo = s.red[kNTT / 64], bo = s.red[kNTT / 64 + 1];
  constexpr bool band = BAND;  // weakly singular levels (the band's pointers are set)
  tail_fft_spectral(lv, s, sp);
  if constexpr (band) {
    // weakly singular levels: + B u with u read back from the level's iterate
    // (every thread stored or holds its part before the FFT's barriers); all
    // new values are formed before any is stored, so no neighbour is
    // overwritten while another thread still reads it
    auto bandu = [&](int i) {
      const int m = 2 * n + 1;
      T y = lv.bmain[i] * lv.u[i];
      if (i > 0) y += lv.bsub[i] * lv.u[i - 1];
      if (i + 1 < m) y += lv.bsup[i] * lv.u[i + 1];
      return y;
    };
    T nv[kTailJ], nw[kTailJ], no = T(0);
#pragma unroll
    for (int k = 0; k < kTailJ; ++k) {
      const int j = threadIdx.x + k * kNTT;
      nv[k] = nw[k] = T(0);
      if (j < n) {
        const int jw = n + 1 + j;
        const cplx<T> y = s.z[j];
        const T yv = y.x + pj[k] * uo + bandu(j), yw = y.y + xj[k] * uo + bandu(jw);
        nv[k] = epi == TE_RESID ? bv[k] - yv : uv[k] + wepi * (bv[k] - yv) * lv.dinv[j];
        nw[k] = epi == TE_RESID ? bw[k] - yw : uw[k] + wepi * (bw[k] - yw) * lv.dinv[jw];
      }
    }
    if (threadIdx.x == 0) {
      const T yo = qdot + lv.o * uo + bandu(n);
      no = epi == TE_RESID ? bo - yo : uo + wepi * (bo - yo) * lv.dinv[n];
    }
    __syncthreads();
    T* dst = epi == TE_RESID ? lv.r : lv.u;
#pragma unroll
    for (int k = 0; k < kTailJ; ++k) {
      const int j = threadIdx.x + k * kNTT;
      if (j < n) {
        dst[j] = nv[k];
        dst[n + 1 + j] = nw[k];
      }
    }
    if (threadIdx.x == 0) dst[n] = no;
  } else {
#pragma unroll
    for (int k = 0; k < kTailJ; ++k) {
      const int j = threadIdx.x + k * kNTT;
      if (j < n) {
        const int jw = n + 1 + j;
        const cplx<T> y = s.z[j];
        const T yv = y.x + pj[k] * uo, yw = y.y + xj[k] * uo;
        if (epi == TE_RESID) {
          lv.r[j] = bv[k] - yv;
          lv.r[jw] = bw[k] - yw;
        } else {
          lv.u[j] = uv[k] + (wepi / lv.dv) * (bv[k] - yv);
          lv.u[jw] = uw[k] + (wepi / lv.dw) * (bw[k] - yw);
        }
      }
    }
    if (threadIdx.x == 0) {
      const T yo = qdot + lv.o * uo;
      if (epi == TE_RESID) lv.r[n] = bo - yo;
      else lv.u[n] = uo + wepi * (bo - yo) / lv.o;
    }
  }
  __syncthreads();  // global writes visible to the next step; z and red reusable
}

// Coarsest level: u = A_c^{-1} b with the inverse formed at setup from the
// LU factors (partial pivoting), or the matrix of a folded sub-cycle.  b is
// staged in LDS as FP64.  When m rows leave threads idle, each row's dot
// product is split over P threads (P m <= kNTT, a power of two, at most 8):
// thread (k, i) sums the columns j = k mod P of row i in ascending order,
// eight loads in flight at a time (coalesced across i), and the P partial sums
// are added in k order through LDS.  The FP32 V-cycle reads the matrix's FP32
// rounding when there is one.
template <typename M>
__device__ __forceinline__ double coarse_row_part(const M* a, const double* bs, int m, int i,
                                                  int k, int P) {
  double acc = 0.0;
  int j = k;
  for (; j + 7 * P < m; j += 8 * P) {
    M v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = a[(j + q * P) * m + i];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += (double)v[q] * bs[j + q * P];
  }
  for (; j < m; j += P) acc += (double)a[j * m + i] * bs[j];
  return acc;
}
template <typename T, typename M>
__device__ void coarse_apply(const M* a, int m, const T* b, T* u, double* bs) {
  for (int i = threadIdx.x; i < m; i += kNTT) bs[i] = (double)b[i];
  __syncthreads();
  int P = 1;
  while (P < 8 && 2 * P * m <= kNTT) P *= 2;
  if (P == 1) {
    for (int i = threadIdx.x; i < m; i += kNTT) u[i] = (T)coarse_row_part(a, bs, m, i, 0, 1);
  } else {
    double* part = bs + m;  // P * m partial sums
    const int i = threadIdx.x % m, k = threadIdx.x / m;
    if (k < P) part[k * m + i] = coarse_row_part(a, bs, m, i, k, P);
    __syncthreads();
    for (int r = threadIdx.x; r < m; r += kNTT) {
      double acc = part[r];
      for (int q = 1; q < P; ++q) acc += part[q * m + r];
      u[r] = (T)acc;
    }
  }
  __syncthreads();
}
template <typename T>
__device__ void coarse_solve(const CoarseLU& lu, const T* b, T* u, double* bs) {
  if constexpr (sizeof(T) == 4) {
    if (lu.ainv32) {
      coarse_apply(lu.ainv32, lu.m, b, u, bs);
      return;
    }
  }
  coarse_apply(lu.ainv, lu.m, b, u, bs);
}

// Pulls the matrix coarse_solve will read into this XCD's L2 at kernel start
// (the large levels have evicted it since the previous cycle; a folded
// sub-cycle's matrix is up to 2 MB): one word per 128-byte line, in batches
// of 8 lines per thread with clamped addresses, folded into one value that is
// stored only if it equals a constant, so that the loads stay live.
template <typename T>
__device__ void coarse_warm(const CoarseLU& lu, T* sink) {
  const char* p = reinterpret_cast<const char*>(lu.ainv);
  long bytes = (long)lu.m * lu.m * 8;
  if constexpr (sizeof(T) == 4) {
    if (lu.ainv32) {
      p = reinterpret_cast<const char*>(lu.ainv32);
      bytes = (long)lu.m * lu.m * 4;
    }
  }
  constexpr int K = 8;
  constexpr long kBatch = (long)K * kNTT * 128;  // bytes covered per batch
  unsigned acc = 0;
  for (long base = 0; base < bytes; base += kBatch) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      long off = base + ((long)threadIdx.x + (long)k * kNTT) * 128;
      off = off < bytes ? off : bytes - 4;
      acc ^= *reinterpret_cast<const unsigned*>(p + off);
    }
  }
  if (acc == 0x5bd1e995u) sink[0] = T(0);
}

template <typename T, bool BAND, bool SYM>
__device__ __forceinline__ void tail_vcycle_body(const LevelDev<T>* levels, int first, int last,
                                                 const T* rf, int m1, int m2, T wpre, T wpost,
                                                 const CoarseLU& lu, const Twiddles<T>& tw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  __shared__ LevelDev<T> lvs[kTailMaxLev];
  __shared__ T warm_sink;
  tail_levels_to_lds(levels, first, last, lvs);
  coarse_warm<T>(lu, &warm_sink);  // under the twiddle table's loads
  const TailLds<T> s = tail_lds<T>(smem_raw, tw.base);  // its barrier publishes lvs too
  // One loop over the V-cycle's matvec steps (a single inlined tail_step):
  // descend (level first..last-1, m1 sweeps each, residual on the last one),
  // the coarsest solve, then ascend (prolongation + m2 post-sweeps).
  const int nlev = last - first;
  const int ndesc = nlev * m1;
  const int nsteps = ndesc + 1 + nlev * m2;
  for (int step = 0; step < nsteps; ++step) {
    if (step == ndesc) {  // coarsest level: b = R r_fine, exact solve by LU
      const LevelDev<T> lc = lv_uniform(lvs[last - first]);
      const T* src = (last == first) ? rf : ptr_uniform(lvs[last - 1 - first].r);
      if (src)
        for (int i = threadIdx.x; i < 2 * lc.n + 1; i += kNTT) lc.b[i] = restrict_at(src, i);
      __syncthreads();
      coarse_solve<T>(lu, lc.b, lc.u, reinterpret_cast<double*>(s.z.p));
      continue;
    }
    int l, pro, epi;
    const T* src;
    T wpro, wepi;
    if (step < ndesc) {
      l = first + step / m1;
      const int sweep = step - (l - first) * m1;  // 0-based
      const T* fine = (l == first) ? rf : ptr_uniform(lvs[l - 1 - first].r);
      pro = sweep > 0 ? TP_USE_U : (fine ? TP_PRE_RESTRICT : TP_PRE_B);
      epi = sweep == m1 - 1 ? TE_RESID : TE_SMOOTH;
      src = fine;
      wpro = wepi = wpre;
    } else {
      const int a = step - ndesc - 1;
      l = last - 1 - a / m2;
      const int sweep = a - (last - 1 - l) * m2;
      pro = sweep == 0 ? TP_PROLONG : TP_USE_U;
      epi = TE_SMOOTH;
      src = ptr_uniform(lvs[l + 1 - first].u);
      wpro = wepi = wpost;
    }
    tail_step<T, BAND, SYM>(lv_uniform(lvs[l - first]), pro, epi, src, wpro, wepi, s);
  }
}

template <typename T, bool BAND, bool SYM>
__global__ __launch_bounds__(kNTT) void k_tail_vcycle(const LevelDev<T>* levels, int first,
                                                      int last, const T* rf, int m1, int m2,
                                                      T wpre, T wpost, CoarseLU lu,
                                                      Twiddles<T> tw) {
  tail_vcycle_body<T, BAND, SYM>(levels, first, last, rf, m1, m2, wpre, wpost, lu, tw);
}
// One block per instance: the small levels of a batch of handles in one launch.
template <typename T, bool BAND, bool SYM>
__global__ __launch_bounds__(kNTT) void k_tail_vcycle_b(const TailArgs<T>* __restrict__ args,
                                                        Twiddles<T> tw) {
  const TailArgs<T>* a = args + blockIdx.x;
  if (gate_skip(a->st, a->gate)) return;
  const CoarseLU lu = a->lu;
  tail_vcycle_body<T, BAND, SYM>(a->levels, a->first, a->last, a->rf, a->m1, a->m2, a->wpre,
                                 a->wpost, lu, tw);
}

// A cycle's small-level part as a program of steps built on the host (the
// W-cycle: the second visit of a level smooths from its current iterate and
// recomputes the residual; see TailOp).
template <typename T, bool BAND, bool SYM>
__global__ __launch_bounds__(kNTT) void k_tail_program(const LevelDev<T>* levels, int first,
                                                       int last, const T* rf, const TailOp* ops,
                                                       int nops, T wpre, T wpost, CoarseLU lu,
                                                       Twiddles<T> tw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  __shared__ LevelDev<T> lvs[kTailMaxLev];
  __shared__ T warm_sink;
  tail_levels_to_lds(levels, first, last, lvs);
  coarse_warm<T>(lu, &warm_sink);  // under the twiddle table's loads
  const TailLds<T> s = tail_lds<T>(smem_raw, tw.base);  // its barrier publishes lvs too
  for (int k = 0; k < nops; ++k) {
    const TailOp op = ops[k];
    if (op.flags & TAILOP_COARSE) {  // coarsest level: b = R r_fine, exact solve
      const LevelDev<T> lc = lv_uniform(lvs[last - first]);
      const T* src = (last == first) ? rf : ptr_uniform(lvs[last - 1 - first].r);
      if (src)
        for (int i = threadIdx.x; i < 2 * lc.n + 1; i += kNTT) lc.b[i] = restrict_at(src, i);
      __syncthreads();
      coarse_solve<T>(lu, lc.b, lc.u, reinterpret_cast<double*>(s.z.p));
      continue;
    }
    const int l = op.level;
    const T* src = nullptr;
    if (op.pro == TP_PRE_RESTRICT) src = (l == first) ? rf : ptr_uniform(lvs[l - 1 - first].r);
    if (op.pro == TP_PROLONG) src = ptr_uniform(lvs[l + 1 - first].u);
    const T w = (op.flags & TAILOP_UP) ? wpost : wpre;
    tail_step<T, BAND, SYM>(lv_uniform(lvs[l - first]), op.pro, op.epi, src, w, w, s);
  }
}

// One tail-level matvec: y = A x (EPI_MV) or the outer residual with the
// refinement update fused in front (COL_OUTER_UPDATE + EPI_OUTER).
template <typename T, int CM, int EM>
__device__ __forceinline__ void tail_matvec_body(const LevelDev<T>& lv, const ColIn<T>& in,
                                                 const EpiOut<T>& out, const Twiddles<T>& tw,
                                                 double* part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const TailLds<T> s = tail_lds<T>(smem_raw, tw.base);
  __shared__ double redd[kNTT / 64];
  const int n = lv.n, L = 1 << lv.logL;
  const T* x = out.xin;
  if constexpr (CM == COL_OUTER_UPDATE) {
    for (int i = threadIdx.x; i < 2 * n + 1; i += kNTT) {
      const double e = in.e_is_float ? (double)((const float*)in.e)[i] : ((const double*)in.e)[i];
      in.xo[i] += e;
    }
    __syncthreads();
  }
  T dot = 0;
  for (int j = threadIdx.x; j < L; j += kNTT) {
    cplx<T> v = {T(0), T(0)};
    if (j < n) {
      v = {x[j], x[n + 1 + j]};
      dot += lv.q[j] * v.x + lv.zeta[j] * v.y;
    }
    s.z[j] = v;
  }
  TailSpec<T> sp;
  if (lv.sym)
    tail_spec_load<T, true>(lv, sp);
  else
    tail_spec_load<T, false>(lv, sp);
  // band product of x (weakly singular levels) at index i of the block-ordered vector
  auto bandx = [&](int i) {
    const int m = 2 * n + 1;
    T y = lv.bmain[i] * x[i];
    if (i > 0) y += lv.bsub[i] * x[i - 1];
    if (i + 1 < m) y += lv.bsup[i] * x[i + 1];
    return y;
  };
  const bool band = lv.bmain != nullptr;
  const T yo = block_sum<T, kNTT>(dot, s.red) + lv.o * x[n] + (band ? bandx(n) : T(0));
  tail_fft_spectral(lv, s, sp);
  const T wo = x[n];
  double ss = 0.0;
  for (int j = threadIdx.x; j < n; j += kNTT) {
    const cplx<T> z = s.z[j];
    T yv = z.x + lv.p[j] * wo, yw = z.y + lv.xi[j] * wo;
    if (band) {
      yv += bandx(j);
      yw += bandx(n + 1 + j);
    }
    if constexpr (EM == EPI_MV) {
      out.y[j] = yv;
      out.y[n + 1 + j] = yw;
    } else {
      const double qv = out.ynear ? out.ynear[j] : 0.0, qw = out.ynear ? out.ynear[n + 1 + j] : 0.0;
      const double rv = out.bo[j] - ((double)yv + qv), rw = out.bo[n + 1 + j] - ((double)yw + qw);
      out.ro[j] = rv;
      out.ro[n + 1 + j] = rw;
      if (out.r32) {
        out.r32[j] = (float)rv;
        out.r32[n + 1 + j] = (float)rw;
      }
      ss += rv * rv + rw * rw;
    }
  }
  if (threadIdx.x == 0) {
    if constexpr (EM == EPI_MV) {
      out.y[n] = yo;
    } else {
      const double ro = out.bo[n] - ((double)yo + (out.ynear ? out.ynear[n] : 0.0));
      out.ro[n] = ro;
      if (out.r32) out.r32[n] = (float)ro;
      ss += ro * ro;
    }
  }
  if constexpr (EM == EPI_OUTER) {
    const double sum = block_sum<double, kNTT>(ss, redd);
    if (threadIdx.x == 0) part[0] = sum;
  }
}

template <typename T, int CM, int EM>
__global__ __launch_bounds__(kNTT) void k_tail_matvec(LevelDev<T> lv, ColIn<T> in, EpiOut<T> out,
                                                      Twiddles<T> tw, double* part) {
  tail_matvec_body<T, CM, EM>(lv, in, out, tw, part);
}
template <typename T, int CM, int EM>
__global__ __launch_bounds__(kNTT) void k_tail_matvec_b(const PassArgs<T>* __restrict__ args,
                                                        Twiddles<T> tw) {
  const PassArgs<T>* a = args + blockIdx.x;
  if (gate_skip(a->st, a->gate)) return;
  const LevelDev<T> lv = a->lv;
  const ColIn<T> in = a->in;
  const EpiOut<T> out = a->out;
  tail_matvec_body<T, CM, EM>(lv, in, out, tw, a->npart_out);
}

// Setup: FFT (natural order) of c_x + i c_y for a tail level.
__global__ __launch_bounds__(kNTT) void k_tail_fft_setup(LevelDev<double> lv, const double* gx,
                                                         const double* gy, cplx<double>* out,
                                                         Twiddles<double> tw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const TailLds<double> s = tail_lds<double>(smem_raw, tw.base);
  const int n = lv.n, L = 1 << lv.logL;
  for (int j = threadIdx.x; j < L; j += kNTT) s.z[j] = {circ_col(gx, n, L, j), circ_col(gy, n, L, j)};
  __syncthreads();
  const FftGeom g{lv.logL, 0, 0, 0, kTailLog, false};
  lds_fft<double, kET, kNTT, false>(s.z, g, s.tw);
  for (int j = threadIdx.x; j < L; j += kNTT) out[j] = s.z[j];
}

// Setup: spectra of the four blocks from two packed transforms
// Z1 = F(c_A + i c_B), Z2 = F(c_C + i c_D); A^ = (Z1 + conj Z1(-f))/2,
// B^ = (Z1 - conj Z1(-f))/(2i), etc.; G1, G2 as above, divided by L.
__global__ void k_combine(int logL, int logL1, int logL2, const cplx<double>* z1,
                          const cplx<double>* z2, int sym, double* g1, double* g2, float* g1f,
                          float* g2f) {
  const int L = 1 << logL;
  const int pos = blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= L) return;
  int pp;
  if (logL2 == 0) {
    pp = (L - pos) & (L - 1);
  } else {
    const int L1 = 1 << logL1, L2 = 1 << logL2;
    const int k2 = pos >> logL1, k1 = pos & (L1 - 1);
    const int f = k2 + L2 * k1;
    const int fn = (L - f) & (L - 1);
    pp = (fn & (L2 - 1)) * L1 + (fn >> logL2);
  }
  const cplx<double> a1 = z1[pos], b1 = conj(z1[pp]), a2 = z2[pos], b2 = conj(z2[pp]);
  const cplx<double> Ah = scale(a1 + b1, 0.5), Ch = scale(a2 + b2, 0.5);
  const cplx<double> Bh = scale(rot<double, false>(a1 - b1), 0.5);  // (z - conj)/(2i)
  const cplx<double> Dh = scale(rot<double, false>(a2 - b2), 0.5);
  const double sc = 0.5 / (double)L;
  const cplx<double> G1 = scale((Ah + Dh) + rot<double, true>(Ch - Bh), sc);
  const cplx<double> G2 = scale((Ah - Dh) + rot<double, true>(Ch + Bh), sc);
  if (sym) {
    g1[pos] = G1.x;
    g2[pos] = G2.y;
    if (g1f) {
      g1f[pos] = (float)G1.x;
      g2f[pos] = (float)G2.y;
    }
  } else {
    g1[2 * pos] = G1.x;
    g1[2 * pos + 1] = G1.y;
    g2[2 * pos] = G2.x;
    g2[2 * pos + 1] = G2.y;
    if (g1f) {
      g1f[2 * pos] = (float)G1.x;
      g1f[2 * pos + 1] = (float)G1.y;
      g2f[2 * pos] = (float)G2.x;
      g2f[2 * pos + 1] = (float)G2.y;
    }
  }
}

// Stopping test of the outer iteration (Sec. 5): ||r_i|| / ||r_0|| < tol.
// host != null: the state is also written to pinned host memory at the end
// (the round's last kernel publishes it itself; see k_publish).
__device__ void finish_state(SolveState* st, double s, double tol, int max_iter, double* hist,
                             int verify) {
  if (st->done) return;
  const double nrm = sqrt(s);
  if (st->iter == 0) {
    st->r0 = nrm;
    st->best = 1.0;
  }
  const double rel = (st->r0 > 0.0) ? nrm / st->r0 : 0.0;
  st->relres = rel;
  hist[st->iter] = rel;
  if (!(rel == rel) || isinf(rel)) {
    st->status = 2;
    st->done = 1;
  } else if (rel < tol) {
    if (verify) {  // a recurrence's residual: b - A x decides (k_gm_check)
      st->cycle_end = 1;
    } else {
      st->status = 0;
      st->done = 1;
    }
  } else if (rel > 1e3 * st->best) {
    st->status = 2;
    st->done = 1;
  } else if (st->iter >= max_iter) {
    st->status = 1;
    st->done = 1;
  }
  if (rel < st->best) st->best = rel;
  if (!st->done && !st->cycle_end) st->iter += 1;
}
__global__ __launch_bounds__(256) void k_finish(SolveState* st, const double* part, int npart,
                                                double tol, int max_iter, double* hist,
                                                int verify, SolveState* host) {
  __shared__ double red[256 / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < npart; i += 256) v += part[i];
  const double s = block_sum<double, 256>(v, red);
  if (threadIdx.x == 0) finish_state(st, s, tol, max_iter, hist, verify);
  if (host) {
    __syncthreads();  // thread 0's state writes before the copy
    constexpr int W = sizeof(SolveState) / 4;
    if (threadIdx.x < W)
      reinterpret_cast<unsigned*>(host)[threadIdx.x] = reinterpret_cast<const unsigned*>(st)[threadIdx.x];
    __threadfence_system();
  }
}

__global__ __launch_bounds__(256) void k_finish_b(const FinishArgs* __restrict__ args) {
  __shared__ double red[256 / 64];
  const FinishArgs* a = args + blockIdx.x;
  if (gate_skip(a->st, a->gate)) return;
  double v = 0.0;
  for (int i = threadIdx.x; i < a->npart; i += 256) v += a->part[i];
  const double s = block_sum<double, 256>(v, red);
  if (threadIdx.x == 0) finish_state(a->st, s, a->tol, a->max_iter, a->hist, a->verify);
  if (a->host) {
    __syncthreads();  // thread 0's state writes before the copy
    constexpr int W = sizeof(SolveState) / 4;
    if (threadIdx.x < W)
      reinterpret_cast<unsigned*>(a->host)[threadIdx.x] =
          reinterpret_cast<const unsigned*>(a->st)[threadIdx.x];
    __threadfence_system();
  }
}

__global__ void k_copy_d2f(const double* a, float* b, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------
// Conjugate gradients preconditioned by the V-cycle (SPD case).  Dot products
// and norms sum fixed contiguous chunks (one per block) and reduce the block
// partials in index order, so every run gives the same bits.  The scalars
// live in the solve state on the device; a finished solve (done) leaves them
// and the vectors untouched.
// ---------------------------------------------------------------------------
template <typename TZ>
__device__ __forceinline__ void vdot_body(const double* a, const TZ* z, const double* c, int64_t m,
                                          int64_t chunk, double* part) {
  __shared__ double red[kVecNT / 64];
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = i0 + chunk < m ? i0 + chunk : m;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kVecNT) {
    const double zi = (double)z[i];
    s0 += a[i] * zi;
    if (c) s1 += c[i] * zi;
  }
  s0 = block_sum<double, kVecNT>(s0, red);
  s1 = block_sum<double, kVecNT>(s1, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0;
    part[2 * blockIdx.x + 1] = s1;
  }
}
template <typename TZ>
__global__ __launch_bounds__(kVecNT) void k_vdot(const double* a, const TZ* z, const double* c,
                                                 int64_t m, int64_t chunk, double* part) {
  vdot_body<TZ>(a, z, c, m, chunk, part);
}
// Batched: block (x, y) is chunk x of instance y (the instance's own
// partition: vec_blocks(m) chunks of vec_chunk(m)).
template <typename TZ>
__global__ __launch_bounds__(kVecNT) void k_vdot_b(const VdotArgs* __restrict__ args) {
  const VdotArgs* g = args + blockIdx.y;
  if (gate_skip(g->st, g->gate)) return;
  if ((int)blockIdx.x >= vec_blocks(g->m)) return;
  vdot_body<TZ>(g->a, static_cast<const TZ*>(g->z), g->c, g->m, vec_chunk(g->m), g->part);
}

__device__ __forceinline__ void cg_scalar_body(SolveState* st, const double* part, int nb,
                                               int stage) {
  __shared__ double red[kVecNT / 64];
  double v0 = 0.0, v1 = 0.0;
  for (int i = threadIdx.x; i < nb; i += kVecNT) {
    v0 += part[2 * i];
    v1 += part[2 * i + 1];
  }
  v0 = block_sum<double, kVecNT>(v0, red);
  v1 = block_sum<double, kVecNT>(v1, red);
  if (threadIdx.x != 0 || st->done) return;
  bool bad = !(v0 > 0.0) || isinf(v0);  // <r, z> and <p, A p> must be positive (SPD)
  if (stage == CG_INIT) {
    st->rz = v0;
    st->beta = 0.0;
  } else if (stage == CG_ALPHA) {
    st->alpha = st->rz / v0;
  } else {
    // Polak-Ribiere: <z_new, r_new - r_old> / <z_old, r_old>
    st->beta = (v0 - v1) / st->rz;
    st->rz = v0;
  }
  if (bad) {
    st->status = 2;  // AMG_DIVERGED: the operator or the preconditioner is not SPD
    st->done = 1;
  }
}
__global__ __launch_bounds__(kVecNT) void k_cg_scalar(SolveState* st, const double* part, int nb,
                                                      int stage) {
  cg_scalar_body(st, part, nb, stage);
}
__global__ __launch_bounds__(kVecNT) void k_cg_scalar_b(const CgArgs* __restrict__ args,
                                                        int stage) {
  const CgArgs* g = args + blockIdx.x;
  if (gate_skip(g->st, g->gate)) return;
  const int sg = stage == CG_AUTO ? (g->st->cg_first ? CG_INIT : CG_BETA) : stage;
  cg_scalar_body(g->st, g->part, g->nb, sg);
}

__device__ __forceinline__ void cg_update_body(const SolveState* st, double* x, const double* p,
                                               double* r, double* r_old, const double* q,
                                               float* r32, int64_t m, int64_t chunk,
                                               double* npart) {
  __shared__ double red[kVecNT / 64];
  if (st->done) return;  // uniform: every thread of every block returns
  const double alpha = st->alpha;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = i0 + chunk < m ? i0 + chunk : m;
  double ss = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kVecNT) {
    x[i] += alpha * p[i];
    const double ro = r[i], rn = ro - alpha * q[i];
    r_old[i] = ro;
    r[i] = rn;
    if (r32) r32[i] = (float)rn;
    ss += rn * rn;
  }
  ss = block_sum<double, kVecNT>(ss, red);
  if (threadIdx.x == 0) npart[blockIdx.x] = ss;
}
__global__ __launch_bounds__(kVecNT) void k_cg_update(const SolveState* st, double* x,
                                                      const double* p, double* r, double* r_old,
                                                      const double* q, float* r32, int64_t m,
                                                      int64_t chunk, double* npart) {
  cg_update_body(st, x, p, r, r_old, q, r32, m, chunk, npart);
}
// Batched; block 0 also clears the instance's cg_first (the direction of
// this step has been formed).
__global__ __launch_bounds__(kVecNT) void k_cg_update_b(const CgArgs* __restrict__ args) {
  const CgArgs* g = args + blockIdx.y;
  if (gate_skip(g->st, g->gate)) return;
  if ((int)blockIdx.x >= vec_blocks(g->m)) return;
  cg_update_body(g->st, g->x, g->p, g->r, g->r_old, g->q, g->r32, g->m, vec_chunk(g->m), g->npart);
  if (blockIdx.x == 0 && threadIdx.x == 0) g->st->cg_first = 0;
}

// ---------------------------------------------------------------------------
// Restarted flexible GMRES (right preconditioner = one V-cycle per step).
// Classical Gram-Schmidt applied twice: each pass is one multi-dot (all
// <v_i, w> of the pass in one launch, fixed-order block partials) and one
// update; the small dense work (Givens rotations, the triangular solve) runs
// in one thread.  Every kernel returns at once when the solve is done.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kVecNT) void k_gm_start(const SolveState* st, const double* r,
                                                     double* v0, double* g, int64_t m,
                                                     double* vin64, float* vin32) {
  if (st->done) return;
  const double beta = st->relres * st->r0;
  const double inv = 1.0 / beta;
  const int64_t i = (int64_t)blockIdx.x * kVecNT + threadIdx.x;
  if (i == 0) g[0] = beta;
  if (i >= m) return;
  const double v = r[i] * inv;
  v0[i] = v;
  if (vin64) vin64[i] = v;
  if (vin32) vin32[i] = (float)v;
}

__global__ __launch_bounds__(kVecNT) void k_gm_dot(const double* V, int cnt, const double* w,
                                                   int64_t m, int64_t chunk, double* part) {
  __shared__ double red[kVecNT / 64];
  const int g0 = blockIdx.y * kGmGroup;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = i0 + chunk < m ? i0 + chunk : m;
  double acc[kGmGroup];
#pragma unroll
  for (int k = 0; k < kGmGroup; ++k) acc[k] = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kVecNT) {
    const double wi = w[i];
#pragma unroll
    for (int k = 0; k < kGmGroup; ++k)
      if (g0 + k < cnt) acc[k] += V[(int64_t)(g0 + k) * m + i] * wi;
  }
#pragma unroll
  for (int k = 0; k < kGmGroup; ++k) {
    const double t = block_sum<double, kVecNT>(acc[k], red);
    if (threadIdx.x == 0 && g0 + k < cnt) part[(int64_t)(g0 + k) * gridDim.x + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kVecNT) void k_gm_reduce(const SolveState* st, const double* part,
                                                      int nb, int cnt, double* hcur, double* hcol,
                                                      int accumulate) {
  __shared__ double red[kVecNT / 64];
  if (st->done) return;
  for (int k = 0; k < cnt; ++k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kVecNT) v += part[(int64_t)k * nb + b];
    v = block_sum<double, kVecNT>(v, red);
    if (threadIdx.x == 0) {
      hcur[k] = v;
      hcol[k] = accumulate ? hcol[k] + v : v;
    }
  }
}

__global__ __launch_bounds__(kVecNT) void k_gm_axpy(const SolveState* st, double* w,
                                                    const double* V, const double* hcur, int cnt,
                                                    int64_t m, int64_t chunk, double* npart) {
  __shared__ double red[kVecNT / 64];
  __shared__ double hs[kGmMax + 1];
  if (st->done) return;
  for (int k = threadIdx.x; k < cnt; k += kVecNT) hs[k] = hcur[k];
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = i0 + chunk < m ? i0 + chunk : m;
  double ss = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kVecNT) {
    double v = w[i];
    for (int k = 0; k < cnt; ++k) v -= hs[k] * V[(int64_t)k * m + i];
    w[i] = v;
    ss += v * v;
  }
  if (npart) {
    ss = block_sum<double, kVecNT>(ss, red);
    if (threadIdx.x == 0) npart[blockIdx.x] = ss;
  }
}

__global__ __launch_bounds__(kVecNT) void k_gm_givens(SolveState* st, double* H, int j,
                                                      double* cs, double* sn, double* g,
                                                      double* hn_out, const double* npart, int nb,
                                                      double tol, int max_iter, int restart,
                                                      double* hist) {
  __shared__ double red[kVecNT / 64];
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += kVecNT) v += npart[b];
  v = block_sum<double, kVecNT>(v, red);
  if (threadIdx.x != 0 || st->done) return;
  const double hn = sqrt(v);
  *hn_out = hn;
  double* Hj = H + (int64_t)j * (kGmMax + 1);
  Hj[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = Hj[i], c = Hj[i + 1];
    Hj[i] = cs[i] * a + sn[i] * c;
    Hj[i + 1] = -sn[i] * a + cs[i] * c;
  }
  const double d = hypot(Hj[j], Hj[j + 1]);
  if (!(d > 0.0) || isinf(d)) {  // singular or non-finite Hessenberg column
    st->status = 2;
    st->done = 1;
    return;
  }
  cs[j] = Hj[j] / d;
  sn[j] = Hj[j + 1] / d;
  Hj[j] = d;
  Hj[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  const double est = fabs(g[j + 1]) / st->r0;
  st->relres = est;
  hist[st->iter] = est;
  if (!(est == est) || isinf(est)) {
    st->status = 2;
    st->done = 1;
    return;
  }
  if (est < tol || j + 1 >= restart || st->iter >= max_iter || hn == 0.0)
    st->cycle_end = 1;
  else
    st->iter += 1;
}

__global__ __launch_bounds__(kVecNT) void k_gm_scale(const SolveState* st, double* w,
                                                     const double* hn, int64_t m, double* vin64,
                                                     float* vin32) {
  if (st->done || st->cycle_end) return;
  const int64_t i = (int64_t)blockIdx.x * kVecNT + threadIdx.x;
  if (i >= m) return;
  const double v = w[i] / *hn;
  w[i] = v;
  if (vin64) vin64[i] = v;
  if (vin32) vin32[i] = (float)v;
}

__global__ void k_gm_solve(const SolveState* st, const double* H, const double* g, int k,
                           double* y) {
  if (threadIdx.x != 0 || st->done) return;
  for (int i = k - 1; i >= 0; --i) {
    double v = g[i];
    for (int l = i + 1; l < k; ++l) v -= H[(int64_t)l * (kGmMax + 1) + i] * y[l];
    y[i] = v / H[(int64_t)i * (kGmMax + 1) + i];
  }
}

__global__ __launch_bounds__(kVecNT) void k_gm_xupdate(const SolveState* st, double* x,
                                                       const double* Z, const double* y, int k,
                                                       int64_t m) {
  __shared__ double ys[kGmMax];
  if (st->done) return;
  for (int l = threadIdx.x; l < k; l += kVecNT) ys[l] = y[l];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kVecNT + threadIdx.x;
  if (i >= m) return;
  double v = x[i];
  for (int l = 0; l < k; ++l) v += ys[l] * Z[(int64_t)l * m + i];
  x[i] = v;
}

__device__ __forceinline__ void gm_check_state(SolveState* st, double v, double tol, int max_iter,
                                               double* hist, int stall) {
  if (st->done) return;
  const double rel = sqrt(v) / st->r0;
  st->relres = rel;
  hist[st->iter] = rel;
  st->cycle_end = 0;
  if (!(rel == rel) || isinf(rel)) {
    st->status = 2;
    st->done = 1;
  } else if (rel < tol) {
    st->status = 0;
    st->done = 1;
  } else if (st->iter >= max_iter || (stall && st->vtrue > 0.0 && rel >= 0.9 * st->vtrue)) {
    st->status = 1;
    st->done = 1;
  } else {
    st->iter += 1;
    // the next recurrence starts from this residual: the growth test of
    // finish_state measures from here (a Krylov method's 2-norm residual is
    // not monotone, and a restart can start above the recurrence's minimum)
    st->best = rel;
    st->cg_first = 1;  // CG restarts from it
  }
  st->vtrue = rel;
}
__global__ __launch_bounds__(kVecNT) void k_gm_check(SolveState* st, const double* npart, int nb,
                                                     double tol, int max_iter, double* hist,
                                                     int stall) {
  __shared__ double red[kVecNT / 64];
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += kVecNT) v += npart[b];
  v = block_sum<double, kVecNT>(v, red);
  if (threadIdx.x == 0) gm_check_state(st, v, tol, max_iter, hist, stall);
}
__global__ __launch_bounds__(kVecNT) void k_gm_check_b(const FinishArgs* __restrict__ args) {
  __shared__ double red[kVecNT / 64];
  const FinishArgs* a = args + blockIdx.x;
  if (gate_skip(a->st, a->gate)) return;
  double v = 0.0;
  for (int b = threadIdx.x; b < a->npart; b += kVecNT) v += a->part[b];
  v = block_sum<double, kVecNT>(v, red);
  if (threadIdx.x == 0) gm_check_state(a->st, v, a->tol, a->max_iter, a->hist, a->verify);
  if (a->host) {
    __syncthreads();
    constexpr int W = sizeof(SolveState) / 4;
    if (threadIdx.x < W)
      reinterpret_cast<unsigned*>(a->host)[threadIdx.x] =
          reinterpret_cast<const unsigned*>(a->st)[threadIdx.x];
    __threadfence_system();
  }
}

// The solve state into pinned host memory (the host's view of the round):
// written by the device directly instead of a copy command.
__global__ void k_publish(const SolveState* st, SolveState* host) {
  const int w = threadIdx.x;
  constexpr int W = sizeof(SolveState) / 4;
  if (w < W) reinterpret_cast<unsigned*>(host)[w] = reinterpret_cast<const unsigned*>(st)[w];
  __threadfence_system();
}
hipError_t launch_publish(const SolveState* st, SolveState* host, hipStream_t s) {
  static_assert(sizeof(SolveState) % 4 == 0 && sizeof(SolveState) / 4 <= 64, "state words");
  hipLaunchKernelGGL(k_publish, 1, 64, 0, s, st, host);
  return hipGetLastError();
}

// b = e_j (length m): the unit vectors a setup applies the V-cycle to.
__global__ void k_basis(double* b, int m, int j) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = i == j ? 1.0 : 0.0;
}
// Column j of a batch of unit-vector right-hand sides: b_j = e_j, where b_j
// starts at base + j * stride (m entries each, m columns).
__global__ void k_basis_batch(double* base, int64_t stride, int m, int j0) {
  const int j = blockIdx.y;
  double* b = base + (int64_t)j * stride;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    b[i] = i == j0 + j ? 1.0 : 0.0;
}
hipError_t launch_basis_batch(double* base, int64_t stride, int m, hipStream_t s, int count,
                              int j0) {
  if (count < 0) count = m;
  if (m < 1 || count < 1 || count > 65535 || j0 < 0 || j0 + count > m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_basis_batch, dim3((m + 255) / 256, count), 256, 0, s, base, stride, m, j0);
  return hipGetLastError();
}
// M[:, j] = u_j (column-major m x m), u_j at base + j * stride.
__global__ void k_gather_columns(double* M, const double* base, int64_t stride, int m) {
  const int j = blockIdx.y;
  const double* u = base + (int64_t)j * stride;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    M[(int64_t)j * m + i] = u[i];
}
hipError_t launch_gather_columns(double* M, const double* base, int64_t stride, int m,
                                 hipStream_t s) {
  if (m < 1 || m > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_columns, dim3((m + 255) / 256, m), 256, 0, s, M, base, stride, m);
  return hipGetLastError();
}

hipError_t launch_basis(double* b, int m, int j, hipStream_t s) {
  hipLaunchKernelGGL(k_basis, (m + 255) / 256, 256, 0, s, b, m, j);
  return hipGetLastError();
}

__global__ void k_copy_f2d(const float* a, double* b, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = (double)a[i];
}

// Band product bc = B x of a level's tridiagonal part (block-ordered vector).
template <typename T>
__global__ __launch_bounds__(kVecNT) void k_band_mv(LevelDev<T> lv, const T* x) {
  const int m = 2 * lv.n + 1;
  const int i = blockIdx.x * kVecNT + threadIdx.x;
  if (i >= m) return;
  T y = lv.bmain[i] * x[i];
  if (i > 0) y += lv.bsub[i] * x[i - 1];
  if (i + 1 < m) y += lv.bsup[i] * x[i + 1];
  lv.bc[i] = y;
}

template <typename T>
hipError_t launch_band_mv(const LevelDev<T>& lv, const T* x, hipStream_t s) {
  const int m = 2 * lv.n + 1;
  hipLaunchKernelGGL(k_band_mv<T>, (m + kVecNT - 1) / kVecNT, kVecNT, 0, s, lv, x);
  return hipGetLastError();
}
template hipError_t launch_band_mv<double>(const LevelDev<double>&, const double*, hipStream_t);
template hipError_t launch_band_mv<float>(const LevelDev<float>&, const float*, hipStream_t);

// BDF4 history combination of eq. (bdf4), one element per thread
__global__ __launch_bounds__(kVecNT) void k_bdf4_rhs(const double* u1, const double* u2,
                                                     const double* u3, const double* u4,
                                                     const double* src, double* b, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * kVecNT + threadIdx.x;
  if (i >= m) return;
  double v = 4.0 * u1[i] - 3.0 * u2[i] + (4.0 / 3.0) * u3[i] - 0.25 * u4[i];
  if (src) v += src[i];
  b[i] = v;
}

template <typename TZ>
__global__ __launch_bounds__(kVecNT) void k_cg_dir(const SolveState* st, double* p, const TZ* z,
                                                   int64_t m, int first) {
  if (st->done) return;
  const int64_t i = (int64_t)blockIdx.x * kVecNT + threadIdx.x;
  if (i >= m) return;
  p[i] = first ? (double)z[i] : (double)z[i] + st->beta * p[i];
}
template <typename TZ>
__global__ __launch_bounds__(kVecNT) void k_cg_dir_b(const CgArgs* __restrict__ args) {
  const CgArgs* g = args + blockIdx.y;
  if (gate_skip(g->st, g->gate)) return;
  const int64_t i = (int64_t)blockIdx.x * kVecNT + threadIdx.x;
  if (i >= g->m) return;
  const TZ* z = static_cast<const TZ*>(g->z);
  const SolveState* st = g->st;
  g->p[i] = st->cg_first ? (double)z[i] : (double)z[i] + st->beta * g->p[i];
}

// ---------------------------------------------------------------------------
// Near field of the split residual.  A workgroup owns kNearTS consecutive
// collocation positions s (units of h/2: nodes at even s, midpoints at odd
// s) and stages x at s - M .. s + kNearTS - 1 + M, read from the block
// order, in LDS; each output sums W(k) (x_{s+k} - x_s) over 0 < |k| <= M in
// (k, -k) pairs in a fixed order and adds R_s x_s.  Only the first and last
// workgroups hold positions whose stencil leaves 1..2N-1; they test every
// column (out-of-range columns are not in the matrix).
// ---------------------------------------------------------------------------
constexpr int kNearTS = 1024;
constexpr int kNearNT = 256;

__device__ __forceinline__ int64_t near_block(int64_t s, int64_t n) {
  // block-order index of position s: node s = 2(i+1) -> i; midpoint s = 2k+1 -> n + k
  return (s & 1) ? n + (s >> 1) : (s >> 1) - 1;
}

__global__ __launch_bounds__(kNearNT) void k_near(const double* x, double* y, int64_t N,
                                                 const double* w, const double* rl,
                                                 const double* rr, double rin_n, double rin_m) {
  constexpr int M = kNearM;
  __shared__ double zs[kNearTS + 2 * M];
  __shared__ double ws[2 * (2 * M + 1)];
  const int64_t last = 2 * N - 1, n = N - 1;
  const int64_t s0 = 1 + (int64_t)blockIdx.x * kNearTS;
  // workgroups with a position within M of either end test every column
  const bool edge = s0 <= M || s0 + kNearTS - 1 > last - M;
  for (int i = threadIdx.x; i < kNearTS + 2 * M; i += kNearNT) {
    const int64_t s = s0 - M + i;
    zs[i] = (s >= 1 && s <= last) ? x[near_block(s, n)] : 0.0;
  }
  for (int i = threadIdx.x; i < 2 * (2 * M + 1); i += kNearNT) ws[i] = w[i];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kNearTS / kNearNT; ++e) {
    const int t = threadIdx.x + e * kNearNT;
    const int64_t s = s0 + t;
    if (s > last) break;
    const double* W = ws + ((s & 1) ? (2 * M + 1) : 0) + M;
    const int c = t + M;
    const double zc = zs[c];
    double acc = 0.0;
    double R = (s & 1) ? rin_m : rin_n;
    if (!edge) {
#pragma unroll 8
      for (int k = 1; k <= M; ++k) acc += W[k] * (zs[c + k] - zc) + W[-k] * (zs[c - k] - zc);
    } else {
      for (int k = 1; k <= M; ++k) {
        if (s + k <= last) acc += W[k] * (zs[c + k] - zc);
        if (s - k >= 1) acc += W[-k] * (zs[c - k] - zc);
      }
      if (s <= M) R = rl[s - 1];
      else if (s > last - M) R = rr[s - (last - M + 1)];
    }
    y[near_block(s, n)] = acc + R * zc;
  }
}

hipError_t launch_near(const double* x, double* y, int64_t N, const double* w, const double* rl,
                       const double* rr, double rin_n, double rin_m, hipStream_t s) {
  const int64_t m = 2 * N - 1;
  const int64_t grid = (m + kNearTS - 1) / kNearTS;
  // the edge test of the kernel assumes a tile longer than the near reach
  static_assert(kNearTS > kNearM, "near tile");
  if (N <= kNearM || grid > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_near, dim3((unsigned)grid), dim3(kNearNT), 0, s, x, y, N, w, rl, rr, rin_n,
                     rin_m);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_tail_matvec(int colmode, int epimode, const LevelDev<T>& lv, const ColIn<T>& in,
                              const EpiOut<T>& out, const Twiddles<T>& tw, double* part,
                              hipStream_t s) {
  if (lv.logL > kTailLog) return hipErrorInvalidValue;
  const size_t lds = tail_lds_bytes(sizeof(T));
  if (colmode == COL_MV && epimode == EPI_MV)
    return launch_lds(k_tail_matvec<T, COL_MV, EPI_MV>, 1, kNTT, lds, s, lv, in, out, tw, part);
  if (colmode == COL_MV && epimode == EPI_OUTER)
    return launch_lds(k_tail_matvec<T, COL_MV, EPI_OUTER>, 1, kNTT, lds, s, lv, in, out, tw, part);
  if (colmode == COL_OUTER_UPDATE && epimode == EPI_OUTER)
    return launch_lds(k_tail_matvec<T, COL_OUTER_UPDATE, EPI_OUTER>, 1, kNTT, lds, s, lv, in, out,
                      tw, part);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_tail_vcycle(const LevelDev<T>* levels_dev, int first, int last, const T* rf,
                              int m1, int m2, T wpre, T wpost, const CoarseLU& lu,
                              const Twiddles<T>& tw, int maxL, int variant, hipStream_t s) {
  if (maxL > (1 << kTailLog) || lu.m > 4 * (1 << kTailLog) || first < 0 ||
      last - first + 1 > kTailMaxLev || last < first)
    return hipErrorInvalidValue;
  const size_t lds = tail_lds_bytes(sizeof(T));
  switch (variant) {
    case 0: return launch_lds(k_tail_vcycle<T, false, false>, 1, kNTT, lds, s, levels_dev, first,
                              last, rf, m1, m2, wpre, wpost, lu, tw);
    case TAIL_SYM: return launch_lds(k_tail_vcycle<T, false, true>, 1, kNTT, lds, s, levels_dev,
                                     first, last, rf, m1, m2, wpre, wpost, lu, tw);
    case TAIL_BAND: return launch_lds(k_tail_vcycle<T, true, false>, 1, kNTT, lds, s, levels_dev,
                                      first, last, rf, m1, m2, wpre, wpost, lu, tw);
    case TAIL_BAND | TAIL_SYM:
      return launch_lds(k_tail_vcycle<T, true, true>, 1, kNTT, lds, s, levels_dev, first, last,
                        rf, m1, m2, wpre, wpost, lu, tw);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_tail_program(const LevelDev<T>* levels_dev, int first, int last, const T* rf,
                               const TailOp* ops, int nops, T wpre, T wpost, const CoarseLU& lu,
                               const Twiddles<T>& tw, int maxL, int variant, hipStream_t s) {
  if (maxL > (1 << kTailLog) || lu.m > 4 * (1 << kTailLog) || first < 0 ||
      last - first + 1 > kTailMaxLev || last < first)
    return hipErrorInvalidValue;
  const size_t lds = tail_lds_bytes(sizeof(T));
  switch (variant) {
    case 0: return launch_lds(k_tail_program<T, false, false>, 1, kNTT, lds, s, levels_dev, first,
                              last, rf, ops, nops, wpre, wpost, lu, tw);
    case TAIL_SYM: return launch_lds(k_tail_program<T, false, true>, 1, kNTT, lds, s, levels_dev,
                                     first, last, rf, ops, nops, wpre, wpost, lu, tw);
    case TAIL_BAND: return launch_lds(k_tail_program<T, true, false>, 1, kNTT, lds, s, levels_dev,
                                      first, last, rf, ops, nops, wpre, wpost, lu, tw);
    case TAIL_BAND | TAIL_SYM:
      return launch_lds(k_tail_program<T, true, true>, 1, kNTT, lds, s, levels_dev, first, last,
                        rf, ops, nops, wpre, wpost, lu, tw);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tail_fft_setup(const LevelDev<double>& lv, const double* gx, const double* gy,
                                 cplx<double>* out, const Twiddles<double>& tw, hipStream_t s) {
  if (lv.logL > kTailLog) return hipErrorInvalidValue;
  const size_t lds = tail_lds_bytes(sizeof(double));
  return launch_lds(k_tail_fft_setup, 1, kNTT, lds, s, lv, gx, gy, out, tw);
}

hipError_t launch_combine(int logL, int logL1, int logL2, const cplx<double>* z1,
                          const cplx<double>* z2, int sym, double* g1, double* g2, float* g1f,
                          float* g2f, hipStream_t s) {
  const int64_t L = int64_t(1) << logL;
  const int grid = (int)((L + 255) / 256);
  hipLaunchKernelGGL(k_combine, grid, 256, 0, s, logL, logL1, logL2, z1, z2, sym, g1, g2, g1f, g2f);
  return hipGetLastError();
}

hipError_t launch_finish(SolveState* st, const double* part, int npart, double tol, int max_iter,
                         double* hist, hipStream_t s, int verify, SolveState* host) {
  static_assert(sizeof(SolveState) % 4 == 0 && sizeof(SolveState) / 4 <= 256, "state words");
  hipLaunchKernelGGL(k_finish, 1, 256, 0, s, st, part, npart, tol, max_iter, hist, verify, host);
  return hipGetLastError();
}

hipError_t launch_copy_d2f(const double* a, float* b, int64_t m, hipStream_t s) {
  const int grid = (int)((m + 255) / 256);
  hipLaunchKernelGGL(k_copy_d2f, grid, 256, 0, s, a, b, m);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_vdot(const double* a, const TZ* z, const double* c, int64_t m, double* part,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_vdot<TZ>, vec_blocks(m), kVecNT, 0, s, a, z, c, m, vec_chunk(m), part);
  return hipGetLastError();
}

hipError_t launch_cg_scalar(SolveState* st, const double* part, int nb, int stage, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_scalar, 1, kVecNT, 0, s, st, part, nb, stage);
  return hipGetLastError();
}

hipError_t launch_cg_update(const SolveState* st, double* x, const double* p, double* r,
                            double* r_old, const double* q, float* r32, int64_t m, double* npart,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update, vec_blocks(m), kVecNT, 0, s, st, x, p, r, r_old, q, r32, m,
                     vec_chunk(m), npart);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_cg_dir(const SolveState* st, double* p, const TZ* z, int64_t m, int first,
                         hipStream_t s) {
  const int grid = (int)((m + kVecNT - 1) / kVecNT);
  hipLaunchKernelGGL(k_cg_dir<TZ>, grid, kVecNT, 0, s, st, p, z, m, first);
  return hipGetLastError();
}

hipError_t launch_gm_start(const SolveState* st, const double* r, double* v0, double* g, int64_t m,
                           double* vin64, float* vin32, hipStream_t s) {
  const int grid = (int)((m + kVecNT - 1) / kVecNT);
  hipLaunchKernelGGL(k_gm_start, grid, kVecNT, 0, s, st, r, v0, g, m, vin64, vin32);
  return hipGetLastError();
}

hipError_t launch_gm_dot(const double* V, int cnt, const double* w, int64_t m, double* part,
                         hipStream_t s) {
  const dim3 grid(vec_blocks(m), (cnt + kGmGroup - 1) / kGmGroup);
  hipLaunchKernelGGL(k_gm_dot, grid, kVecNT, 0, s, V, cnt, w, m, vec_chunk(m), part);
  return hipGetLastError();
}

hipError_t launch_gm_reduce(const SolveState* st, const double* part, int nb, int cnt,
                            double* hcur, double* hcol, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_reduce, 1, kVecNT, 0, s, st, part, nb, cnt, hcur, hcol, accumulate);
  return hipGetLastError();
}

hipError_t launch_gm_axpy(const SolveState* st, double* w, const double* V, const double* hcur,
                          int cnt, int64_t m, double* npart, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_axpy, vec_blocks(m), kVecNT, 0, s, st, w, V, hcur, cnt, m, vec_chunk(m),
                     npart);
  return hipGetLastError();
}

hipError_t launch_gm_givens(SolveState* st, double* H, int j, double* cs, double* sn, double* g,
                            double* hn, const double* npart, int nb, double tol, int max_iter,
                            int restart, double* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_givens, 1, kVecNT, 0, s, st, H, j, cs, sn, g, hn, npart, nb, tol,
                     max_iter, restart, hist);
  return hipGetLastError();
}

hipError_t launch_gm_scale(const SolveState* st, double* w, const double* hn, int64_t m,
                           double* vin64, float* vin32, hipStream_t s) {
  const int grid = (int)((m + kVecNT - 1) / kVecNT);
  hipLaunchKernelGGL(k_gm_scale, grid, kVecNT, 0, s, st, w, hn, m, vin64, vin32);
  return hipGetLastError();
}

hipError_t launch_gm_update(const SolveState* st, const double* H, const double* g, int k,
                            double* y, double* x, const double* Z, int64_t m, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_solve, 1, 64, 0, s, st, H, g, k, y);
  const int grid = (int)((m + kVecNT - 1) / kVecNT);
  hipLaunchKernelGGL(k_gm_xupdate, grid, kVecNT, 0, s, st, x, Z, y, k, m);
  return hipGetLastError();
}

hipError_t launch_gm_check(SolveState* st, const double* npart, int nb, double tol, int max_iter,
                           double* hist, hipStream_t s, int stall) {
  hipLaunchKernelGGL(k_gm_check, 1, kVecNT, 0, s, st, npart, nb, tol, max_iter, hist, stall);
  return hipGetLastError();
}

hipError_t launch_copy_f2d(const float* a, double* b, int64_t m, hipStream_t s) {
  const int grid = (int)((m + 255) / 256);
  hipLaunchKernelGGL(k_copy_f2d, grid, 256, 0, s, a, b, m);
  return hipGetLastError();
}

hipError_t launch_bdf4_rhs(const double* u1, const double* u2, const double* u3,
                           const double* u4, const double* src, double* b, int64_t m,
                           hipStream_t s) {
  const int grid = (int)((m + kVecNT - 1) / kVecNT);
  hipLaunchKernelGGL(k_bdf4_rhs, grid, kVecNT, 0, s, u1, u2, u3, u4, src, b, m);
  return hipGetLastError();
}

// ---- batched launchers ------------------------------------------------------
template <typename T>
hipError_t launch_tail_vcycle_batch(const TailArgs<T>* args, int count, int variant,
                                    const Twiddles<T>& tw, hipStream_t s) {
  if (count < 1) return hipErrorInvalidValue;
  const size_t lds = tail_lds_bytes(sizeof(T));
  switch (variant) {
    case 0: return launch_lds(k_tail_vcycle_b<T, false, false>, count, kNTT, lds, s, args, tw);
    case TAIL_SYM: return launch_lds(k_tail_vcycle_b<T, false, true>, count, kNTT, lds, s, args, tw);
    case TAIL_BAND: return launch_lds(k_tail_vcycle_b<T, true, false>, count, kNTT, lds, s, args, tw);
    case TAIL_BAND | TAIL_SYM:
      return launch_lds(k_tail_vcycle_b<T, true, true>, count, kNTT, lds, s, args, tw);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// The folded V-cycle below the four-step levels (its matrix formed at setup
// from the unit vectors) as one product over many workgroups: every block
// restricts the fine residual into LDS (FP64), then each wavefront takes
// rows, lanes striding the row (coalesced), four partial sums per lane in a
// fixed order and a butterfly over the wavefront.
// ---------------------------------------------------------------------------
constexpr int kFoldNT = 512;
constexpr int kFoldRows = 8;  // one row per wavefront

template <typename T, typename MT>
__device__ __forceinline__ void fold_gemv_body(const T* __restrict__ rf, int m,
                                               const MT* __restrict__ M, T* __restrict__ u,
                                               int block) {
  extern __shared__ double fb[];  // m values of R rf
  for (int i = threadIdx.x; i < m; i += kFoldNT) fb[i] = (double)restrict_at(rf, i);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int rr = wave; rr < kFoldRows; rr += kFoldNT / 64) {
    const int row = block * kFoldRows + rr;
    if (row >= m) break;  // uniform in the wavefront
    const MT* a = M + (size_t)row * (size_t)m;
    // U loads in flight per lane (a row of 4095 in two batches of FP32 or
    // four of FP64), four partial sums
    constexpr int U = sizeof(MT) == 4 ? 32 : 16;
    double acc[4] = {0, 0, 0, 0};
    int j = lane;
    for (; j + 64 * (U - 1) < m; j += 64 * U) {
      MT av[U];
#pragma unroll
      for (int k = 0; k < U; ++k) av[k] = a[j + 64 * k];
#pragma unroll
      for (int k = 0; k < U; ++k) acc[k & 3] += (double)av[k] * fb[j + 64 * k];
    }
    {
      // the rest (fewer than U per lane): clamped loads, masked terms
      MT av[U];
#pragma unroll
      for (int k = 0; k < U; ++k) av[k] = a[min(j + 64 * k, m - 1)];
#pragma unroll
      for (int k = 0; k < U; ++k)
        if (j + 64 * k < m) acc[k & 3] += (double)av[k] * fb[j + 64 * k];
    }
    double v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) u[row] = (T)v;
  }
}

template <typename T, typename MT>
__global__ __launch_bounds__(kFoldNT) void k_fold_gemv(const T* rf, int m, const MT* M, T* u) {
  fold_gemv_body<T, MT>(rf, m, M, u, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kFoldNT) void k_fold_gemv_b(const FoldArgs<T>* __restrict__ args) {
  const FoldArgs<T>* a = args + blockIdx.y;
  if (gate_skip(a->st, a->gate)) return;
  if ((int)blockIdx.x * kFoldRows >= a->m) return;
  fold_gemv_body<T, T>(a->rf, a->m, a->M, a->u, blockIdx.x);
}

template <typename T, typename MT>
hipError_t launch_fold_gemv(const T* rf, int m, const MT* M, T* u, hipStream_t s) {
  if (m < 1 || m > kFoldMax) return hipErrorInvalidValue;
  const int grid = (m + kFoldRows - 1) / kFoldRows;
  return launch_lds(k_fold_gemv<T, MT>, grid, kFoldNT, (size_t)m * sizeof(double), s, rf, m, M, u);
}

template <typename T>
hipError_t launch_fold_gemv_batch(const FoldArgs<T>* args, int count, int m, hipStream_t s) {
  if (count < 1 || m < 1 || m > kFoldMax) return hipErrorInvalidValue;
  const dim3 grid((m + kFoldRows - 1) / kFoldRows, count);
  return launch_lds(k_fold_gemv_b<T>, grid, kFoldNT, (size_t)m * sizeof(double), s, args);
}

// 32 x 32 tiles through LDS: reads along the source vectors, writes along
// the matrix rows.
__global__ __launch_bounds__(256) void k_gather_rows(double* M, const double* src, int64_t stride,
                                                     int m, int j0, int count) {
  __shared__ double tile[32][33];
  const int ib = blockIdx.x * 32, kb = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int k = kb + r, i = ib + tx;
    tile[r][tx] = (k < count && i < m) ? src[(int64_t)k * stride + i] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = ib + r, k = kb + tx;
    if (i < m && k < count) M[(int64_t)i * m + j0 + k] = tile[tx][r];
  }
}

hipError_t launch_gather_rows(double* M, const double* src, int64_t stride, int m, int j0,
                              int count, hipStream_t s) {
  if (m < 1 || count < 1 || j0 < 0 || j0 + count > m) return hipErrorInvalidValue;
  const dim3 grid((m + 31) / 32, (count + 31) / 32);
  hipLaunchKernelGGL(k_gather_rows, grid, 256, 0, s, M, src, stride, m, j0, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail_matvec_batch(int colmode, int epimode, const PassArgs<T>* args, int count,
                                    const Twiddles<T>& tw, hipStream_t s) {
  if (count < 1) return hipErrorInvalidValue;
  const size_t lds = tail_lds_bytes(sizeof(T));
  if (colmode == COL_MV && epimode == EPI_MV)
    return launch_lds(k_tail_matvec_b<T, COL_MV, EPI_MV>, count, kNTT, lds, s, args, tw);
  if (colmode == COL_MV && epimode == EPI_OUTER)
    return launch_lds(k_tail_matvec_b<T, COL_MV, EPI_OUTER>, count, kNTT, lds, s, args, tw);
  if (colmode == COL_OUTER_UPDATE && epimode == EPI_OUTER)
    return launch_lds(k_tail_matvec_b<T, COL_OUTER_UPDATE, EPI_OUTER>, count, kNTT, lds, s, args,
                      tw);
  return hipErrorInvalidValue;
}

template <typename TZ>
hipError_t launch_vdot_batch(const VdotArgs* args, int count, int64_t mmax, hipStream_t s) {
  if (count < 1 || count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vdot_b<TZ>, dim3(vec_blocks(mmax), count), kVecNT, 0, s, args);
  return hipGetLastError();
}
hipError_t launch_cg_scalar_batch(const CgArgs* args, int count, int stage, hipStream_t s) {
  if (count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_scalar_b, count, kVecNT, 0, s, args, stage);
  return hipGetLastError();
}
template <typename TZ>
hipError_t launch_cg_dir_batch(const CgArgs* args, int count, int64_t mmax, hipStream_t s) {
  if (count < 1 || count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_dir_b<TZ>, dim3((unsigned)((mmax + kVecNT - 1) / kVecNT), count), kVecNT,
                     0, s, args);
  return hipGetLastError();
}
hipError_t launch_cg_update_batch(const CgArgs* args, int count, int64_t mmax, hipStream_t s) {
  if (count < 1 || count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_update_b, dim3(vec_blocks(mmax), count), kVecNT, 0, s, args);
  return hipGetLastError();
}
hipError_t launch_finish_batch(const FinishArgs* args, int count, hipStream_t s) {
  if (count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finish_b, count, 256, 0, s, args);
  return hipGetLastError();
}
hipError_t launch_gm_check_batch(const FinishArgs* args, int count, hipStream_t s) {
  if (count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gm_check_b, count, kVecNT, 0, s, args);
  return hipGetLastError();
}
template hipError_t launch_vdot_batch<double>(const VdotArgs*, int, int64_t, hipStream_t);
template hipError_t launch_vdot_batch<float>(const VdotArgs*, int, int64_t, hipStream_t);
template hipError_t launch_cg_dir_batch<double>(const CgArgs*, int, int64_t, hipStream_t);
template hipError_t launch_cg_dir_batch<float>(const CgArgs*, int, int64_t, hipStream_t);

template hipError_t launch_vdot<double>(const double*, const double*, const double*, int64_t,
                                        double*, hipStream_t);
template hipError_t launch_vdot<float>(const double*, const float*, const double*, int64_t,
                                       double*, hipStream_t);
template hipError_t launch_cg_dir<double>(const SolveState*, double*, const double*, int64_t, int,
                                          hipStream_t);
template hipError_t launch_cg_dir<float>(const SolveState*, double*, const float*, int64_t, int,
                                         hipStream_t);
#define AMG_INSTANTIATE(T)                                                                      \
  template hipError_t launch_tail_matvec<T>(int, int, const LevelDev<T>&, const ColIn<T>&,     \
                                            const EpiOut<T>&, const Twiddles<T>&, double*,     \
                                            hipStream_t);                                      \
  template hipError_t launch_tail_vcycle<T>(const LevelDev<T>*, int, int, const T*, int, int,  \
                                            T, T, const CoarseLU&, const Twiddles<T>&, int,    \
                                            int, hipStream_t);                                 \
  template hipError_t launch_tail_program<T>(const LevelDev<T>*, int, int, const T*,           \
                                             const TailOp*, int, T, T, const CoarseLU&,        \
                                             const Twiddles<T>&, int, int, hipStream_t);
AMG_INSTANTIATE(double)
AMG_INSTANTIATE(float)
template hipError_t launch_fold_gemv<double, double>(const double*, int, const double*, double*,
                                                     hipStream_t);
template hipError_t launch_fold_gemv<float, float>(const float*, int, const float*, float*,
                                                   hipStream_t);
template hipError_t launch_fold_gemv_batch<double>(const FoldArgs<double>*, int, int, hipStream_t);
template hipError_t launch_fold_gemv_batch<float>(const FoldArgs<float>*, int, int, hipStream_t);
template hipError_t launch_tail_vcycle_batch<double>(const TailArgs<double>*, int, int,
                                                     const Twiddles<double>&, hipStream_t);
template hipError_t launch_tail_vcycle_batch<float>(const TailArgs<float>*, int, int,
                                                    const Twiddles<float>&, hipStream_t);
template hipError_t launch_tail_matvec_batch<double>(int, int, const PassArgs<double>*, int,
                                                     const Twiddles<double>&, hipStream_t);
template hipError_t launch_tail_matvec_batch<float>(int, int, const PassArgs<float>*, int,
                                                    const Twiddles<float>&, hipStream_t);

}  // namespace amg
