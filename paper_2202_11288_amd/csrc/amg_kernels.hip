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
#include <mutex>
#include <unordered_map>

#include "amg_device.hpp"
#include "fft_lds.hpp"

namespace amg {

template <typename T>
struct Cfg;
template <>
struct Cfg<double> {
  static constexpr int E4 = 16;  // elements per thread, four-step passes (4096 / WG)
  static constexpr int ET = 8;   // elements per thread, tail kernels (4096 / WG)
};
template <>
struct Cfg<float> {
  static constexpr int E4 = 32;  // 8192 / WG
  static constexpr int ET = 8;
};

__device__ __forceinline__ int ilog2(int x) { return 31 - __clz(x); }

template <typename T>
__device__ __forceinline__ cplx<T> tw4(const Twiddles<T>& tw, int logL, int e) {
  // e^{-2 pi i e / L}, e < L <= 2^23, from two table lookups
  const int idx = e << (kTw4Log - logL);
  return cmul(tw.hi[idx >> 12], tw.lo[idx & (kTw4Lo - 1)]);
}

// Prolongation 2 R^T at fine index m of a fine vector of length 2*mc + 1
// (mc = coarse length): odd m = 2i+1 -> e[i]; even m = 2i -> (e[i-1] + e[i])/2.
template <typename T>
__device__ __forceinline__ T prolong_at(const T* e, int mc, int m) {
  if (m & 1) return e[m >> 1];
  const int i = m >> 1;
  T s = 0;
  if (i >= 1) s += e[i - 1];
  if (i < mc) s += e[i];
  return T(0.5) * s;
}

// Restriction 1/4 [1 2 1] at coarse index i (Sec. 3.1).
template <typename T>
__device__ __forceinline__ T restrict_at(const T* r, int i) {
  return T(0.25) * (r[2 * i] + T(2) * r[2 * i + 1] + r[2 * i + 2]);
}

// Circulant first column of the embedding of T[i][j] = t_{j-i} (eq. (ccs3.4)):
// c_m = t_{-m} (m < n), c_m = t_{L-m} (m > L-n), 0 otherwise.
__device__ __forceinline__ double circ_col(const double* g, int n, int L, int m) {
  if (m < n) return g[n - 1 - m];
  if (m > L - n) return g[n - 1 + (L - m)];
  return 0.0;
}

// Column tiles: consecutive tiles go to the same XCD (blocks are dealt to the
// 8 XCDs round robin), so neighbouring row segments share an L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  return (G % 8 == 0) ? (b & 7) * (G >> 3) + (b >> 3) : b;
}

// ---------------------------------------------------------------------------
// Pass 1: forward column FFTs (length L2, stride L1) of a tile of T columns,
// four-step twiddle, with the level's vector formation fused in front.
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(kNT4) void k_col_fwd(LevelDev<T> lv, ColIn<T> in, cplx<T>* buf,
                                                  Twiddles<T> tw, T* part) {
  extern __shared__ unsigned char smem_raw[];
  const Lds<T> lds{reinterpret_cast<cplx<T>*>(smem_raw)};
  __shared__ T red[kNT4 / 64];
  const int n = lv.n;
  const int L = 1 << lv.logL;
  const int TC = lv.tcols, logTC = ilog2(TC);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c0 = tile * TC;
  const int cnt = TC << lv.logL2;
  T dot = 0;
  for (int idx = threadIdx.x; idx < cnt; idx += kNT4) {
    const int i = idx >> logTC, t = idx & (TC - 1);
    const int j = c0 + t + (i << lv.logL1);
    cplx<T> z = {T(0), T(0)};
    if constexpr (MODE == COL_SETUP) {
      z.x = (T)circ_col(in.gx, n, L, j);
      z.y = (T)circ_col(in.gy, n, L, j);
    } else if (j < n) {
      const int jw = n + 1 + j;
      T v, w;
      if constexpr (MODE == COL_MV) {
        v = in.x[j];
        w = in.x[jw];
      } else if constexpr (MODE == COL_PRE || MODE == COL_PRE_RESTRICT) {
        T bv, bw;
        if constexpr (MODE == COL_PRE_RESTRICT) {
          bv = restrict_at(in.x, j);
          bw = restrict_at(in.x, jw);
          lv.b[j] = bv;
          lv.b[jw] = bw;
        } else {
          bv = lv.b[j];
          bw = lv.b[jw];
        }
        v = in.omega * bv / lv.dv;
        w = in.omega * bw / lv.dw;
        lv.u[j] = v;
        lv.u[jw] = w;
      } else if constexpr (MODE == COL_PROLONG) {
        // coarse vector length = n (2 n_c + 1 = n)
        v = lv.u[j] + prolong_at(in.x, n, j);
        w = lv.u[jw] + prolong_at(in.x, n, jw);
        lv.u[j] = v;
        lv.u[jw] = w;
      } else {  // COL_OUTER_UPDATE (T = double)
        const double ev = in.e_is_float ? (double)((const float*)in.e)[j] : ((const double*)in.e)[j];
        const double ew = in.e_is_float ? (double)((const float*)in.e)[jw] : ((const double*)in.e)[jw];
        const double xv = in.xo[j] + ev, xw = in.xo[jw] + ew;
        in.xo[j] = xv;
        in.xo[jw] = xw;
        v = (T)xv;
        w = (T)xw;
      }
      z.x = v;
      z.y = w;
      dot += lv.q[j] * v + lv.zeta[j] * w;
    }
    lds[idx] = z;
  }
  if constexpr (MODE != COL_SETUP && MODE != COL_MV) {
    if (tile == 0 && threadIdx.x == 0) {  // the w_o entry
      if constexpr (MODE == COL_PRE) {
        lv.u[n] = in.omega * lv.b[n] / lv.o;
      } else if constexpr (MODE == COL_PRE_RESTRICT) {
        const T bo = restrict_at(in.x, n);
        lv.b[n] = bo;
        lv.u[n] = in.omega * bo / lv.o;
      } else if constexpr (MODE == COL_PROLONG) {
        lv.u[n] += prolong_at(in.x, n, n);
      } else if constexpr (MODE == COL_OUTER_UPDATE) {
        const double e = in.e_is_float ? (double)((const float*)in.e)[n] : ((const double*)in.e)[n];
        in.xo[n] += e;
      }
    }
  }
  if constexpr (MODE != COL_SETUP) {
    const T s = block_sum<T, kNT4>(dot, red);
    if (threadIdx.x == 0) part[tile] = s;
  } else {
    __syncthreads();
  }
  const FftGeom g{lv.logL2, logTC, 0, logTC, kTwLog, true};
  lds_fft<T, Cfg<T>::E4, kNT4, false>(lds, g, tw.base);
  for (int idx = threadIdx.x; idx < cnt; idx += kNT4) {
    const int k2 = idx >> logTC, t = idx & (TC - 1);
    const int j1 = c0 + t;
    buf[j1 + (k2 << lv.logL1)] = cmul(lds[idx], tw4(tw, lv.logL, j1 * k2));
  }
}

// ---------------------------------------------------------------------------
// Pass 2: for the row pair (k2, L2-k2) (or {0, L2/2}): forward row FFTs,
// spectral 2x2 product (bins f and -f live in the paired rows), inverse row
// FFTs, inverse four-step twiddle.  Block 0 also finishes the w_o row
// y_o = q.v + o w_o + zeta.w_bar from pass 1's partial sums.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void spec_pair(const LevelDev<T>& lv, Lds<T> lds, int la, int lb,
                                          int ga, int gb) {
  const cplx<T> za = lds[la], zb = lds[lb];
  cplx<T> ya, yb;
  if (lv.sym) {
    const T g1a = lv.g1[ga], g2a = lv.g2[ga], g1b = lv.g1[gb], g2b = lv.g2[gb];
    // G1 z + (i g2) conj(z')
    ya = {g1a * za.x + g2a * zb.y, g1a * za.y + g2a * zb.x};
    yb = {g1b * zb.x + g2b * za.y, g1b * zb.y + g2b * za.x};
  } else {
    const cplx<T>* G1 = reinterpret_cast<const cplx<T>*>(lv.g1);
    const cplx<T>* G2 = reinterpret_cast<const cplx<T>*>(lv.g2);
    ya = cmul(G1[ga], za) + cmul(G2[ga], conj(zb));
    yb = cmul(G1[gb], zb) + cmul(G2[gb], conj(za));
  }
  lds[la] = ya;
  if (la != lb) lds[lb] = yb;
}

template <typename T, bool SPECTRAL>
__global__ __launch_bounds__(kNT4) void k_row(LevelDev<T> lv, cplx<T>* buf, Twiddles<T> tw,
                                              const T* part, int npart, const T* xin) {
  extern __shared__ unsigned char smem_raw[];
  const Lds<T> lds{reinterpret_cast<cplx<T>*>(smem_raw)};
  const int L1 = 1 << lv.logL1, L2 = 1 << lv.logL2;
  const int item = blockIdx.x;
  const int ka = item == 0 ? 0 : item;
  const int kb = item == 0 ? L2 / 2 : L2 - item;
  const int ra = ka << lv.logL1, rb = kb << lv.logL1;
  for (int t = threadIdx.x; t < L1; t += kNT4) {
    lds[t] = buf[ra + t];
    lds[L1 + t] = buf[rb + t];
  }
  __syncthreads();
  const FftGeom g{lv.logL1, 1, lv.logL1, 0, kTwLog, false};
  lds_fft<T, Cfg<T>::E4, kNT4, false>(lds, g, tw.base);
  if constexpr (!SPECTRAL) {
    for (int t = threadIdx.x; t < L1; t += kNT4) {
      buf[ra + t] = lds[t];
      buf[rb + t] = lds[L1 + t];
    }
    return;
  } else {
    if (item != 0) {
      // (ka, k1) pairs with (kb, L1-1-k1)
      for (int t = threadIdx.x; t < L1; t += kNT4)
        spec_pair(lv, lds, t, L1 + (L1 - 1 - t), ra + t, rb + (L1 - 1 - t));
    } else {
      // row 0: k1 pairs with (L1-k1) mod L1; row L2/2: k1 pairs with L1-1-k1
      const int npair0 = L1 / 2 + 1;
      for (int t = threadIdx.x; t < npair0 + L1 / 2; t += kNT4) {
        if (t < npair0) {
          const int tb = (L1 - t) & (L1 - 1);
          spec_pair(lv, lds, t, tb, ra + t, ra + tb);
        } else {
          const int k1 = t - npair0;
          spec_pair(lv, lds, L1 + k1, L1 + (L1 - 1 - k1), rb + k1, rb + (L1 - 1 - k1));
        }
      }
    }
    __syncthreads();
    lds_fft<T, Cfg<T>::E4, kNT4, true>(lds, g, tw.base);
    for (int t = threadIdx.x; t < L1; t += kNT4) {
      buf[ra + t] = cmul(lds[t], conj(tw4(tw, lv.logL, t * ka)));
      buf[rb + t] = cmul(lds[L1 + t], conj(tw4(tw, lv.logL, t * kb)));
    }
    if (item == 0 && threadIdx.x == 0) {
      T s = 0;
      for (int i = 0; i < npart; ++i) s += part[i];
      const T wo = xin[lv.n];
      lv.scal[0] = s + lv.o * wo;
      // snapshot of the input's w_o: pass 3 may update u[n] in place (Jacobi)
      // while its other blocks still need the value the product used
      lv.scal[1] = wo;
    }
  }
}

// ---------------------------------------------------------------------------
// Pass 3: inverse column FFTs; keeps the first n outputs and applies the
// Cross terms and the residual / Jacobi / output epilogue.
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(kNT4) void k_col_inv(LevelDev<T> lv, EpiOut<T> out,
                                                  const cplx<T>* buf, Twiddles<T> tw,
                                                  double* part) {
  extern __shared__ unsigned char smem_raw[];
  const Lds<T> lds{reinterpret_cast<cplx<T>*>(smem_raw)};
  __shared__ double red[kNT4 / 64];
  const int n = lv.n;
  const int TC = lv.tcols, logTC = ilog2(TC);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c0 = tile * TC;
  const int cnt = TC << lv.logL2;
  for (int idx = threadIdx.x; idx < cnt; idx += kNT4) {
    const int i = idx >> logTC, t = idx & (TC - 1);
    lds[idx] = buf[c0 + t + (i << lv.logL1)];
  }
  __syncthreads();
  const FftGeom g{lv.logL2, logTC, 0, logTC, kTwLog, true};
  lds_fft<T, Cfg<T>::E4, kNT4, true>(lds, g, tw.base);
  const T wo = lv.scal[1];  // the matvec input's w_o (see k_row)
  double ss = 0.0;
  const int half = cnt >> 1;  // outputs j2 < L2/2 cover j < n
  for (int idx = threadIdx.x; idx < half; idx += kNT4) {
    const int i = idx >> logTC, t = idx & (TC - 1);
    const int j = c0 + t + (i << lv.logL1);
    if (j >= n) continue;
    const int jw = n + 1 + j;
    const cplx<T> y = lds[idx];
    const T yv = y.x + lv.p[j] * wo;
    const T yw = y.y + lv.xi[j] * wo;
    if constexpr (MODE == EPI_MV) {
      out.y[j] = yv;
      out.y[jw] = yw;
    } else if constexpr (MODE == EPI_RESID) {
      lv.r[j] = lv.b[j] - yv;
      lv.r[jw] = lv.b[jw] - yw;
    } else if constexpr (MODE == EPI_SMOOTH) {
      lv.u[j] += out.omega * (lv.b[j] - yv) / lv.dv;
      lv.u[jw] += out.omega * (lv.b[jw] - yw) / lv.dw;
    } else {  // EPI_OUTER
      const double rv = out.bo[j] - (double)yv, rw = out.bo[jw] - (double)yw;
      out.ro[j] = rv;
      out.ro[jw] = rw;
      if (out.r32) {
        out.r32[j] = (float)rv;
        out.r32[jw] = (float)rw;
      }
      ss += rv * rv + rw * rw;
    }
  }
  if (tile == 0 && threadIdx.x == 0) {
    const T yo = lv.scal[0];
    if constexpr (MODE == EPI_MV) {
      out.y[n] = yo;
    } else if constexpr (MODE == EPI_RESID) {
      lv.r[n] = lv.b[n] - yo;
    } else if constexpr (MODE == EPI_SMOOTH) {
      lv.u[n] += out.omega * (lv.b[n] - yo) / lv.o;
    } else {
      const double ro = out.bo[n] - (double)yo;
      out.ro[n] = ro;
      if (out.r32) out.r32[n] = (float)ro;
      ss += ro * ro;
    }
  }
  if constexpr (MODE == EPI_OUTER) {
    const double s = block_sum<double, kNT4>(ss, red);
    if (threadIdx.x == 0) part[tile] = s;
  }
}

// ---------------------------------------------------------------------------
// Tail levels: L <= 2^12, one workgroup of 512 threads, FFT and twiddles in LDS.
// ---------------------------------------------------------------------------
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

constexpr int kTailP = (1 << (kTailLog - 1)) / kNTT + 1;  // spectral pairs per thread (f <= L/2)

// Spectra of the pairs (f, L-f), f = threadIdx.x + k*kNTT, loaded into
// registers before the forward FFT so their latency overlaps it.
template <typename T>
struct TailSpec {
  cplx<T> a1[kTailP], a2[kTailP], b1[kTailP], b2[kTailP];  // G1[f], G2[f], G1[-f], G2[-f]
};

template <typename T>
__device__ __forceinline__ void tail_spec_load(const LevelDev<T>& lv, TailSpec<T>& sp) {
  const int L = 1 << lv.logL;
#pragma unroll
  for (int k = 0; k < kTailP; ++k) {
    const int f = threadIdx.x + k * kNTT;
    if (f <= L / 2) {
      const int fb = (L - f) & (L - 1);
      if (lv.sym) {
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
}

// z holds the packed input (zero-padded); leaves y_v + i y_w_bar (without the
// Cross terms) in z[0..n).
template <typename T>
__device__ void tail_fft_spectral(const LevelDev<T>& lv, const TailLds<T>& s, const TailSpec<T>& sp) {
  const int L = 1 << lv.logL;
  const FftGeom g{lv.logL, 0, 0, 0, kTailLog, false};
  lds_fft<T, Cfg<T>::ET, kNTT, false>(s.z, g, s.tw);
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
  lds_fft<T, Cfg<T>::ET, kNTT, true>(s.z, g, s.tw);
}

enum TailPro { TP_PRE_B = 0, TP_PRE_RESTRICT, TP_USE_U, TP_PROLONG };
enum TailEpi { TE_RESID = 0, TE_SMOOTH };
constexpr int kTailJ = (1 << (kTailLog - 1)) / kNTT;  // v/w slots per thread (n < L/2)

// One matvec step of a tail level: form u (prologue), y = A u, then the
// residual or Jacobi epilogue; b and u stay in registers between the two.
template <typename T>
__device__ __forceinline__ void tail_step(const LevelDev<T>& lv, int pro, int epi, const T* src,
                                          T wpro, T wepi, const TailLds<T>& s) {
  const int n = lv.n, L = 1 << lv.logL;
  TailSpec<T> sp;
  tail_spec_load(lv, sp);
  T bv[kTailJ], bw[kTailJ], uv[kTailJ], uw[kTailJ], pj[kTailJ], xj[kTailJ];
  T dot = 0;
#pragma unroll
  for (int k = 0; k < kTailJ; ++k) {
    const int j = threadIdx.x + k * kNTT;
    bv[k] = bw[k] = uv[k] = uw[k] = pj[k] = xj[k] = T(0);
    if (j < n) {
      pj[k] = lv.p[j];
      xj[k] = lv.xi[j];
    }
    if (j < n) {
      const int jw = n + 1 + j;
      if (pro == TP_PRE_RESTRICT) {
        bv[k] = restrict_at(src, j);
        bw[k] = restrict_at(src, jw);
        lv.b[j] = bv[k];
        lv.b[jw] = bw[k];
      } else {
        bv[k] = lv.b[j];
        bw[k] = lv.b[jw];
      }
      if (pro == TP_PRE_B || pro == TP_PRE_RESTRICT) {
        uv[k] = wpro * bv[k] / lv.dv;
        uw[k] = wpro * bw[k] / lv.dw;
        lv.u[j] = uv[k];
        lv.u[jw] = uw[k];
      } else if (pro == TP_PROLONG) {
        uv[k] = lv.u[j] + prolong_at(src, n, j);
        uw[k] = lv.u[jw] + prolong_at(src, n, jw);
        lv.u[j] = uv[k];
        lv.u[jw] = uw[k];
      } else {
        uv[k] = lv.u[j];
        uw[k] = lv.u[jw];
      }
      s.z[j] = {uv[k], uw[k]};
      dot += lv.q[j] * uv[k] + lv.zeta[j] * uw[k];
    }
  }
  for (int j = n + threadIdx.x; j < L; j += kNTT) s.z[j] = {T(0), T(0)};
  if (threadIdx.x == 0) {  // the w_o entry
    const T bo = (pro == TP_PRE_RESTRICT) ? restrict_at(src, n) : lv.b[n];
    if (pro == TP_PRE_RESTRICT) lv.b[n] = bo;
    T uo;
    if (pro == TP_PRE_B || pro == TP_PRE_RESTRICT) uo = wpro * bo / lv.o;
    else if (pro == TP_PROLONG) uo = lv.u[n] + prolong_at(src, n, n);
    else uo = lv.u[n];
    if (pro != TP_USE_U) lv.u[n] = uo;
    s.red[kNTT / 64] = uo;
    s.red[kNTT / 64 + 1] = bo;
  }
  const T qdot = block_sum<T, kNTT>(dot, s.red);  // also publishes z and the w_o slots
  const T uo = s.red[kNTT / 64], bo = s.red[kNTT / 64 + 1];
  tail_fft_spectral(lv, s, sp);
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
        lv.u[j] = uv[k] + wepi * (bv[k] - yv) / lv.dv;
        lv.u[jw] = uw[k] + wepi * (bw[k] - yw) / lv.dw;
      }
    }
  }
  if (threadIdx.x == 0) {
    const T yo = qdot + lv.o * uo;
    if (epi == TE_RESID) lv.r[n] = bo - yo;
    else lv.u[n] = uo + wepi * (bo - yo) / lv.o;
  }
  __syncthreads();  // global writes visible to the next step; z and red reusable
}

// Coarsest level: u = A_c^{-1} b with the inverse formed at setup from the
// LU factors (partial pivoting).  b is staged in LDS as FP64; thread i < m
// forms row i from the column-major inverse (loads coalesced across threads,
// all independent).
template <typename T>
__device__ void coarse_solve(const CoarseLU& lu, const T* b, T* u, double* bs) {
  const int m = lu.m;
  for (int i = threadIdx.x; i < m; i += kNTT) bs[i] = (double)b[i];
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += kNTT) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += lu.ainv[j * m + i] * bs[j];
    u[i] = (T)acc;
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kNTT) void k_tail_vcycle(const LevelDev<T>* levels, int first,
                                                      int last, const T* rf, int m1, int m2,
                                                      T wpre, T wpost, CoarseLU lu,
                                                      Twiddles<T> tw) {
  extern __shared__ unsigned char smem_raw[];
  const TailLds<T> s = tail_lds<T>(smem_raw, tw.base);
  // One loop over the V-cycle's matvec steps (a single inlined tail_step):
  // descend (level first..last-1, m1 sweeps each, residual on the last one),
  // the coarsest solve, then ascend (prolongation + m2 post-sweeps).
  const int nlev = last - first;
  const int ndesc = nlev * m1;
  const int nsteps = ndesc + 1 + nlev * m2;
  for (int step = 0; step < nsteps; ++step) {
    if (step == ndesc) {  // coarsest level: b = R r_fine, exact solve by LU
      const LevelDev<T> lc = levels[last];
      const T* src = (last == first) ? rf : levels[last - 1].r;
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
      const T* fine = (l == first) ? rf : levels[l - 1].r;
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
      src = levels[l + 1].u;
      wpro = wepi = wpost;
    }
    const LevelDev<T> lv = levels[l];
    tail_step(lv, pro, epi, src, wpro, wepi, s);
  }
}

// One tail-level matvec: y = A x (EPI_MV) or the outer residual with the
// refinement update fused in front (COL_OUTER_UPDATE + EPI_OUTER).
template <typename T, int CM, int EM>
__global__ __launch_bounds__(kNTT) void k_tail_matvec(LevelDev<T> lv, ColIn<T> in, EpiOut<T> out,
                                                      Twiddles<T> tw, double* part) {
  extern __shared__ unsigned char smem_raw[];
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
  tail_spec_load(lv, sp);
  const T yo = block_sum<T, kNTT>(dot, s.red) + lv.o * x[n];
  tail_fft_spectral(lv, s, sp);
  const T wo = x[n];
  double ss = 0.0;
  for (int j = threadIdx.x; j < n; j += kNTT) {
    const cplx<T> z = s.z[j];
    const T yv = z.x + lv.p[j] * wo, yw = z.y + lv.xi[j] * wo;
    if constexpr (EM == EPI_MV) {
      out.y[j] = yv;
      out.y[n + 1 + j] = yw;
    } else {
      const double rv = out.bo[j] - (double)yv, rw = out.bo[n + 1 + j] - (double)yw;
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
      const double ro = out.bo[n] - (double)yo;
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

// Setup: FFT (natural order) of c_x + i c_y for a tail level.
__global__ __launch_bounds__(kNTT) void k_tail_fft_setup(LevelDev<double> lv, const double* gx,
                                                         const double* gy, cplx<double>* out,
                                                         Twiddles<double> tw) {
  extern __shared__ unsigned char smem_raw[];
  const TailLds<double> s = tail_lds<double>(smem_raw, tw.base);
  const int n = lv.n, L = 1 << lv.logL;
  for (int j = threadIdx.x; j < L; j += kNTT) s.z[j] = {circ_col(gx, n, L, j), circ_col(gy, n, L, j)};
  __syncthreads();
  const FftGeom g{lv.logL, 0, 0, 0, kTailLog, false};
  lds_fft<double, Cfg<double>::ET, kNTT, false>(s.z, g, s.tw);
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
__global__ __launch_bounds__(256) void k_finish(SolveState* st, const double* part, int npart,
                                                double tol, int max_iter, double* hist) {
  __shared__ double red[256 / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < npart; i += 256) v += part[i];
  const double s = block_sum<double, 256>(v, red);
  if (threadIdx.x != 0) return;
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
    st->status = 0;
    st->done = 1;
  } else if (rel > 1e3 * st->best) {
    st->status = 2;
    st->done = 1;
  } else if (st->iter >= max_iter) {
    st->status = 1;
    st->done = 1;
  }
  if (rel < st->best) st->best = rel;
  if (!st->done) st->iter += 1;
}

__global__ void k_copy_d2f(const double* a, float* b, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {
// Raise a kernel's dynamic-LDS limit once to the largest size it is launched
// with (gfx950 has 160 KB of LDS per workgroup).
template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> done;
  const void* key = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> g(mu);
  auto it = done.find(key);
  if (it != done.end() && it->second >= bytes) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done[key] = bytes;
  return e;
}
}  // namespace

template <typename T>
hipError_t launch_col_fwd(int mode, const LevelDev<T>& lv, const ColIn<T>& in, cplx<T>* buf,
                          const Twiddles<T>& tw, T* part, hipStream_t s) {
  const int grid = col_blocks(lv.logL1, lv.tcols);
  const size_t lds = sizeof(cplx<T>) * (size_t)lds_slots(lv.tcols << lv.logL2);
  hipError_t e = hipSuccess;
  switch (mode) {
    case COL_MV: e = set_lds(k_col_fwd<T, COL_MV>, lds); break;
    case COL_PRE: e = set_lds(k_col_fwd<T, COL_PRE>, lds); break;
    case COL_PRE_RESTRICT: e = set_lds(k_col_fwd<T, COL_PRE_RESTRICT>, lds); break;
    case COL_PROLONG: e = set_lds(k_col_fwd<T, COL_PROLONG>, lds); break;
    case COL_OUTER_UPDATE: e = set_lds(k_col_fwd<T, COL_OUTER_UPDATE>, lds); break;
    case COL_SETUP: e = set_lds(k_col_fwd<T, COL_SETUP>, lds); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (mode) {
    case COL_MV: hipLaunchKernelGGL((k_col_fwd<T, COL_MV>), grid, kNT4, lds, s, lv, in, buf, tw, part); break;
    case COL_PRE: hipLaunchKernelGGL((k_col_fwd<T, COL_PRE>), grid, kNT4, lds, s, lv, in, buf, tw, part); break;
    case COL_PRE_RESTRICT: hipLaunchKernelGGL((k_col_fwd<T, COL_PRE_RESTRICT>), grid, kNT4, lds, s, lv, in, buf, tw, part); break;
    case COL_PROLONG: hipLaunchKernelGGL((k_col_fwd<T, COL_PROLONG>), grid, kNT4, lds, s, lv, in, buf, tw, part); break;
    case COL_OUTER_UPDATE: hipLaunchKernelGGL((k_col_fwd<T, COL_OUTER_UPDATE>), grid, kNT4, lds, s, lv, in, buf, tw, part); break;
    case COL_SETUP: hipLaunchKernelGGL((k_col_fwd<T, COL_SETUP>), grid, kNT4, lds, s, lv, in, buf, tw, part); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_row(int spectral, const LevelDev<T>& lv, cplx<T>* buf, const Twiddles<T>& tw,
                      const T* part, int npart, const T* xin, hipStream_t s) {
  const int grid = (1 << lv.logL2) / 2;
  const size_t lds = sizeof(cplx<T>) * (size_t)lds_slots(2 << lv.logL1);
  hipError_t e = spectral ? set_lds(k_row<T, true>, lds) : set_lds(k_row<T, false>, lds);
  if (e != hipSuccess) return e;
  if (spectral)
    hipLaunchKernelGGL((k_row<T, true>), grid, kNT4, lds, s, lv, buf, tw, part, npart, xin);
  else
    hipLaunchKernelGGL((k_row<T, false>), grid, kNT4, lds, s, lv, buf, tw, part, npart, xin);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_col_inv(int mode, const LevelDev<T>& lv, const EpiOut<T>& out,
                          const cplx<T>* buf, const Twiddles<T>& tw, double* part, hipStream_t s) {
  const int grid = col_blocks(lv.logL1, lv.tcols);
  const size_t lds = sizeof(cplx<T>) * (size_t)lds_slots(lv.tcols << lv.logL2);
  hipError_t e = hipSuccess;
  switch (mode) {
    case EPI_MV: e = set_lds(k_col_inv<T, EPI_MV>, lds); break;
    case EPI_RESID: e = set_lds(k_col_inv<T, EPI_RESID>, lds); break;
    case EPI_SMOOTH: e = set_lds(k_col_inv<T, EPI_SMOOTH>, lds); break;
    case EPI_OUTER: e = set_lds(k_col_inv<T, EPI_OUTER>, lds); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (mode) {
    case EPI_MV: hipLaunchKernelGGL((k_col_inv<T, EPI_MV>), grid, kNT4, lds, s, lv, out, buf, tw, part); break;
    case EPI_RESID: hipLaunchKernelGGL((k_col_inv<T, EPI_RESID>), grid, kNT4, lds, s, lv, out, buf, tw, part); break;
    case EPI_SMOOTH: hipLaunchKernelGGL((k_col_inv<T, EPI_SMOOTH>), grid, kNT4, lds, s, lv, out, buf, tw, part); break;
    case EPI_OUTER: hipLaunchKernelGGL((k_col_inv<T, EPI_OUTER>), grid, kNT4, lds, s, lv, out, buf, tw, part); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail_matvec(int colmode, int epimode, const LevelDev<T>& lv, const ColIn<T>& in,
                              const EpiOut<T>& out, const Twiddles<T>& tw, double* part,
                              hipStream_t s) {
  if (lv.logL > kTailLog) return hipErrorInvalidValue;
  const size_t lds = tail_lds_bytes(sizeof(T));
  hipError_t e;
  if (colmode == COL_MV && epimode == EPI_MV) {
    auto k = k_tail_matvec<T, COL_MV, EPI_MV>;
    if ((e = set_lds(k, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(k, 1, kNTT, lds, s, lv, in, out, tw, part);
  } else if (colmode == COL_MV && epimode == EPI_OUTER) {
    auto k = k_tail_matvec<T, COL_MV, EPI_OUTER>;
    if ((e = set_lds(k, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(k, 1, kNTT, lds, s, lv, in, out, tw, part);
  } else if (colmode == COL_OUTER_UPDATE && epimode == EPI_OUTER) {
    auto k = k_tail_matvec<T, COL_OUTER_UPDATE, EPI_OUTER>;
    if ((e = set_lds(k, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(k, 1, kNTT, lds, s, lv, in, out, tw, part);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail_vcycle(const LevelDev<T>* levels_dev, int first, int last, const T* rf,
                              int m1, int m2, T wpre, T wpost, const CoarseLU& lu,
                              const Twiddles<T>& tw, int maxL, hipStream_t s) {
  if (maxL > (1 << kTailLog) || lu.m > 4 * (1 << kTailLog)) return hipErrorInvalidValue;
  const size_t lds = tail_lds_bytes(sizeof(T));
  auto k = k_tail_vcycle<T>;
  hipError_t e = set_lds(k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, 1, kNTT, lds, s, levels_dev, first, last, rf, m1, m2, wpre, wpost, lu, tw);
  return hipGetLastError();
}

hipError_t launch_tail_fft_setup(const LevelDev<double>& lv, const double* gx, const double* gy,
                                 cplx<double>* out, const Twiddles<double>& tw, hipStream_t s) {
  if (lv.logL > kTailLog) return hipErrorInvalidValue;
  const size_t lds = tail_lds_bytes(sizeof(double));
  hipError_t e = set_lds(k_tail_fft_setup, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tail_fft_setup, 1, kNTT, lds, s, lv, gx, gy, out, tw);
  return hipGetLastError();
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
                         double* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, 1, 256, 0, s, st, part, npart, tol, max_iter, hist);
  return hipGetLastError();
}

hipError_t launch_copy_d2f(const double* a, float* b, int64_t m, hipStream_t s) {
  const int grid = (int)((m + 255) / 256);
  hipLaunchKernelGGL(k_copy_d2f, grid, 256, 0, s, a, b, m);
  return hipGetLastError();
}

#define AMG_INSTANTIATE(T)                                                                      \
  template hipError_t launch_col_fwd<T>(int, const LevelDev<T>&, const ColIn<T>&, cplx<T>*,    \
                                        const Twiddles<T>&, T*, hipStream_t);                  \
  template hipError_t launch_row<T>(int, const LevelDev<T>&, cplx<T>*, const Twiddles<T>&,     \
                                    const T*, int, const T*, hipStream_t);                     \
  template hipError_t launch_col_inv<T>(int, const LevelDev<T>&, const EpiOut<T>&,             \
                                        const cplx<T>*, const Twiddles<T>&, double*,           \
                                        hipStream_t);                                          \
  template hipError_t launch_tail_matvec<T>(int, int, const LevelDev<T>&, const ColIn<T>&,     \
                                            const EpiOut<T>&, const Twiddles<T>&, double*,     \
                                            hipStream_t);                                      \
  template hipError_t launch_tail_vcycle<T>(const LevelDev<T>*, int, int, const T*, int, int,  \
                                            T, T, const CoarseLU&, const Twiddles<T>&, int,    \
                                            hipStream_t);
AMG_INSTANTIATE(double)
AMG_INSTANTIATE(float)

}  // namespace amg
