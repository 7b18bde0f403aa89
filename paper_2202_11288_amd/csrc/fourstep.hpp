// Four-step FFT passes of a large level's Toeplitz-plus-Cross matvec (Sec. 3.2,
// eq. (ccs3.4), eq. (split01)): L = L1 * L2 points, three HBM passes.
//   pass 1 (k_col_fwd): vector formation fused in front (smoothing start,
//            restriction, prolongation, refinement update), column FFTs of
//            length L2, four-step twiddle;
//   pass 2 (k_row):     for a row pair (k2, L2-k2): row FFTs, the 2x2 spectral
//            product (bins f and -f sit in the paired rows), inverse row FFTs,
//            inverse twiddle;
//   pass 3 (k_col_inv): inverse column FFTs, Cross terms, residual / Jacobi /
//            output epilogue.
// A workgroup holds at most kCap4 complex values (a tile of T columns or a
// row pair); the largest levels use column tiles of 2 kCap4 on twice the
// threads, so that each row segment of a real vector spans 32 bytes rather
// than 16 (the column passes there are bound by the number of distinct
// cache lines their loads touch), and L >= 2^22 also row pairs of 2 kCap4
// (rows of 4096 points, so that their columns come in tiles of 8 or 4).
// The per-thread element counts are template parameters (EPT column
// elements, KR row elements per row) so that every global load of a pass is
// issued in compile-time batches into registers, with clamped addresses and
// masked values, before any of them is used.  Internal header.
#pragma once

#include <type_traits>

#include "kernel_common.hpp"

namespace amg {

// Elements per thread of the LDS FFTs (a full tile or row pair).
constexpr int kE4 = kCap4 / kNT4;

// ---------------------------------------------------------------------------
// Pass 1.  Thread tid owns column j1 = c0 + (tid mod T) at rows i0 + e*di.
// ---------------------------------------------------------------------------
template <typename T, int MODE, int EPT, int NT = kNT4, int LOG2 = 0>
__device__ __forceinline__ void col_fwd_body(const LevelDev<T>& lv, const ColIn<T>& in,
                                             cplx<T>* buf, const Twiddles<T>& tw, T* part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Lds<T> lds{reinterpret_cast<cplx<T>*>(smem_raw)};
  __shared__ T red[NT / 64];
  const int n = lv.n;
  const int L = 1 << lv.logL;
  // column length and tile width: compile-time constants when LOG2 != 0
  const int logL2 = LOG2 ? LOG2 : lv.logL2;
  const int logTC = LOG2 ? ilog2(EPT * NT) - LOG2 : ilog2(lv.tcols);
  const int tcols = 1 << logTC;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int j1 = tile * tcols + (threadIdx.x & (tcols - 1));
  const int i0 = threadIdx.x >> logTC, di = NT >> logTC;
  // elements per load batch: FP32 issues the whole column's loads at once
  constexpr int CH = (EPT < 8 || sizeof(T) == 4) ? EPT : 8;
  const FftGeom g{logL2, logTC, 0, logTC, kTwLog, true};
  // partial tiles: every twiddle of the pass is fetched first, under the loads
  FftTw<T> ft;
  RunTw<T, EPT> rt;
  if constexpr (EPT < 16) {
    lds_fft_tw_prefetch(g, tw.base, ft);
    run_tw_load<T, EPT>(tw, lv.logL, j1 * i0, j1 * di, rt);
  }
  // the w_o entry (tile 0, thread 0): its operands are fetched first
  constexpr bool kWo = MODE != COL_SETUP && MODE != COL_MV;
  const bool wo_thread = kWo && tile == 0 && threadIdx.x == 0;
  T wo0 = 0, wo1 = 0, wo2 = 0;
  if (wo_thread) {
    if constexpr (MODE == COL_PRE) {
      wo0 = lv.b[n];
    } else if constexpr (MODE == COL_PRE_RESTRICT) {
      wo0 = in.x[2 * n];
      wo1 = in.x[2 * n + 1];
      wo2 = in.x[2 * n + 2];
    } else if constexpr (MODE == COL_PROLONG) {
      wo0 = lv.u[n];
      wo1 = prolong_at(in.x, n, n);
    } else if constexpr (MODE == COL_OUTER_UPDATE) {
      wo0 = (T)in.xo[n];
      wo1 = in.e_is_float ? (T)((const float*)in.e)[n] : (T)((const double*)in.e)[n];
    }
  }
  // the damped inverse diagonal of the two blocks, one division per thread
  const T wdv = in.omega / lv.dv, wdw = in.omega / lv.dw;
  T dot = 0;
  cplx<T> a[EPT];  // formed vector at rows i0 + e*di of column j1
#pragma unroll
  for (int e0 = 0; e0 < EPT; e0 += CH) {
    int jj[CH];
    bool ok[CH];
    T r0[CH], r1[CH], r2[CH], r3[CH], r4[CH], r5[CH], qq[CH], zz[CH];
    // (a) loads only
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int j = j1 + ((i0 + (e0 + c) * di) << lv.logL1);
      jj[c] = j;
      if constexpr (MODE == COL_SETUP) {
        ok[c] = true;
        r0[c] = (T)circ_col(in.gx, n, L, j);
        r1[c] = (T)circ_col(in.gy, n, L, j);
      } else {
        ok[c] = j < n;
        const int js = ok[c] ? j : 0, jw = n + 1 + js;
        qq[c] = lv.q[js];
        zz[c] = lv.zeta[js];
        if constexpr (MODE == COL_MV) {
          r0[c] = in.x[js];
          r1[c] = in.x[jw];
        } else if constexpr (MODE == COL_PRE) {
          r0[c] = lv.b[js];
          r1[c] = lv.b[jw];
        } else if constexpr (MODE == COL_PRE_RESTRICT) {
          r0[c] = in.x[2 * js];
          r1[c] = in.x[2 * js + 1];
          r2[c] = in.x[2 * js + 2];
          r3[c] = in.x[2 * jw];
          r4[c] = in.x[2 * jw + 1];
          r5[c] = in.x[2 * jw + 2];
        } else if constexpr (MODE == COL_PROLONG) {
          // coarse vector length = n (2 n_c + 1 = n)
          int lo, hi;
          bool ml, mh;
          r0[c] = lv.u[js];
          r1[c] = lv.u[jw];
          prolong_idx(js, n, lo, hi, ml, mh);
          r2[c] = in.x[lo];
          r3[c] = in.x[hi];
          r2[c] = ml ? r2[c] : T(0);
          r3[c] = mh ? r3[c] : T(0);
          prolong_idx(jw, n, lo, hi, ml, mh);
          r4[c] = in.x[lo];
          r5[c] = in.x[hi];
          r4[c] = ml ? r4[c] : T(0);
          r5[c] = mh ? r5[c] : T(0);
        } else {  // COL_OUTER_UPDATE (T = double)
          r0[c] = (T)in.xo[js];
          r1[c] = (T)in.xo[jw];
        }
      }
    }
    if constexpr (MODE == COL_OUTER_UPDATE) {
      if (in.e_is_float) {
        const float* ef = static_cast<const float*>(in.e);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int js = ok[c] ? jj[c] : 0;
          r2[c] = (T)ef[js];
          r3[c] = (T)ef[n + 1 + js];
        }
      } else {
        const double* ed = static_cast<const double*>(in.e);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int js = ok[c] ? jj[c] : 0;
          r2[c] = (T)ed[js];
          r3[c] = (T)ed[n + 1 + js];
        }
      }
    }
    // (b) vector formation, stores, Cross dot product, LDS
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int j = jj[c], jw = n + 1 + j;
      T v = r0[c], w = r1[c];
      if constexpr (MODE == COL_PRE || MODE == COL_PRE_RESTRICT) {
        if constexpr (MODE == COL_PRE_RESTRICT) {
          const T bv = T(0.25) * (r0[c] + T(2) * r1[c] + r2[c]);
          const T bw = T(0.25) * (r3[c] + T(2) * r4[c] + r5[c]);
          if (ok[c]) {
            lv.b[j] = bv;
            lv.b[jw] = bw;
          }
          v = bv;
          w = bw;
        }
        if (lv.dinv) {  // variable diagonal (weakly singular levels)
          const int js = ok[c] ? j : 0;
          v = in.omega * v * lv.dinv[js];
          w = in.omega * w * lv.dinv[n + 1 + js];
        } else {
          v = wdv * v;
          w = wdw * w;
        }
        if (ok[c]) {
          lv.u[j] = v;
          lv.u[jw] = w;
        }
      } else if constexpr (MODE == COL_PROLONG) {
        v = r0[c] + T(0.5) * (r2[c] + r3[c]);
        w = r1[c] + T(0.5) * (r4[c] + r5[c]);
        if (ok[c]) {
          lv.u[j] = v;
          lv.u[jw] = w;
        }
      } else if constexpr (MODE == COL_OUTER_UPDATE) {
        v = r0[c] + r2[c];
        w = r1[c] + r3[c];
        if (ok[c]) {
          in.xo[j] = v;
          in.xo[jw] = w;
        }
      }
      if (!ok[c]) v = w = T(0);
      if constexpr (MODE != COL_SETUP) dot += qq[c] * v + zz[c] * w;
      a[e0 + c] = cplx<T>{v, w};
    }
  }
  if (wo_thread) {
    if constexpr (MODE == COL_PRE) {
      lv.u[n] = in.omega * wo0 * (lv.dinv ? lv.dinv[n] : T(1) / lv.o);
    } else if constexpr (MODE == COL_PRE_RESTRICT) {
      const T bo = T(0.25) * (wo0 + T(2) * wo1 + wo2);
      lv.b[n] = bo;
      lv.u[n] = in.omega * bo * (lv.dinv ? lv.dinv[n] : T(1) / lv.o);
    } else if constexpr (MODE == COL_PROLONG) {
      lv.u[n] = wo0 + wo1;
    } else if constexpr (MODE == COL_OUTER_UPDATE) {
      in.xo[n] = (double)wo0 + (double)wo1;
    }
  }
  if constexpr (MODE != COL_SETUP) {
    const T s = block_sum<T, NT>(dot, red);
    if (threadIdx.x == 0) part[tile] = s;
  }
  if constexpr (EPT == 16) {
    // the thread's rows i0 + e*di are the positions j0 + e*L2/16 of its
    // last-pass butterfly (j0 = i0): first and last passes on registers
    fft_reg16<T, NT, false>(a, lds, g, threadIdx.x & (tcols - 1), i0, tw.base);
    twiddle_run_mul<T, EPT, false>(tw, lv.logL, j1 * i0, j1 * di, a);
  } else {
#pragma unroll
    for (int e = 0; e < EPT; ++e) lds[(int)threadIdx.x + e * NT] = a[e];
    __syncthreads();
    lds_fft_pf<T, NT, false>(lds, g, ft);
#pragma unroll
    for (int e = 0; e < EPT; ++e) a[e] = lds[(int)threadIdx.x + e * NT];
    twiddle_run_mul_pre<T, EPT, false>(rt, a);
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) stg(buf + j1 + ((i0 + e * di) << lv.logL1), a[e]);
}

template <typename T, int MODE, int EPT, int NT = kNT4, int LOG2 = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_col_fwd(LevelDev<T> lv, ColIn<T> in, cplx<T>* buf, Twiddles<T> tw, T* part) {
  col_fwd_body<T, MODE, EPT, NT, LOG2>(lv, in, buf, tw, part);
}
// The same pass for a batch of instances of one geometry: block (x, y) runs
// tile x of instance y with that instance's arguments (gated by its solve
// state), so each instance's arithmetic is that of its own launch.
template <typename T, int MODE, int EPT, int NT = kNT4, int LOG2 = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_col_fwd_b(const PassArgs<T>* __restrict__ args, Twiddles<T> tw) {
  const PassArgs<T>* a = args + blockIdx.y;
  if (gate_skip(a->st, a->gate)) return;
  const LevelDev<T> lv = a->lv;
  const ColIn<T> in = a->in;
  col_fwd_body<T, MODE, EPT, NT, LOG2>(lv, in, a->buf, tw, a->part);
}

// ---------------------------------------------------------------------------
// Pass 2.  Row pair (ka, kb) = (item, L2-item), or (0, L2/2) for item 0; the
// thread owns elements t = tid + e*kNT4 of both rows (KR of each; KR = 1 also
// covers L1 < kNT4).  Block 0 also finishes the w_o row
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

// The y_o row of the product, in block 0: pass 1's partial sums of
// q.v + zeta.w_bar (fetched by all threads at the start, reduced in a fixed
// order at the end) plus o w_o, and a snapshot of the input's w_o (pass 3 may
// update u[n] in place (Jacobi) while its other blocks still need the value
// the product used).
template <typename T, int NT = kNT4>
__device__ __forceinline__ T wo_partial(const T* part, int npart) {
  T v = 0;
  for (int i = threadIdx.x; i < npart; i += NT) v += part[i];
  return v;
}
template <typename T, int NT = kNT4>
__device__ __forceinline__ void finish_wo(const LevelDev<T>& lv, T v, T* red, const T* xin) {
  const T s = block_sum<T, NT>(v, red);
  if (threadIdx.x == 0) {
    const T wo = xin[lv.n];
    lv.scal[0] = s + lv.o * wo;
    lv.scal[1] = wo;
  }
}

// Row pair with L1 = 16 NT / 2 (each thread owns one radix-16 butterfly of
// the last pass: row s = tid / (L1/16), j0 = tid mod (L1/16), positions
// p = j0 + e L1/16).  Loads feed the first FFT pass directly; the spectral
// product exchanges the partner bins through LDS once; the last inverse pass
// feeds the twiddle and the stores.  NT = kNT4: rows of 2048 points;
// NT = 2 kNT4: rows of 4096 (the levels with L >= 2^22, whose columns then
// stay short enough for wide tiles of 8 or 4 columns).
template <typename T, bool SPECTRAL, bool SYM, int NT = kNT4>
__device__ __forceinline__ void row_pair_regs(const LevelDev<T>& lv, Lds<T> lds, cplx<T>* buf,
                                              const Twiddles<T>& tw, int item) {
  constexpr int Q = 16 * NT / 2 / 16;  // L1/16 butterflies per row
  // log2 L1: the geometry is a compile-time constant
  constexpr int kLog1 = NT == kNT4 ? 11 : 12;
  static_assert((1 << kLog1) == 16 * Q, "row length of the register row pass");
  constexpr int L1 = 1 << kLog1;
  const int L2 = 1 << lv.logL2;
  const int tid = threadIdx.x;
  const int s = tid / Q, j0 = tid % Q;
  const int k2 = item == 0 ? (s == 0 ? 0 : L2 / 2) : (s == 0 ? item : L2 - item);
  const int row = k2 << kLog1;
  cplx<T> a[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) a[e] = ldg(buf + row + j0 + e * Q);
  // SPD spectra at the thread's positions: FP32 fetches them under the
  // forward FFT; FP64 right after it (holding them across the FFT would spill)
  constexpr bool kEarly = sizeof(T) == 4;
  T g1[16], g2[16];
  auto load_spec = [&]() {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      g1[e] = lv.g1[row + j0 + e * Q];
      g2[e] = lv.g2[row + j0 + e * Q];
    }
  };
  if (kEarly && SPECTRAL && SYM) load_spec();
  const FftGeom g{kLog1, 1, kLog1, 0, kTwLog, false};
  fft_reg16<T, NT, false>(a, lds, g, s, j0, tw.base);
  if (!kEarly && SPECTRAL && SYM) load_spec();
  if constexpr (!SPECTRAL) {
#pragma unroll
    for (int e = 0; e < 16; ++e) stg(buf + row + j0 + e * Q, a[e]);
  } else {
    // bin f = k2 + L2 k1 pairs with -f: (kb, L1-1-k1) for item != 0; within
    // row 0 with (L1-k1) mod L1 and within row L2/2 with L1-1-k1 for item 0
    __syncthreads();  // last-pass LDS reads done before the exchange writes
#pragma unroll
    for (int e = 0; e < 16; ++e) lds[(s << kLog1) + j0 + e * Q] = a[e];
    __syncthreads();
    auto partner = [&](int e) {
      const int p = j0 + e * Q;
      int slot;
      if (item != 0) slot = s == 0 ? L1 + (L1 - 1 - p) : (L1 - 1 - p);
      else slot = s == 0 ? ((L1 - p) & (L1 - 1)) : L1 + (L1 - 1 - p);
      return lds[slot];
    };
    if constexpr (SYM) {
      // G1 real, G2 = i g2: Y = g1 z + i g2 conj(z')
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const cplx<T> zp = partner(e);
        a[e] = {g1[e] * a[e].x + g2[e] * zp.y, g1[e] * a[e].y + g2[e] * zp.x};
      }
    } else {
      const cplx<T>* G1 = reinterpret_cast<const cplx<T>*>(lv.g1);
      const cplx<T>* G2 = reinterpret_cast<const cplx<T>*>(lv.g2);
#pragma unroll
      for (int e0 = 0; e0 < 16; e0 += 4) {
        cplx<T> h1[4], h2[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          h1[c] = ldg(G1 + row + j0 + (e0 + c) * Q);
          h2[c] = ldg(G2 + row + j0 + (e0 + c) * Q);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
          a[e0 + c] = cmul(h1[c], a[e0 + c]) + cmul(h2[c], conj(partner(e0 + c)));
      }
    }
    __syncthreads();  // partner reads done before the inverse FFT writes LDS
    fft_reg16<T, NT, true>(a, lds, g, s, j0, tw.base);
    twiddle_run_mul<T, 16, true>(tw, lv.logL, j0 * k2, Q * k2, a);
#pragma unroll
    for (int e = 0; e < 16; ++e) stg(buf + row + j0 + e * Q, a[e]);
  }
}

template <typename T, bool SPECTRAL, bool SYM, int KR, int LOG1 = 0>
__device__ __forceinline__ void row_body(const LevelDev<T>& lv, cplx<T>* buf, const Twiddles<T>& tw,
                                         const T* part, int npart, const T* xin) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Lds<T> lds{reinterpret_cast<cplx<T>*>(smem_raw)};
  __shared__ T red[kNT4 / 64];
  // row length: a compile-time constant when LOG1 != 0
  const int logL1 = LOG1 ? LOG1 : lv.logL1;
  const int L1 = 1 << logL1, L2 = 1 << lv.logL2;
  const int item = blockIdx.x;
  const int tid = threadIdx.x;
  const T wpart = (SPECTRAL && item == 0) ? wo_partial(part, npart) : T(0);
  if constexpr (KR == 8) {
    row_pair_regs<T, SPECTRAL, SYM>(lv, lds, buf, tw, item);
    if (SPECTRAL && item == 0) finish_wo(lv, wpart, red, xin);
    return;
  }
  const int ka = item == 0 ? 0 : item;
  const int kb = item == 0 ? L2 / 2 : L2 - item;
  const int ra = ka << logL1, rb = kb << logL1;
  // every twiddle of the pass is fetched first, under the loads
  const FftGeom g{logL1, 1, logL1, 0, kTwLog, false};
  FftTw<T> ft;
  lds_fft_tw_prefetch(g, tw.base, ft);
  const bool act = KR > 1 || tid < L1;  // KR == 1: rows shorter than the workgroup
  const int t0 = act ? tid : 0;
  RunTw<T, KR> rta, rtb;
  if constexpr (SPECTRAL) {
    run_tw_load<T, KR>(tw, lv.logL, t0 * ka, kNT4 * ka, rta);
    run_tw_load<T, KR>(tw, lv.logL, t0 * kb, kNT4 * kb, rtb);
  }
  {
    cplx<T> za[KR], zb[KR];
#pragma unroll
    for (int e = 0; e < KR; ++e) {
      za[e] = ldg(buf + ra + t0 + e * kNT4);
      zb[e] = ldg(buf + rb + t0 + e * kNT4);
    }
    if (act) {
#pragma unroll
      for (int e = 0; e < KR; ++e) {
        lds[t0 + e * kNT4] = za[e];
        lds[L1 + t0 + e * kNT4] = zb[e];
      }
    }
  }
  // SPD spectra of this thread's pairs (t, L1-1-t), fetched under the FFT
  T g1a[KR], g2a[KR], g1b[KR], g2b[KR];
  const bool pre = SPECTRAL && SYM && item != 0;
  if (pre) {
#pragma unroll
    for (int e = 0; e < KR; ++e) {
      const int t = t0 + e * kNT4;
      g1a[e] = lv.g1[ra + t];
      g2a[e] = lv.g2[ra + t];
      g1b[e] = lv.g1[rb + (L1 - 1 - t)];
      g2b[e] = lv.g2[rb + (L1 - 1 - t)];
    }
  }
  __syncthreads();
  lds_fft_pf<T, kNT4, false>(lds, g, ft);
  if constexpr (!SPECTRAL) {
    if (act) {
#pragma unroll
      for (int e = 0; e < KR; ++e) {
        buf[ra + t0 + e * kNT4] = lds[t0 + e * kNT4];
        buf[rb + t0 + e * kNT4] = lds[L1 + t0 + e * kNT4];
      }
    }
    return;
  } else {
    if (pre) {
      if (act) {
#pragma unroll
        for (int e = 0; e < KR; ++e) {
          const int la = t0 + e * kNT4, lb = L1 + (L1 - 1 - la);
          const cplx<T> za = lds[la], zb = lds[lb];
          lds[la] = {g1a[e] * za.x + g2a[e] * zb.y, g1a[e] * za.y + g2a[e] * zb.x};
          lds[lb] = {g1b[e] * zb.x + g2b[e] * za.y, g1b[e] * zb.y + g2b[e] * za.x};
        }
      }
    } else if (!SYM && item != 0) {
      // general spectra: (ka, k1) pairs with (kb, L1-1-k1); batches of 4 pairs
      const cplx<T>* G1 = reinterpret_cast<const cplx<T>*>(lv.g1);
      const cplx<T>* G2 = reinterpret_cast<const cplx<T>*>(lv.g2);
      constexpr int CB = KR < 4 ? KR : 4;
#pragma unroll
      for (int e0 = 0; e0 < KR; e0 += CB) {
        cplx<T> a1[CB], a2[CB], b1[CB], b2[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          const int t = t0 + (e0 + c) * kNT4;
          a1[c] = ldg(G1 + ra + t);
          a2[c] = ldg(G2 + ra + t);
          b1[c] = ldg(G1 + rb + (L1 - 1 - t));
          b2[c] = ldg(G2 + rb + (L1 - 1 - t));
        }
        if (act) {
#pragma unroll
          for (int c = 0; c < CB; ++c) {
            const int la = t0 + (e0 + c) * kNT4, lb = L1 + (L1 - 1 - la);
            const cplx<T> za = lds[la], zb = lds[lb];
            lds[la] = cmul(a1[c], za) + cmul(a2[c], conj(zb));
            lds[lb] = cmul(b1[c], zb) + cmul(b2[c], conj(za));
          }
        }
      }
    } else {
      // row 0: k1 pairs with (L1-k1) mod L1; row L2/2: k1 pairs with L1-1-k1
      const int npair0 = L1 / 2 + 1;
      for (int t = tid; t < npair0 + L1 / 2; t += kNT4) {
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
    lds_fft_pf<T, kNT4, true>(lds, g, ft);
    cplx<T> ya[KR], yb[KR];
#pragma unroll
    for (int e = 0; e < KR; ++e) {
      ya[e] = lds[t0 + e * kNT4];
      yb[e] = lds[L1 + t0 + e * kNT4];
    }
    twiddle_run_mul_pre<T, KR, true>(rta, ya);
    twiddle_run_mul_pre<T, KR, true>(rtb, yb);
    if (act) {
#pragma unroll
      for (int e = 0; e < KR; ++e) {
        const int t = t0 + e * kNT4;
        stg(buf + ra + t, ya[e]);
        stg(buf + rb + t, yb[e]);
      }
    }
    if (item == 0) finish_wo(lv, wpart, red, xin);
  }
}

template <typename T, bool SPECTRAL, bool SYM, int KR, int LOG1 = 0>
__global__ __launch_bounds__(kNT4) __attribute__((amdgpu_waves_per_eu(2)))
void k_row(LevelDev<T> lv, cplx<T>* buf, Twiddles<T> tw, const T* part, int npart, const T* xin) {
  row_body<T, SPECTRAL, SYM, KR, LOG1>(lv, buf, tw, part, npart, xin);
}
template <typename T, bool SPECTRAL, bool SYM, int KR, int LOG1 = 0>
__global__ __launch_bounds__(kNT4) __attribute__((amdgpu_waves_per_eu(2)))
void k_row_b(const PassArgs<T>* __restrict__ args, Twiddles<T> tw) {
  const PassArgs<T>* a = args + blockIdx.y;
  if (gate_skip(a->st, a->gate)) return;
  const LevelDev<T> lv = a->lv;
  row_body<T, SPECTRAL, SYM, KR, LOG1>(lv, a->buf, tw, a->part, a->npart, a->xin);
}

// Pass 2 for rows of 4096 points: the register row pass on 2 kNT4 threads.
// The FP32 symmetric form fits two workgroups per CU (70 KB of LDS each).
template <typename T, bool SPECTRAL, bool SYM>
__device__ __forceinline__ void row_w_body(const LevelDev<T>& lv, cplx<T>* buf,
                                           const Twiddles<T>& tw, const T* part, int npart,
                                           const T* xin) {
  constexpr int NT = 2 * kNT4;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Lds<T> lds{reinterpret_cast<cplx<T>*>(smem_raw)};
  __shared__ T red[NT / 64];
  const int item = blockIdx.x;
  const T wpart = (SPECTRAL && item == 0) ? wo_partial<T, NT>(part, npart) : T(0);
  row_pair_regs<T, SPECTRAL, SYM, NT>(lv, lds, buf, tw, item);
  if (SPECTRAL && item == 0) finish_wo<T, NT>(lv, wpart, red, xin);
}

template <typename T, bool SPECTRAL, bool SYM>
__global__ __launch_bounds__(2 * kNT4)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && SYM ? 4 : 2)))
void k_row_w(LevelDev<T> lv, cplx<T>* buf, Twiddles<T> tw, const T* part, int npart, const T* xin) {
  row_w_body<T, SPECTRAL, SYM>(lv, buf, tw, part, npart, xin);
}
template <typename T, bool SPECTRAL, bool SYM>
__global__ __launch_bounds__(2 * kNT4)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && SYM ? 4 : 2)))
void k_row_w_b(const PassArgs<T>* __restrict__ args, Twiddles<T> tw) {
  const PassArgs<T>* a = args + blockIdx.y;
  if (gate_skip(a->st, a->gate)) return;
  const LevelDev<T> lv = a->lv;
  row_w_body<T, SPECTRAL, SYM>(lv, a->buf, tw, a->part, a->npart, a->xin);
}

// ---------------------------------------------------------------------------
// Pass 3.  Same ownership as pass 1; the outputs j < n are the rows
// j2 < L2/2, i.e. e < EPT/2 (EPT = 1: threads tid < kNT4/2).  The epilogue's
// operands are fetched before the FFT so their latency overlaps it.
// ---------------------------------------------------------------------------
template <typename T, int MODE, int EPT, int NT = kNT4, int LOG2 = 0>
__device__ __forceinline__ void col_inv_body(const LevelDev<T>& lv, const EpiOut<T>& out,
                                             const cplx<T>* buf, const Twiddles<T>& tw,
                                             double* part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const Lds<T> lds{reinterpret_cast<cplx<T>*>(smem_raw)};
  __shared__ double red[NT / 64];
  constexpr int KH = EPT > 1 ? EPT / 2 : 1;
  const int n = lv.n;
  // column length and tile width: compile-time constants when LOG2 != 0
  const int logL2 = LOG2 ? LOG2 : lv.logL2;
  const int logTC = LOG2 ? ilog2(EPT * NT) - LOG2 : ilog2(lv.tcols);
  const int tcols = 1 << logTC;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int j1 = tile * tcols + (threadIdx.x & (tcols - 1));
  const int i0 = threadIdx.x >> logTC, di = NT >> logTC;
  const FftGeom g{logL2, logTC, 0, logTC, kTwLog, true};
  FftTw<T> ft;  // partial tiles: the FFT's twiddles are fetched first
  if constexpr (EPT < 16) lds_fft_tw_prefetch(g, tw.base, ft);
  cplx<T> a[EPT];  // rows i0 + e*di of column j1
#pragma unroll
  for (int e = 0; e < EPT; ++e) a[e] = ldg(buf + j1 + ((i0 + e * di) << lv.logL1));
  // the w_o row (tile 0, thread 0): its operands are fetched first
  const bool wo_thread = tile == 0 && threadIdx.x == 0;
  T yo = 0, wb = 0, wu = 0;
  double wbo = 0.0;
  if (wo_thread) {
    yo = lv.scal[0];
    if constexpr (MODE == EPI_RESID || MODE == EPI_SMOOTH) wb = lv.b[n];
    if constexpr (MODE == EPI_SMOOTH) wu = lv.u[n];
    if constexpr (MODE == EPI_OUTER) wbo = out.bo[n] - (out.ynear ? out.ynear[n] : 0.0);
  }
  bool ok[KH];
  int jj[KH];
  T pp[KH], xx[KH], b0[KH], b1[KH], u0[KH], u1[KH];
  double o0[KH], o1[KH], q0[KH], q1[KH];
#pragma unroll
  for (int e = 0; e < KH; ++e) {
    const int j = j1 + ((i0 + e * di) << lv.logL1);
    ok[e] = (EPT > 1 || (int)threadIdx.x < NT / 2) && j < n;
    jj[e] = j;
    const int js = ok[e] ? j : 0, jw = n + 1 + js;
    pp[e] = lv.p[js];
    xx[e] = lv.xi[js];
    if constexpr (MODE == EPI_RESID || MODE == EPI_SMOOTH) {
      b0[e] = lv.b[js];
      b1[e] = lv.b[jw];
    }
    if constexpr (MODE == EPI_SMOOTH && (sizeof(T) == 4 || EPT < 16)) {
      u0[e] = lv.u[js];
      u1[e] = lv.u[jw];
    }
    if constexpr (MODE == EPI_OUTER) {
      o0[e] = out.bo[js];
      o1[e] = out.bo[jw];
      q0[e] = out.ynear ? out.ynear[js] : 0.0;
      q1[e] = out.ynear ? out.ynear[jw] : 0.0;
    }
  }
  if constexpr (EPT == 16) {
    fft_reg16<T, NT, true>(a, lds, g, threadIdx.x & (tcols - 1), i0, tw.base);
  } else {
#pragma unroll
    for (int e = 0; e < EPT; ++e) lds[(int)threadIdx.x + e * NT] = a[e];
    __syncthreads();
    lds_fft_pf<T, NT, true>(lds, g, ft);
#pragma unroll
    for (int e = 0; e < KH; ++e) a[e] = lds[(int)threadIdx.x + e * NT];
  }
  if constexpr (MODE == EPI_SMOOTH && sizeof(T) == 8 && EPT == 16) {
    // FP64 full tiles: the iterate is fetched after the FFT (register budget)
#pragma unroll
    for (int e = 0; e < KH; ++e) {
      const int js = ok[e] ? jj[e] : 0;
      u0[e] = lv.u[js];
      u1[e] = lv.u[n + 1 + js];
    }
  }
  const T wo = lv.scal[1];  // the matvec input's w_o (see k_row)
  const bool band = lv.bc != nullptr;  // weakly singular levels: + B x, variable diagonal
  const T wdv = out.omega / lv.dv, wdw = out.omega / lv.dw;  // Jacobi factors, constant diagonal
  double ss = 0.0;
#pragma unroll
  for (int e = 0; e < KH; ++e) {
    if (!ok[e]) continue;
    const int j = jj[e], jw = n + 1 + j;
    const cplx<T> y = a[e];
    T yv = y.x + pp[e] * wo;
    T yw = y.y + xx[e] * wo;
    if (band) {
      yv += lv.bc[j];
      yw += lv.bc[jw];
    }
    if constexpr (MODE == EPI_MV) {
      out.y[j] = yv;
      out.y[jw] = yw;
    } else if constexpr (MODE == EPI_RESID) {
      lv.r[j] = b0[e] - yv;
      lv.r[jw] = b1[e] - yw;
    } else if constexpr (MODE == EPI_SMOOTH) {
      if (band) {
        lv.u[j] = u0[e] + out.omega * (b0[e] - yv) * lv.dinv[j];
        lv.u[jw] = u1[e] + out.omega * (b1[e] - yw) * lv.dinv[jw];
      } else {
        lv.u[j] = u0[e] + wdv * (b0[e] - yv);
        lv.u[jw] = u1[e] + wdw * (b1[e] - yw);
      }
    } else {  // EPI_OUTER
      const double rv = o0[e] - ((double)yv + q0[e]), rw = o1[e] - ((double)yw + q1[e]);
      out.ro[j] = rv;
      out.ro[jw] = rw;
      if (out.r32) {
        out.r32[j] = (float)rv;
        out.r32[jw] = (float)rw;
      }
      ss += rv * rv + rw * rw;
    }
  }
  if (wo_thread) {
    if (band) yo += lv.bc[n];
    if constexpr (MODE == EPI_MV) {
      out.y[n] = yo;
    } else if constexpr (MODE == EPI_RESID) {
      lv.r[n] = wb - yo;
    } else if constexpr (MODE == EPI_SMOOTH) {
      lv.u[n] = wu + out.omega * (wb - yo) * (band ? lv.dinv[n] : T(1) / lv.o);
    } else {
      const double ro = wbo - (double)yo;
      out.ro[n] = ro;
      if (out.r32) out.r32[n] = (float)ro;
      ss += ro * ro;
    }
  }
  if constexpr (MODE == EPI_OUTER) {
    const double s = block_sum<double, NT>(ss, red);
    if (threadIdx.x == 0) part[tile] = s;
  }
}

template <typename T, int MODE, int EPT, int NT = kNT4, int LOG2 = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_col_inv(LevelDev<T> lv, EpiOut<T> out, const cplx<T>* buf, Twiddles<T> tw, double* part) {
  col_inv_body<T, MODE, EPT, NT, LOG2>(lv, out, buf, tw, part);
}
template <typename T, int MODE, int EPT, int NT = kNT4, int LOG2 = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2)))
void k_col_inv_b(const PassArgs<T>* __restrict__ args, Twiddles<T> tw) {
  const PassArgs<T>* a = args + blockIdx.y;
  if (gate_skip(a->st, a->gate)) return;
  const LevelDev<T> lv = a->lv;
  const EpiOut<T> out = a->out;
  col_inv_body<T, MODE, EPT, NT, LOG2>(lv, out, a->buf, tw, a->npart_out);
}

// ---------------------------------------------------------------------------
// Launchers: the level geometry picks the instance (EPT = T L2 / kNT4,
// KR = max(1, L1 / kNT4)); checked against the kernels' assumptions here.
// ---------------------------------------------------------------------------
// A column tile of cnt = tcols * L2 elements runs on kNT4 threads, cnt / kNT4
// each (reported as ept), up to kCap4; a wide tile of 2 kCap4 elements runs on
// 2 kNT4 threads with 16 each (reported as ept = 32).
inline bool col_geom_ok(int logL1, int logL2, int tcols, int* ept) {
  const int cnt = tcols << logL2;
  if (tcols < 1 || (tcols & (tcols - 1)) || tcols > kNT4 || (1 << logL1) % tcols) return false;
  if (cnt % kNT4 || cnt > kCapWide) return false;
  *ept = cnt / kNT4;
  return true;
}

// The compile-time geometry of a column pass, from the element count per
// thread (ept; 32 = a wide tile of 2 kNT4 threads with 16 each), the tile
// width and the column length: f(EPT, NT, LOG2) as integral constants.
template <int V>
using IC = std::integral_constant<int, V>;
template <typename F>
hipError_t col_pick(int ept, int tcols, int logL2, F&& f) {
  switch (ept) {
    case 1: return tcols == 4 ? f(IC<1>{}, IC<kNT4>{}, IC<6>{}) : f(IC<1>{}, IC<kNT4>{}, IC<0>{});
    case 2: return tcols == 4 ? f(IC<2>{}, IC<kNT4>{}, IC<7>{}) : f(IC<2>{}, IC<kNT4>{}, IC<0>{});
    case 4: return tcols == 4 ? f(IC<4>{}, IC<kNT4>{}, IC<8>{}) : f(IC<4>{}, IC<kNT4>{}, IC<0>{});
    case 8: return tcols == 4 ? f(IC<8>{}, IC<kNT4>{}, IC<9>{}) : f(IC<8>{}, IC<kNT4>{}, IC<0>{});
    case 16:
      if (logL2 == 10) return f(IC<16>{}, IC<kNT4>{}, IC<10>{});
      if (logL2 == 9) return f(IC<16>{}, IC<kNT4>{}, IC<9>{});
      return f(IC<16>{}, IC<kNT4>{}, IC<0>{});
    case 32:
      switch (logL2) {
        case 10: return f(IC<16>{}, IC<2 * kNT4>{}, IC<10>{});
        case 11: return f(IC<16>{}, IC<2 * kNT4>{}, IC<11>{});
        case 12: return f(IC<16>{}, IC<2 * kNT4>{}, IC<12>{});
        default: return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;
  }
}

// The row pass's compile-time geometry: f(KR, LOG1) (KR = 16: rows of 4096
// points, the wide register row pass).
template <typename F>
hipError_t row_pick(int kr, int logL1, F&& f) {
  switch (kr) {
    case 1:
      if (logL1 == 7) return f(IC<1>{}, IC<7>{});
      if (logL1 == 8) return f(IC<1>{}, IC<8>{});
      return f(IC<1>{}, IC<0>{});
    case 2: return f(IC<2>{}, IC<9>{});
    case 4: return f(IC<4>{}, IC<10>{});
    case 8: return f(IC<8>{}, IC<0>{});
    case 16: return f(IC<16>{}, IC<0>{});
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int MODE>
hipError_t col_fwd_ept(int ept, int grid, size_t lds, hipStream_t s, const LevelDev<T>& lv,
                       const ColIn<T>& in, cplx<T>* buf, const Twiddles<T>& tw, T* part) {
  return col_pick(ept, lv.tcols, lv.logL2, [&](auto E, auto NTc, auto G) {
    constexpr int NT = decltype(NTc)::value;
    return launch_lds(k_col_fwd<T, MODE, decltype(E)::value, NT, decltype(G)::value>, grid, NT,
                      lds, s, lv, in, buf, tw, part);
  });
}

template <typename T, int MODE>
hipError_t col_inv_ept(int ept, int grid, size_t lds, hipStream_t s, const LevelDev<T>& lv,
                       const EpiOut<T>& out, const cplx<T>* buf, const Twiddles<T>& tw,
                       double* part) {
  return col_pick(ept, lv.tcols, lv.logL2, [&](auto E, auto NTc, auto G) {
    constexpr int NT = decltype(NTc)::value;
    return launch_lds(k_col_inv<T, MODE, decltype(E)::value, NT, decltype(G)::value>, grid, NT,
                      lds, s, lv, out, buf, tw, part);
  });
}

template <typename T, bool SPECTRAL, bool SYM>
hipError_t row_kr(int kr, int grid, size_t lds, hipStream_t s, const LevelDev<T>& lv,
                  cplx<T>* buf, const Twiddles<T>& tw, const T* part, int npart, const T* xin) {
  return row_pick(kr, lv.logL1, [&](auto K, auto G) {
    constexpr int KR = decltype(K)::value;
    if constexpr (KR == 16)
      return launch_lds(k_row_w<T, SPECTRAL, SYM>, grid, 2 * kNT4, lds, s, lv, buf, tw, part,
                        npart, xin);
    else
      return launch_lds(k_row<T, SPECTRAL, SYM, KR, decltype(G)::value>, grid, kNT4, lds, s, lv,
                        buf, tw, part, npart, xin);
  });
}

// Modes built for FP32 (the V-cycle) and FP64 (everything).
template <typename T>
constexpr bool col_mode_built(int mode) {
  return sizeof(T) == 8 || mode == COL_MV || mode == COL_PRE || mode == COL_PRE_RESTRICT ||
         mode == COL_PROLONG;
}
template <typename T>
constexpr bool epi_mode_built(int mode) {
  return sizeof(T) == 8 || mode == EPI_MV || mode == EPI_RESID || mode == EPI_SMOOTH;
}

template <typename T>
hipError_t launch_col_fwd(int mode, const LevelDev<T>& lv, const ColIn<T>& in, cplx<T>* buf,
                               const Twiddles<T>& tw, T* part, hipStream_t s) {
  int ept;
  if (!col_geom_ok(lv.logL1, lv.logL2, lv.tcols, &ept) || !col_mode_built<T>(mode))
    return hipErrorInvalidValue;
  const int grid = col_blocks(lv.logL1, lv.tcols);
  const size_t lds = sizeof(cplx<T>) * (size_t)lds_slots(ept * kNT4);
  switch (mode) {
    case COL_MV: return col_fwd_ept<T, COL_MV>(ept, grid, lds, s, lv, in, buf, tw, part);
    case COL_PRE: return col_fwd_ept<T, COL_PRE>(ept, grid, lds, s, lv, in, buf, tw, part);
    case COL_PRE_RESTRICT:
      return col_fwd_ept<T, COL_PRE_RESTRICT>(ept, grid, lds, s, lv, in, buf, tw, part);
    case COL_PROLONG: return col_fwd_ept<T, COL_PROLONG>(ept, grid, lds, s, lv, in, buf, tw, part);
    default: break;
  }
  if constexpr (sizeof(T) == 8) {
    switch (mode) {
      case COL_OUTER_UPDATE:
        return col_fwd_ept<T, COL_OUTER_UPDATE>(ept, grid, lds, s, lv, in, buf, tw, part);
      case COL_SETUP: return col_fwd_ept<T, COL_SETUP>(ept, grid, lds, s, lv, in, buf, tw, part);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_row(int spectral, const LevelDev<T>& lv, cplx<T>* buf,
                           const Twiddles<T>& tw, const T* part, int npart, const T* xin,
                           hipStream_t s) {
  const int L1 = 1 << lv.logL1;
  if (2 * L1 > kCapWide || lv.logL2 < 1) return hipErrorInvalidValue;
  const int kr = L1 >= kNT4 ? L1 / kNT4 : 1;
  const int grid = (1 << lv.logL2) / 2;
  const size_t lds = sizeof(cplx<T>) * (size_t)lds_slots(2 * L1);
  if (spectral && lv.sym) return row_kr<T, true, true>(kr, grid, lds, s, lv, buf, tw, part, npart, xin);
  if (spectral) return row_kr<T, true, false>(kr, grid, lds, s, lv, buf, tw, part, npart, xin);
  if constexpr (sizeof(T) == 8)
    return row_kr<T, false, false>(kr, grid, lds, s, lv, buf, tw, part, npart, xin);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_col_inv(int mode, const LevelDev<T>& lv, const EpiOut<T>& out,
                               const cplx<T>* buf, const Twiddles<T>& tw, double* part,
                               hipStream_t s) {
  int ept;
  if (!col_geom_ok(lv.logL1, lv.logL2, lv.tcols, &ept) || !epi_mode_built<T>(mode))
    return hipErrorInvalidValue;
  const int grid = col_blocks(lv.logL1, lv.tcols);
  const size_t lds = sizeof(cplx<T>) * (size_t)lds_slots(ept * kNT4);
  switch (mode) {
    case EPI_MV: return col_inv_ept<T, EPI_MV>(ept, grid, lds, s, lv, out, buf, tw, part);
    case EPI_RESID: return col_inv_ept<T, EPI_RESID>(ept, grid, lds, s, lv, out, buf, tw, part);
    case EPI_SMOOTH: return col_inv_ept<T, EPI_SMOOTH>(ept, grid, lds, s, lv, out, buf, tw, part);
    default: break;
  }
  if constexpr (sizeof(T) == 8) {
    switch (mode) {
      case EPI_OUTER: return col_inv_ept<T, EPI_OUTER>(ept, grid, lds, s, lv, out, buf, tw, part);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Batched launches: `count` instances of one level geometry (the geometry of
// `geom`; each instance's own arguments in the device table `args`), block
// row y = instance y.  Same kernels bodies, same per-instance arithmetic.
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_col_fwd_batch(int mode, const LevelDev<T>& geom, const PassArgs<T>* args,
                                int count, const Twiddles<T>& tw, hipStream_t s) {
  int ept;
  if (count < 1 || count > 65535 || !col_geom_ok(geom.logL1, geom.logL2, geom.tcols, &ept) ||
      !col_mode_built<T>(mode))
    return hipErrorInvalidValue;
  const dim3 grid(col_blocks(geom.logL1, geom.tcols), count);
  const size_t lds = sizeof(cplx<T>) * (size_t)lds_slots(ept * kNT4);
  auto go = [&](auto M) {
    constexpr int MODE = decltype(M)::value;
    return col_pick(ept, geom.tcols, geom.logL2, [&](auto E, auto NTc, auto G) {
      constexpr int NT = decltype(NTc)::value;
      return launch_lds(k_col_fwd_b<T, MODE, decltype(E)::value, NT, decltype(G)::value>, grid,
                        NT, lds, s, args, tw);
    });
  };
  switch (mode) {
    case COL_MV: return go(IC<COL_MV>{});
    case COL_PRE: return go(IC<COL_PRE>{});
    case COL_PRE_RESTRICT: return go(IC<COL_PRE_RESTRICT>{});
    case COL_PROLONG: return go(IC<COL_PROLONG>{});
    default: break;
  }
  if constexpr (sizeof(T) == 8) {
    if (mode == COL_OUTER_UPDATE) return go(IC<COL_OUTER_UPDATE>{});
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_row_batch(const LevelDev<T>& geom, const PassArgs<T>* args, int count,
                            const Twiddles<T>& tw, hipStream_t s) {
  const int L1 = 1 << geom.logL1;
  if (count < 1 || count > 65535 || 2 * L1 > kCapWide || geom.logL2 < 1)
    return hipErrorInvalidValue;
  const int kr = L1 >= kNT4 ? L1 / kNT4 : 1;
  const dim3 grid((1 << geom.logL2) / 2, count);
  const size_t lds = sizeof(cplx<T>) * (size_t)lds_slots(2 * L1);
  auto go = [&](auto SY) {
    constexpr bool SYM = decltype(SY)::value != 0;
    return row_pick(kr, geom.logL1, [&](auto K, auto G) {
      constexpr int KR = decltype(K)::value;
      if constexpr (KR == 16)
        return launch_lds(k_row_w_b<T, true, SYM>, grid, 2 * kNT4, lds, s, args, tw);
      else
        return launch_lds(k_row_b<T, true, SYM, KR, decltype(G)::value>, grid, kNT4, lds, s, args,
                          tw);
    });
  };
  return geom.sym ? go(IC<1>{}) : go(IC<0>{});
}

template <typename T>
hipError_t launch_col_inv_batch(int mode, const LevelDev<T>& geom, const PassArgs<T>* args,
                                int count, const Twiddles<T>& tw, hipStream_t s) {
  int ept;
  if (count < 1 || count > 65535 || !col_geom_ok(geom.logL1, geom.logL2, geom.tcols, &ept) ||
      !epi_mode_built<T>(mode))
    return hipErrorInvalidValue;
  const dim3 grid(col_blocks(geom.logL1, geom.tcols), count);
  const size_t lds = sizeof(cplx<T>) * (size_t)lds_slots(ept * kNT4);
  auto go = [&](auto M) {
    constexpr int MODE = decltype(M)::value;
    return col_pick(ept, geom.tcols, geom.logL2, [&](auto E, auto NTc, auto G) {
      constexpr int NT = decltype(NTc)::value;
      return launch_lds(k_col_inv_b<T, MODE, decltype(E)::value, NT, decltype(G)::value>, grid,
                        NT, lds, s, args, tw);
    });
  };
  switch (mode) {
    case EPI_MV: return go(IC<EPI_MV>{});
    case EPI_RESID: return go(IC<EPI_RESID>{});
    case EPI_SMOOTH: return go(IC<EPI_SMOOTH>{});
    default: break;
  }
  if constexpr (sizeof(T) == 8) {
    if (mode == EPI_OUTER) return go(IC<EPI_OUTER>{});
  }
  return hipErrorInvalidValue;
}

}  // namespace amg
