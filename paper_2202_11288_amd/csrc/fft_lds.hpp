// Device building blocks of the circulant-embedding FFTs (Sec. 3.2,
// eq. (ccs3.4)): complex arithmetic, in-register DFTs of size 2/4/8/16, and a
// Stockham autosort FFT over signals held in LDS.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>

namespace amg {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> scale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
// Global loads / stores of one complex value as a single 2-wide vector access
// (keeps register staging arrays of complex values in registers).
template <typename T>
__device__ __forceinline__ cplx<T> ldg(const cplx<T>* p) {
  using V = T __attribute__((ext_vector_type(2)));
  const V v = *reinterpret_cast<const V*>(p);
  return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void stg(cplx<T>* p, cplx<T> a) {
  using V = T __attribute__((ext_vector_type(2)));
  *reinterpret_cast<V*>(p) = V{a.x, a.y};
}

// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> rot(cplx<T> a) {
  return INV ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
}

// ---- in-register DFTs: X_k = sum_j a_j e^{-+2 pi i jk/R} (natural order) ----

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cplx<T>& a0, cplx<T>& a1) {
  const cplx<T> t = a0 - a1;
  a0 = a0 + a1;
  a1 = t;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cplx<T>& a0, cplx<T>& a1, cplx<T>& a2, cplx<T>& a3) {
  const cplx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = rot<T, INV>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

// (1 -+ i)/sqrt2 * a and (-1 -+ i)/sqrt2 * a without a general complex product
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> w8_1(cplx<T> a) {
  const T s = T(0.70710678118654752440);
  return INV ? cplx<T>{s * (a.x - a.y), s * (a.x + a.y)} : cplx<T>{s * (a.x + a.y), s * (a.y - a.x)};
}
template <typename T, bool INV>
__device__ __forceinline__ cplx<T> w8_3(cplx<T> a) {
  const T s = T(0.70710678118654752440);
  return INV ? cplx<T>{-s * (a.x + a.y), s * (a.x - a.y)} : cplx<T>{s * (a.y - a.x), -s * (a.x + a.y)};
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cplx<T>* a) {
  // radix-2 decimation in time: even/odd DFT4s, twiddles e^{-+2 pi i k/8}
  cplx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cplx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  o1 = w8_1<T, INV>(o1);
  o2 = rot<T, INV>(o2);
  o3 = w8_3<T, INV>(o3);
  a[0] = e0 + o0; a[4] = e0 - o0;
  a[1] = e1 + o1; a[5] = e1 - o1;
  a[2] = e2 + o2; a[6] = e2 - o2;
  a[3] = e3 + o3; a[7] = e3 - o3;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft16(cplx<T>* a) {
  cplx<T> e[8], o[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    e[j] = a[2 * j];
    o[j] = a[2 * j + 1];
  }
  dft8<T, INV>(e);
  dft8<T, INV>(o);
  // e^{-+2 pi i k/16}: k = 2, 4, 6 reuse the eighth roots; 1, 3, 5, 7 need a product
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
  const cplx<T> w1 = INV ? cplx<T>{c1, s1} : cplx<T>{c1, -s1};
  const cplx<T> w3 = INV ? cplx<T>{s1, c1} : cplx<T>{s1, -c1};
  const cplx<T> w5 = INV ? cplx<T>{-s1, c1} : cplx<T>{-s1, -c1};
  const cplx<T> w7 = INV ? cplx<T>{-c1, s1} : cplx<T>{-c1, -s1};
  o[1] = cmul(o[1], w1);
  o[2] = w8_1<T, INV>(o[2]);
  o[3] = cmul(o[3], w3);
  o[4] = rot<T, INV>(o[4]);
  o[5] = cmul(o[5], w5);
  o[6] = w8_3<T, INV>(o[6]);
  o[7] = cmul(o[7], w7);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a[k] = e[k] + o[k];
    a[k + 8] = e[k] - o[k];
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cplx<T>* a) {
  if constexpr (R == 2) dft2<T, INV>(a[0], a[1]);
  else if constexpr (R == 4) dft4<T, INV>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<T, INV>(a);
  else dft16<T, INV>(a);
}

// ---- LDS view with a one-in-sixteen skew -------------------------------------
// Element i lives at slot i + i/16: the power-of-two strides of the Stockham
// stores (R*16 B, R*T*16 B) then fall on distinct 16-byte bank groups.
template <typename T>
struct Lds {
  cplx<T>* p;
  __device__ __forceinline__ cplx<T>& operator[](int i) const { return p[i + (i >> 4)]; }
};
__host__ __device__ constexpr int lds_slots(int count) { return count + (count >> 4) + 1; }

// Twiddles w_r = e^{-2 pi i r step / 2^logtw} for r = 1..R-1 from at most four
// table loads (w1, w2, w4, w8) and products of two or three of them.
template <typename T, int R>
__device__ __forceinline__ void twiddle_set(const cplx<T>* __restrict__ tw, int step, cplx<T>* w) {
  w[1] = tw[step];
  if constexpr (R >= 4) {
    w[2] = tw[2 * step];
    w[3] = cmul(w[1], w[2]);
  }
  if constexpr (R >= 8) {
    w[4] = tw[4 * step];
    w[5] = cmul(w[1], w[4]);
    w[6] = cmul(w[2], w[4]);
    w[7] = cmul(w[3], w[4]);
  }
  if constexpr (R >= 16) {
    w[8] = tw[8 * step];
#pragma unroll
    for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
  }
}

// a[r] *= w_r (conjugated for the inverse), r = 1..15, with the same products
// as twiddle_set formed just before use (conj(x) conj(y) = conj(xy) exactly),
// so that at most eight twiddles are live at a time.
template <typename T, bool INV>
__device__ __forceinline__ void twiddle16_mul(cplx<T> (&a)[16], cplx<T> w1, cplx<T> w2, cplx<T> w4,
                                              cplx<T> w8) {
  if (INV) {
    w1 = conj(w1);
    w2 = conj(w2);
    w4 = conj(w4);
    w8 = conj(w8);
  }
  const cplx<T> w3 = cmul(w1, w2), w5 = cmul(w1, w4), w6 = cmul(w2, w4), w7 = cmul(w3, w4);
  a[1] = cmul(a[1], w1);
  a[2] = cmul(a[2], w2);
  a[3] = cmul(a[3], w3);
  a[4] = cmul(a[4], w4);
  a[5] = cmul(a[5], w5);
  a[6] = cmul(a[6], w6);
  a[7] = cmul(a[7], w7);
  a[8] = cmul(a[8], w8);
  a[9] = cmul(a[9], cmul(w1, w8));
  a[10] = cmul(a[10], cmul(w2, w8));
  a[11] = cmul(a[11], cmul(w3, w8));
  a[12] = cmul(a[12], cmul(w4, w8));
  a[13] = cmul(a[13], cmul(w5, w8));
  a[14] = cmul(a[14], cmul(w6, w8));
  a[15] = cmul(a[15], cmul(w7, w8));
}
template <typename T, bool INV>
__device__ __forceinline__ void twiddle16_apply(cplx<T> (&a)[16], const cplx<T>* __restrict__ tw,
                                                int step) {
  twiddle16_mul<T, INV>(a, tw[step], tw[2 * step], tw[4 * step], tw[8 * step]);
}

// ---- Stockham FFT over signals in LDS ---------------------------------------
//
// S = 2^logS signals of length M = 2^logM; element i of signal s lives at
// lds[(s << logss) + (i << loges)].  NT threads each own E elements per pass
// (S*M <= E*NT).  Twiddles come from a base table tw[m] = e^{-2 pi i m/2^logtw}
// (conjugated for the inverse transform), M <= 2^logtw.  Output is in natural
// order, in place.  sigfast: consecutive threads take consecutive signals (use
// when signals are interleaved), otherwise consecutive butterflies.
struct FftGeom {
  int logM, logS, logss, loges, logtw;
  bool sigfast;
};

template <typename T, int R, int E, int NT, bool INV>
__device__ __forceinline__ void stockham_pass(Lds<T> lds, const FftGeom& g, int logNs,
                                              const cplx<T>* __restrict__ tw) {
  constexpr int NB = E / R;
  constexpr int LR = R == 16 ? 4 : (R == 8 ? 3 : (R == 4 ? 2 : 1));
  static_assert(NB >= 1 && NB * R == E, "radix must divide E");
  const int lognbs = g.logM - LR;  // butterflies per signal = M / R
  const int total = 1 << (lognbs + g.logS);
  const int Ns = 1 << logNs;
  cplx<T> a[E];
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int bf = threadIdx.x + e * NT;
    if (bf < total) {
      const int s = g.sigfast ? (bf & ((1 << g.logS) - 1)) : (bf >> lognbs);
      const int j = g.sigfast ? (bf >> g.logS) : (bf & ((1 << lognbs) - 1));
      const int base = s << g.logss;
#pragma unroll
      for (int r = 0; r < R; ++r) a[e * R + r] = lds[base + ((j + (r << lognbs)) << g.loges)];
      if (logNs > 0) {
        // e^{-+2 pi i r k / (Ns R)}, k = j mod Ns
        const int k = j & (Ns - 1);
        cplx<T> w[R];
        twiddle_set<T, R>(tw, k << (g.logtw - logNs - LR), w);
#pragma unroll
        for (int r = 1; r < R; ++r) a[e * R + r] = cmul(a[e * R + r], INV ? conj(w[r]) : w[r]);
      }
      dft<T, R, INV>(a + e * R);
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int bf = threadIdx.x + e * NT;
    if (bf < total) {
      const int s = g.sigfast ? (bf & ((1 << g.logS) - 1)) : (bf >> lognbs);
      const int j = g.sigfast ? (bf >> g.logS) : (bf & ((1 << lognbs) - 1));
      const int k = j & (Ns - 1);
      const int out = ((j - k) << LR) + k;
      const int base = s << g.logss;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[base + ((out + (r << logNs)) << g.loges)] = a[e * R + r];
    }
  }
  __syncthreads();
}

// Full FFT (forward if !INV) of the signals in LDS, natural order in and out.
// A single radix-2/4/8 pass first (no twiddles), then radix RMAX passes.
template <typename T, int E, int NT, bool INV>
__device__ __forceinline__ void lds_fft(Lds<T> lds, const FftGeom& g, const cplx<T>* __restrict__ tw) {
  constexpr int RMAX = E >= 16 ? 16 : E;
  constexpr int LR = RMAX == 16 ? 4 : (RMAX == 8 ? 3 : (RMAX == 4 ? 2 : 1));
  const int rem = g.logM % LR;
  int logNs = 0;
  if (rem == 1) {
    stockham_pass<T, 2, E, NT, INV>(lds, g, 0, tw);
    logNs = 1;
  } else if (rem == 2) {
    stockham_pass<T, 4, E, NT, INV>(lds, g, 0, tw);
    logNs = 2;
  } else if (rem == 3) {
    stockham_pass<T, 8, E, NT, INV>(lds, g, 0, tw);
    logNs = 3;
  }
  while (logNs < g.logM) {
    stockham_pass<T, RMAX, E, NT, INV>(lds, g, logNs, tw);
    logNs += LR;
  }
}

// FFT of the signals in LDS with the first and last passes on registers.
// Each thread owns one radix-16 butterfly of the last pass: signal s, index
// j0 < M/16 (M = 2^logM >= 32).  On entry a[e] = x_s[j0 + e M/16] (natural
// order), on exit a[e] = X_s[j0 + e M/16]; the NT threads of the workgroup
// must cover every (s, j0) pair exactly once.  The first pass (radix
// 2^(logM mod 4), or 16) works on the registers and writes LDS, the middle
// radix-16 passes stay in LDS, the last one reads LDS back into registers.
// No barrier at the end: synchronise before the LDS region is written again.
template <typename T, int R0, bool INV>
__device__ __forceinline__ void first_pass_regs(cplx<T> (&a)[16], Lds<T> lds, const FftGeom& g,
                                                int base, int j0, int q) {
  constexpr int NB = 16 / R0;
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    cplx<T> b[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) b[r] = a[e + r * NB];  // x[j + r M/R0], j = j0 + e M/16
    dft<T, R0, INV>(b);
    const int j = j0 + (e << q);
#pragma unroll
    for (int r = 0; r < R0; ++r) lds[base + ((j * R0 + r) << g.loges)] = b[r];
  }
}

template <typename T, int NT, bool INV>
__device__ __forceinline__ void fft_reg16(cplx<T> (&a)[16], Lds<T> lds, const FftGeom& g, int s,
                                          int j0, const cplx<T>* __restrict__ tw) {
  const int q = g.logM - 4;  // log2(M/16)
  const int base = s << g.logss;
  const int rem = g.logM & 3;
  if (rem == 1) first_pass_regs<T, 2, INV>(a, lds, g, base, j0, q);
  else if (rem == 2) first_pass_regs<T, 4, INV>(a, lds, g, base, j0, q);
  else if (rem == 3) first_pass_regs<T, 8, INV>(a, lds, g, base, j0, q);
  else first_pass_regs<T, 16, INV>(a, lds, g, base, j0, q);
  __syncthreads();
  for (int logNs = rem == 0 ? 4 : rem; logNs < q; logNs += 4)
    stockham_pass<T, 16, 16, NT, INV>(lds, g, logNs, tw);
  // last pass, Ns = M/16: butterfly j0 (k = j0), outputs j0 + r M/16
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = lds[base + ((j0 + (r << q)) << g.loges)];
  twiddle16_apply<T, INV>(a, tw, j0 << (g.logtw - g.logM));
  dft<T, 16, INV>(a);
}

// ---- LDS FFT with prefetched twiddles ----------------------------------------
// The same pass sequence as lds_fft with E = 16 (a radix 2/4/8/16 first pass
// without twiddles, then radix-16 passes, one butterfly per thread), for
// signals of at most 4096 points in all (at most two radix-16 passes after the
// first).  The twiddle bases w, w^2, w^4, w^8 of every radix-16 pass depend
// only on the geometry and the thread, so they are fetched at kernel start,
// under the signal's own loads, instead of inside each pass.
template <typename T>
struct FftTw {
  cplx<T> w[2][4];
};

template <typename T>
__device__ __forceinline__ void lds_fft_tw_prefetch(const FftGeom& g, const cplx<T>* __restrict__ tw,
                                                    FftTw<T>& f) {
  const int rem = g.logM & 3;
  const int lognbs = g.logM - 4;
  const int bf = threadIdx.x;
  const int j = g.sigfast ? (bf >> g.logS) : (bf & ((1 << lognbs) - 1));
  int logNs = rem == 0 ? 4 : rem;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    // threads past the last butterfly load in-range entries they never use
    const int k = j & ((1 << logNs) - 1);
    const int step = logNs < g.logM ? (k << (g.logtw - logNs - 4)) : 0;
    f.w[p][0] = tw[step];
    f.w[p][1] = tw[2 * step];
    f.w[p][2] = tw[4 * step];
    f.w[p][3] = tw[8 * step];
    logNs += 4;
  }
}

// One radix-16 pass (E = 16, NB = 1) with the thread's twiddle bases given.
template <typename T, int NT, bool INV>
__device__ __forceinline__ void stockham16_pre(Lds<T> lds, const FftGeom& g, int logNs,
                                               const cplx<T> (&w)[4]) {
  const int lognbs = g.logM - 4;
  const int total = 1 << (lognbs + g.logS);
  const int bf = threadIdx.x;
  const bool act = bf < total;
  const int s = g.sigfast ? (bf & ((1 << g.logS) - 1)) : (bf >> lognbs);
  const int j = g.sigfast ? (bf >> g.logS) : (bf & ((1 << lognbs) - 1));
  const int base = s << g.logss;
  cplx<T> a[16];
  if (act) {
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = lds[base + ((j + (r << lognbs)) << g.loges)];
    twiddle16_mul<T, INV>(a, w[0], w[1], w[2], w[3]);
    dft<T, 16, INV>(a);
  }
  __syncthreads();
  if (act) {
    const int k = j & ((1 << logNs) - 1);
    const int out = ((j - k) << 4) + k;
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[base + ((out + (r << logNs)) << g.loges)] = a[r];
  }
  __syncthreads();
}

template <typename T, int NT, bool INV>
__device__ __forceinline__ void lds_fft_pf(Lds<T> lds, const FftGeom& g, const FftTw<T>& f) {
  const int rem = g.logM & 3;
  int logNs;
  if (rem == 1) {
    stockham_pass<T, 2, 16, NT, INV>(lds, g, 0, nullptr);
    logNs = 1;
  } else if (rem == 2) {
    stockham_pass<T, 4, 16, NT, INV>(lds, g, 0, nullptr);
    logNs = 2;
  } else if (rem == 3) {
    stockham_pass<T, 8, 16, NT, INV>(lds, g, 0, nullptr);
    logNs = 3;
  } else {
    stockham_pass<T, 16, 16, NT, INV>(lds, g, 0, nullptr);
    logNs = 4;
  }
  if (logNs < g.logM) {
    stockham16_pre<T, NT, INV>(lds, g, logNs, f.w[0]);
    logNs += 4;
  }
  if (logNs < g.logM) stockham16_pre<T, NT, INV>(lds, g, logNs, f.w[1]);
}

// Deterministic reduction of one value per thread over a workgroup of NT
// threads: butterfly within each wave (lane 0's fixed order), then the wave
// partials in index order.  Every thread returns the same value.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v, T* red /* >= NT/64 entries */) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

}  // namespace amg
