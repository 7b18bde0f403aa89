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
__device__ __forceinline__ cplx<T> mk(T a, T b) { return cplx<T>{a, b}; }
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

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cplx<T>* a) {
  // radix-2 decimation in time: even/odd DFT4s, twiddles e^{-+2 pi i k/8}
  cplx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cplx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  const T s = T(0.70710678118654752440);
  // w1 = (1 -+ i)/sqrt2, w2 = -+i, w3 = (-1 -+ i)/sqrt2
  const cplx<T> w1 = INV ? cplx<T>{s, s} : cplx<T>{s, -s};
  const cplx<T> w3 = INV ? cplx<T>{-s, s} : cplx<T>{-s, -s};
  o1 = cmul(o1, w1);
  o2 = rot<T, INV>(o2);
  o3 = cmul(o3, w3);
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
  // cos/sin(k pi / 8), k = 0..7
  const T c[8] = {T(1.0), T(0.92387953251128675613), T(0.70710678118654752440),
                  T(0.38268343236508977173), T(0.0), T(-0.38268343236508977173),
                  T(-0.70710678118654752440), T(-0.92387953251128675613)};
  const T s[8] = {T(0.0), T(0.38268343236508977173), T(0.70710678118654752440),
                  T(0.92387953251128675613), T(1.0), T(0.92387953251128675613),
                  T(0.70710678118654752440), T(0.38268343236508977173)};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const cplx<T> w = INV ? cplx<T>{c[k], s[k]} : cplx<T>{c[k], -s[k]};
    const cplx<T> t = (k == 0) ? o[k] : cmul(o[k], w);
    a[k] = e[k] + t;
    a[k + 8] = e[k] - t;
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cplx<T>* a) {
  if constexpr (R == 2) dft2<T, INV>(a[0], a[1]);
  else if constexpr (R == 4) dft4<T, INV>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<T, INV>(a);
  else dft16<T, INV>(a);
}

// ---- Stockham FFT over signals in LDS ---------------------------------------
//
// S signals of length M (power of two); element i of signal s lives at
// lds[s*ss + i*es].  NT threads each own E elements per pass (S*M <= E*NT).
// Twiddles come from a base table tw[m] = e^{-2 pi i m / TWM} (conjugated for
// the inverse transform); M must divide TWM.  Output is in natural order, in
// place.  sigfast: consecutive threads take consecutive signals (use when
// ss == 1, i.e. signals interleaved), otherwise consecutive butterflies.

template <typename T, int R, int E, int NT, bool INV>
__device__ __forceinline__ void stockham_pass(cplx<T>* lds, int M, int S, int ss, int es,
                                              int Ns, bool sigfast, const cplx<T>* __restrict__ tw,
                                              int twM) {
  constexpr int NB = E / R;
  static_assert(NB >= 1 && NB * R == E, "radix must divide E");
  const int nbs = M / R;  // butterflies per signal
  const int total = nbs * S;
  cplx<T> a[E];
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int bf = threadIdx.x + e * NT;
    if (bf < total) {
      int s, j;
      if (sigfast) {
        s = bf % S;
        j = bf / S;
      } else {
        s = bf / nbs;
        j = bf - s * nbs;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) a[e * R + r] = lds[s * ss + (j + r * nbs) * es];
      // twiddle e^{-+2 pi i r k / (Ns R)}, k = j mod Ns
      const int k = j & (Ns - 1);
      if (Ns > 1) {
        const int step = twM / (Ns * R) * k;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = tw[r * step];
          if (INV) w.y = -w.y;
          a[e * R + r] = cmul(a[e * R + r], w);
        }
      }
      dft<T, R, INV>(a + e * R);
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int bf = threadIdx.x + e * NT;
    if (bf < total) {
      int s, j;
      if (sigfast) {
        s = bf % S;
        j = bf / S;
      } else {
        s = bf / nbs;
        j = bf - s * nbs;
      }
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[s * ss + (base + r * Ns) * es] = a[e * R + r];
    }
  }
  __syncthreads();
}

// Full FFT (forward if !INV) of S signals of length M in LDS, natural order in
// and out.  A single radix-2/4/8 pass first (no twiddles), then radix RMAX.
template <typename T, int E, int NT, bool INV>
__device__ void lds_fft(cplx<T>* lds, int M, int S, int ss, int es, bool sigfast,
                        const cplx<T>* __restrict__ tw, int twM) {
  constexpr int RMAX = E >= 16 ? 16 : E;
  constexpr int LR = RMAX == 16 ? 4 : (RMAX == 8 ? 3 : (RMAX == 4 ? 2 : 1));
  const int logM = 31 - __builtin_clz(M);
  int rem = logM % LR;
  int Ns = 1;
  if (rem == 1) {
    stockham_pass<T, 2, E, NT, INV>(lds, M, S, ss, es, Ns, sigfast, tw, twM);
    Ns = 2;
  } else if (rem == 2) {
    stockham_pass<T, 4, E, NT, INV>(lds, M, S, ss, es, Ns, sigfast, tw, twM);
    Ns = 4;
  } else if (rem == 3) {
    stockham_pass<T, 8, E, NT, INV>(lds, M, S, ss, es, Ns, sigfast, tw, twM);
    Ns = 8;
  }
  while (Ns < M) {
    stockham_pass<T, RMAX, E, NT, INV>(lds, M, S, ss, es, Ns, sigfast, tw, twM);
    Ns *= RMAX;
  }
}

}  // namespace amg
