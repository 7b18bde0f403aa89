// Device helpers shared by the four-step kernels and the one-workgroup tail
// kernels: four-step twiddles, restriction / prolongation stencils,
// circulant embedding columns, XCD-aware tile order, and the launch helper.
// Internal header.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <unordered_map>

#include "amg_device.hpp"
#include "fft_lds.hpp"

namespace amg {

__device__ __forceinline__ int ilog2(int x) { return 31 - __clz(x); }

template <typename T>
__device__ __forceinline__ cplx<T> tw4(const Twiddles<T>& tw, int logL, int e) {
  // e^{-2 pi i e / L}, 0 <= e < L <= 2^23, from two table lookups
  const int idx = e << (kTw4Log - logL);
  return cmul(tw.hi[idx >> 12], tw.lo[idx & (kTw4Lo - 1)]);
}

// w[k] = e^{-2 pi i (m0 + k ds) / L}, k < K <= 16: table values for the base
// and for ds, 2 ds, 4 ds, 8 ds; every other step power is a product of two of
// the ones before it (at most four roundings in all).
template <typename T, int K>
__device__ __forceinline__ void twiddle_run(const Twiddles<T>& tw, int logL, int m0, int ds,
                                            cplx<T>* w) {
  static_assert(K >= 1 && K <= 16, "run length");
  const int mask = (1 << logL) - 1;
  cplx<T> p[16];
  p[0] = tw4(tw, logL, m0 & mask);
  if constexpr (K > 1) p[1] = tw4(tw, logL, ds & mask);
  if constexpr (K > 2) p[2] = tw4(tw, logL, (2 * ds) & mask);
  if constexpr (K > 4) p[4] = tw4(tw, logL, (4 * ds) & mask);
  if constexpr (K > 8) p[8] = tw4(tw, logL, (8 * ds) & mask);
  if constexpr (K > 3) p[3] = cmul(p[1], p[2]);
  if constexpr (K > 5) {
#pragma unroll
    for (int r = 5; r < 8; ++r) p[r] = cmul(p[r - 4], p[4]);
  }
  if constexpr (K > 9) {
#pragma unroll
    for (int r = 9; r < 16; ++r) p[r] = cmul(p[r - 8], p[8]);
  }
  w[0] = p[0];
#pragma unroll
  for (int k = 1; k < K; ++k) w[k] = cmul(p[0], p[k]);
}

// The table entries behind the twiddle run e^{-2 pi i (m0 + k ds)/L}, k < K:
// hi/lo pairs of the base and of ds, 2 ds, 4 ds, 8 ds (as many as K needs),
// loaded ahead of their use.
template <typename T, int K>
struct RunTw {
  static constexpr int P = K == 1 ? 1 : (K == 2 ? 2 : (K == 4 ? 3 : (K == 8 ? 4 : 5)));
  cplx<T> hi[P], lo[P];
};
template <typename T, int K>
__device__ __forceinline__ void run_tw_load(const Twiddles<T>& tw, int logL, int m0, int ds,
                                            RunTw<T, K>& r) {
  const int mask = (1 << logL) - 1;
#pragma unroll
  for (int i = 0; i < RunTw<T, K>::P; ++i) {
    const int e = (i == 0 ? m0 : (ds << (i - 1))) & mask;
    const int idx = e << (kTw4Log - logL);
    r.hi[i] = tw.hi[idx >> 12];
    r.lo[i] = tw.lo[idx & (kTw4Lo - 1)];
  }
}

// a[k] *= w[k] (CONJ: conj(w[k])) for the run, with the same products as
// twiddle_run formed just before use so that few twiddles are live at a time.
template <typename T, int K, bool CONJ>
__device__ __forceinline__ void twiddle_run_mul_pre(const RunTw<T, K>& r, cplx<T>* a) {
  static_assert(K == 1 || K == 2 || K == 4 || K == 8 || K == 16, "run length");
  auto cj = [](cplx<T> x) { return CONJ ? conj(x) : x; };
  const cplx<T> p0 = cmul(r.hi[0], r.lo[0]);
  a[0] = cmul(a[0], cj(p0));
  if constexpr (K >= 2) {
    const cplx<T> p1 = cmul(r.hi[1], r.lo[1]);
    a[1] = cmul(a[1], cj(cmul(p0, p1)));
    if constexpr (K >= 4) {
      const cplx<T> p2 = cmul(r.hi[2], r.lo[2]);
      const cplx<T> p3 = cmul(p1, p2);
      a[2] = cmul(a[2], cj(cmul(p0, p2)));
      a[3] = cmul(a[3], cj(cmul(p0, p3)));
      if constexpr (K >= 8) {
        const cplx<T> p4 = cmul(r.hi[3], r.lo[3]);
        const cplx<T> p5 = cmul(p1, p4), p6 = cmul(p2, p4), p7 = cmul(p3, p4);
        a[4] = cmul(a[4], cj(cmul(p0, p4)));
        a[5] = cmul(a[5], cj(cmul(p0, p5)));
        a[6] = cmul(a[6], cj(cmul(p0, p6)));
        a[7] = cmul(a[7], cj(cmul(p0, p7)));
        if constexpr (K >= 16) {
          const cplx<T> p8 = cmul(r.hi[4], r.lo[4]);
          a[8] = cmul(a[8], cj(cmul(p0, p8)));
          a[9] = cmul(a[9], cj(cmul(p0, cmul(p1, p8))));
          a[10] = cmul(a[10], cj(cmul(p0, cmul(p2, p8))));
          a[11] = cmul(a[11], cj(cmul(p0, cmul(p3, p8))));
          a[12] = cmul(a[12], cj(cmul(p0, cmul(p4, p8))));
          a[13] = cmul(a[13], cj(cmul(p0, cmul(p5, p8))));
          a[14] = cmul(a[14], cj(cmul(p0, cmul(p6, p8))));
          a[15] = cmul(a[15], cj(cmul(p0, cmul(p7, p8))));
        }
      }
    }
  }
}

template <typename T, int K, bool CONJ>
__device__ __forceinline__ void twiddle_run_mul(const Twiddles<T>& tw, int logL, int m0, int ds,
                                                cplx<T>* a) {
  RunTw<T, K> r;
  run_tw_load<T, K>(tw, logL, m0, ds, r);
  twiddle_run_mul_pre<T, K, CONJ>(r, a);
}

// Prolongation 2 R^T at fine index m of a fine vector of length 2*mc + 1
// (mc = coarse length): odd m = 2i+1 -> e[i]; even m = 2i -> (e[i-1] + e[i])/2.
// Written as (e[lo] + e[hi])/2 with lo = floor((m-1)/2), hi = floor(m/2) and
// out-of-range terms dropped (for odd m both are e[i] and the halving is exact).
__device__ __forceinline__ void prolong_idx(int m, int mc, int& lo, int& hi, bool& oklo,
                                            bool& okhi) {
  lo = (m - 1) >> 1;
  hi = m >> 1;
  oklo = lo >= 0;
  okhi = hi < mc;
  lo = oklo ? lo : 0;
  hi = okhi ? hi : mc - 1;
}
template <typename T>
__device__ __forceinline__ T prolong_at(const T* e, int mc, int m) {
  int lo, hi;
  bool oklo, okhi;
  prolong_idx(m, mc, lo, hi, oklo, okhi);
  const T a = e[lo], b = e[hi];
  return T(0.5) * ((oklo ? a : T(0)) + (okhi ? b : T(0)));
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

// Raise a kernel's dynamic-LDS limit once to the largest size it is launched
// with (gfx950 has 160 KB of LDS per workgroup), then launch it.
template <typename... P, typename... A>
hipError_t launch_lds(void (*kernel)(P...), dim3 grid, int block, size_t lds, hipStream_t s,
                      A&&... args) {
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> done;
  const void* key = reinterpret_cast<const void*>(kernel);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = done.find(key);
    if (it == done.end() || it->second < lds) {
      const hipError_t e =
          hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      done[key] = lds;
    }
  }
  hipLaunchKernelGGL(kernel, grid, dim3(block), lds, s, std::forward<A>(args)...);
  return hipGetLastError();
}

}  // namespace amg
