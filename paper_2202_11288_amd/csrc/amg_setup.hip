// Hierarchy setup on the device: the finest Toeplitz-plus-Cross level from
// the row stencils (eq. (split01), eq. (ccs2.6)), the Galerkin coarse levels
// by the recurrences of Lemma 3.1, and the few scalars the host needs.  The
// same arithmetic as the host setup in amg_host.cpp, one thread per entry,
// so that a hierarchy of 2^22 intervals forms in milliseconds.
#include <hip/hip_runtime.h>

#include "amg_device.hpp"

namespace amg {

namespace {

__device__ __forceinline__ double stencil_at(const double* W, int64_t S, int64_t s2) {
  return (s2 < -S || s2 > S) ? 0.0 : W[s2 + S];
}

__device__ __forceinline__ void flag_bad(int* bad, double v) {
  if (!isfinite(v)) atomicOr(bad, 1);
}

constexpr int kSetupNT = 256;

inline unsigned setup_grid(int64_t count) {
  const int64_t g = (count + kSetupNT - 1) / kSetupNT;
  return (unsigned)(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

}  // namespace

// Finest level (N - 1 = n): generators a, b, c, d (2n - 1 entries, offsets
// -(n-1)..n-1) and Cross vectors from the node-row stencil Wn and the
// midpoint-row stencil Wm (half-grid offsets); then scale * (all) + shift on
// the diagonal entries a_0, d_0, o.
__global__ __launch_bounds__(kSetupNT) void k_finest_level(const double* Wn, int64_t Sn,
                                                           const double* Wm, int64_t Sm, int64_t n,
                                                           double scale, double shift, double* a,
                                                           double* b, double* c, double* d,
                                                           double* p, double* q, double* xi,
                                                           double* zeta, double* o, int* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 2 * n - 1; k += stride) {
    const int64_t dd = k - (n - 1);
    const double sh = dd == 0 ? shift : 0.0;
    a[k] = stencil_at(Wn, Sn, 2 * dd) * scale + sh;
    b[k] = stencil_at(Wn, Sn, 2 * dd + 1) * scale;
    c[k] = stencil_at(Wm, Sm, 2 * dd - 1) * scale;
    d[k] = stencil_at(Wm, Sm, 2 * dd) * scale + sh;
    flag_bad(bad, a[k] + b[k] + c[k] + d[k]);
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    p[i] = stencil_at(Wn, Sn, -2 * i - 1) * scale;
    q[i] = stencil_at(Wm, Sm, 2 * i + 1) * scale;
    xi[i] = stencil_at(Wm, Sm, -2 * i - 2) * scale;
    zeta[i] = stencil_at(Wm, Sm, 2 * i + 2) * scale;
    flag_bad(bad, p[i] + q[i] + xi[i] + zeta[i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    o[0] = stencil_at(Wm, Sm, 0) * scale + shift;
    flag_bad(bad, o[0]);
  }
}

// Lemma 3.1, Toeplitz part: t'_i = (t_{2i-2} + 4 t_{2i-1} + 6 t_{2i} +
// 4 t_{2i+1} + t_{2i+2}) / 8 for the four blocks (blockIdx.y).
__global__ __launch_bounds__(kSetupNT) void k_coarsen_toeplitz(const double* fa, const double* fb,
                                                               const double* fc, const double* fd,
                                                               int64_t n, double* ca, double* cb,
                                                               double* cc, double* cd, int* bad) {
  const double* f = blockIdx.y == 0 ? fa : (blockIdx.y == 1 ? fb : (blockIdx.y == 2 ? fc : fd));
  double* t = blockIdx.y == 0 ? ca : (blockIdx.y == 1 ? cb : (blockIdx.y == 2 ? cc : cd));
  const int64_t nc = (n - 1) / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 2 * nc - 1; k += stride) {
    const int64_t i = k - (nc - 1);
    const double* g = f + (n - 1);  // g[off] = t_off
    t[k] = (g[2 * i - 2] + 4 * g[2 * i - 1] + 6 * g[2 * i] + 4 * g[2 * i + 1] + g[2 * i + 2]) / 8.0;
    flag_bad(bad, t[k]);
  }
}

// Lemma 3.1, Cross part, first step: the fine w_o column A z (z = P e_{w_o})
// and row rho^T A on the v and w_bar blocks (n entries each).
__global__ __launch_bounds__(kSetupNT) void k_coarsen_cols(const double* fa, const double* fb,
                                                           const double* fc, const double* fd,
                                                           const double* p, const double* q,
                                                           const double* xi, const double* zeta,
                                                           int64_t n, double* colv, double* colw,
                                                           double* rowv, double* roww) {
  const double *ga = fa + (n - 1), *gb = fb + (n - 1), *gc = fc + (n - 1), *gd = fd + (n - 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    colv[i] = 0.5 * ga[n - 1 - i] + p[i] + 0.5 * gb[-i];
    colw[i] = 0.5 * gc[n - 1 - i] + xi[i] + 0.5 * gd[-i];
    rowv[i] = 0.25 * ga[i - n + 1] + 0.5 * q[i] + 0.25 * gc[i];
    roww[i] = 0.25 * gb[i - n + 1] + 0.5 * zeta[i] + 0.25 * gd[i];
  }
}

// Lemma 3.1, Cross part, second step: restrictions of those vectors give the
// coarse p, xi (column) and q, zeta (row, times 2), and the coarse o.
__global__ __launch_bounds__(kSetupNT) void k_coarsen_cross(const double* colv, const double* colw,
                                                            const double* rowv, const double* roww,
                                                            const double* q, const double* zeta,
                                                            const double* o, int64_t n,
                                                            double* pc, double* xic, double* qc,
                                                            double* zetac, double* oc, int* bad) {
  const int64_t nc = (n - 1) / 2;
  auto R = [](const double* x, int64_t i) {
    return 0.25 * (x[2 * i] + 2 * x[2 * i + 1] + x[2 * i + 2]);
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
    pc[i] = R(colv, i);
    xic[i] = R(colw, i);
    qc[i] = 2.0 * R(rowv, i);
    zetac[i] = 2.0 * R(roww, i);
    flag_bad(bad, pc[i] + xic[i] + qc[i] + zetac[i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double colo = 0.5 * q[n - 1] + o[0] + 0.5 * zeta[0];
    oc[0] = 0.25 * colv[n - 1] + 0.5 * colo + 0.25 * colw[0];
    flag_bad(bad, oc[0]);
  }
}

// A symmetric level's coarse image: the recurrences give mirror entries that
// agree only up to rounding; their averages keep the level exactly symmetric
// (A = D, C = B mirrored, p = q, xi = zeta).  Thread i owns the pair
// (i, m-1-i) of the generators (m = 2nc - 1) and entry i of the vectors.
__global__ __launch_bounds__(kSetupNT) void k_symmetrize(double* a, double* b, double* c, double* d,
                                                         double* p, double* q, double* xi,
                                                         double* zeta, int64_t nc) {
  const int64_t m = 2 * nc - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= (m - 1) / 2; i += stride) {
    const int64_t j = m - 1 - i;
    const double ai = a[i], aj = a[j], bi = b[i], bj = b[j], ci = c[i], cj = c[j];
    const double Ai = 0.5 * (ai + aj), Aj = 0.5 * (aj + ai);
    const double Bi = 0.5 * (bi + cj), Bj = 0.5 * (bj + ci);
    a[i] = Ai;
    a[j] = Aj;
    d[i] = Ai;
    d[j] = Aj;
    b[i] = Bi;
    b[j] = Bj;
    c[j] = Bi;
    c[i] = Bj;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
    const double pq = 0.5 * (p[i] + q[i]), xz = 0.5 * (xi[i] + zeta[i]);
    p[i] = pq;
    q[i] = pq;
    xi[i] = xz;
    zeta[i] = xz;
  }
}

// The level's diagonal scalars for the host: o, a_0, d_0.
__global__ void k_level_scalars(const double* a, const double* d, const double* o, int64_t n,
                                double* out) {
  if (threadIdx.x == 0) {
    out[0] = o[0];
    out[1] = a[n - 1];
    out[2] = d[n - 1];
  }
}

// Deterministic test data in [-1/2, 1/2) (a 32-bit integer hash of the
// index and the seed; inputs of the geometry tuner, whose results are only
// compared with each other).
__global__ __launch_bounds__(kSetupNT) void k_fill_hash(double* p, int64_t n, unsigned seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    unsigned h = (unsigned)i * 0x9E3779B1u ^ (unsigned)(i >> 32) ^ (seed * 0x85EBCA77u);
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    p[i] = (double)(h >> 8) * (1.0 / 16777216.0) - 0.5;
  }
}

hipError_t launch_fill_hash(double* p, int64_t n, unsigned seed, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_hash, setup_grid(n), kSetupNT, 0, s, p, n, seed);
  return hipGetLastError();
}

hipError_t launch_finest_level(const double* Wn, int64_t Sn, const double* Wm, int64_t Sm,
                               int64_t n, double scale, double shift, const DevTpx& f, int* bad,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_finest_level, setup_grid(2 * n), kSetupNT, 0, s, Wn, Sn, Wm, Sm, n, scale,
                     shift, f.a, f.b, f.c, f.d, f.p, f.q, f.xi, f.zeta, f.o, bad);
  return hipGetLastError();
}

hipError_t launch_coarsen(const DevTpx& f, int64_t n, const DevTpx& c, double* scratch, bool sym,
                          int* bad, hipStream_t s) {
  const int64_t nc = (n - 1) / 2;
  if (n < 3 || (n & 1) == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_coarsen_toeplitz, dim3(setup_grid(2 * nc), 4), kSetupNT, 0, s, f.a, f.b,
                     f.c, f.d, n, c.a, c.b, c.c, c.d, bad);
  double *colv = scratch, *colw = scratch + n, *rowv = scratch + 2 * n, *roww = scratch + 3 * n;
  hipLaunchKernelGGL(k_coarsen_cols, setup_grid(n), kSetupNT, 0, s, f.a, f.b, f.c, f.d, f.p, f.q,
                     f.xi, f.zeta, n, colv, colw, rowv, roww);
  hipLaunchKernelGGL(k_coarsen_cross, setup_grid(nc), kSetupNT, 0, s, colv, colw, rowv, roww, f.q,
                     f.zeta, f.o, n, c.p, c.xi, c.q, c.zeta, c.o, bad);
  if (sym)
    hipLaunchKernelGGL(k_symmetrize, setup_grid(nc), kSetupNT, 0, s, c.a, c.b, c.c, c.d, c.p, c.q,
                       c.xi, c.zeta, nc);
  return hipGetLastError();
}

hipError_t launch_level_scalars(const DevTpx& t, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_level_scalars, 1, 64, 0, s, t.a, t.d, t.o, n, out);
  return hipGetLastError();
}

}  // namespace amg
