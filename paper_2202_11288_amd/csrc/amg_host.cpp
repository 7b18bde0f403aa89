// Host numerics: product-integration generators (Sec. 2.2, eq. (ccs2.1),
// shifted-symmetric rule of eq. (system1)), Galerkin coarsening (Lemma 3.1),
// coarsest LU (Algorithm 2, B_1 = A_1^{-1}), twiddle tables.
#include "amg_host.hpp"

#include <cmath>
#include <complex>
#include <cstring>
#include <sstream>

namespace amg {

namespace {

double kernel_c(const KernelSpec& k) {
  if (is_fractional(k.kind)) return (1.0 - k.alpha) * std::pow(k.delta, 2.0 * k.alpha - 2.0);
  return 3.0 / (2.0 * k.delta * k.delta * k.delta);
}

// Gauss-Legendre nodes/weights on [0,1] (Newton iteration on P_n, long double).
struct GaussLegendre {
  std::vector<double> x, w;
  explicit GaussLegendre(int n) : x(n), w(n) {
    const long double pi = acosl(-1.0L);
    for (int i = 0; i < n; ++i) {
      long double z = cosl(pi * (i + 0.75L) / (n + 0.5L)), dp = 0;
      for (int it = 0; it < 100; ++it) {
        long double p0 = 1, p1 = z;
        for (int j = 2; j <= n; ++j) {
          long double p2 = ((2 * j - 1) * z * p1 - (j - 1) * p0) / j;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1);
        long double dz = p1 / dp;
        z -= dz;
        if (fabsl(dz) < 1e-19L) break;
      }
      x[i] = (double)((1 - z) / 2);
      w[i] = (double)(1 / ((1 - z * z) * dp * dp));  // = 2/((1-z^2)P'^2) / 2
    }
  }
};

// int_0^theta (k + t)^beta t^j dt for j = 0,1,2 (dimensionless).  k = 0:
// closed form (j >= 1; j = 0 diverges and is never requested).  k >= 1: the
// integrand is analytic on a neighbourhood of [0, theta] whose nearest
// singularity is at t = -k, so 32-point Gauss-Legendre is exact to rounding.
void frac_cell(int64_t k, double theta, double beta, double J[3]) {
  if (k == 0) {
    J[0] = NAN;
    J[1] = std::pow(theta, beta + 2) / (beta + 2);
    J[2] = std::pow(theta, beta + 3) / (beta + 3);
    return;
  }
  // nearest singularity at distance k from the cell: 12 points suffice for
  // k >= 4 (Bernstein-ellipse factor > 17), 32 points below.
  static const GaussLegendre gl32(32), gl12(12);
  const GaussLegendre& gl = (k >= 4) ? gl12 : gl32;
  long double s0 = 0, s1 = 0, s2 = 0;
  for (size_t i = 0; i < gl.x.size(); ++i) {
    const double t = theta * gl.x[i];
    const long double f = (long double)gl.w[i] * std::pow((double)k + t, beta);
    s0 += f;
    s1 += f * t;
    s2 += f * t * t;
  }
  J[0] = (double)(s0 * theta);
  J[1] = (double)(s1 * theta);
  J[2] = (double)(s2 * theta);
}

// int_{t0}^{t1} t^beta t^j dt for j = 0,1,2 and 0 < t0 (zero when t1 <= t0):
// the integrand's singularity at t = 0 lies a distance t0 >= (t1 - t0)
// before the interval on the cells this is used for, so 32-point
// Gauss-Legendre is exact to rounding.
void frac_cell_from(double t0, double t1, double beta, double J[3]) {
  J[0] = J[1] = J[2] = 0.0;
  if (!(t1 > t0)) return;
  static const GaussLegendre gl32(32);
  const double len = t1 - t0;
  long double s0 = 0, s1 = 0, s2 = 0;
  for (size_t i = 0; i < gl32.x.size(); ++i) {
    const double t = t0 + len * gl32.x[i];
    const long double f = (long double)gl32.w[i] * std::pow(t, beta);
    s0 += f;
    s1 += f * t;
    s2 += f * t * t;
  }
  J[0] = (double)(s0 * len);
  J[1] = (double)(s1 * len);
  J[2] = (double)(s2 * len);
}

}  // namespace

bool TpxLevel::symmetric() const {
  if (has_band()) return false;
  const int64_t m = 2 * n - 1;
  for (int64_t i = 0; i < m; ++i) {
    if (a[i] != a[m - 1 - i] || d[i] != a[i] || c[i] != b[m - 1 - i]) return false;
  }
  for (int64_t i = 0; i < n; ++i)
    if (p[i] != q[i] || xi[i] != zeta[i]) return false;
  return true;
}

std::string validate(const KernelSpec& k, int64_t N, int coarsest_log2) {
  std::ostringstream e;
  if (N <= 0 || (N & (N - 1)) != 0) e << "N must be a power of two; ";
  int K = 0;
  while (N > 0 && (int64_t(1) << K) < N) ++K;
  if (coarsest_log2 < 2) e << "coarsest_log2 must be >= 2; ";
  if (K <= coarsest_log2) e << "need log2(N) > coarsest_log2; ";
  if (K > 22) e << "log2(N) <= 22 is supported; ";
  if (k.kind < 0 || k.kind > 5) e << "unknown kernel kind; ";
  if (k.kind == K_WEAKLY_SINGULAR) {
    if (!(k.gamma >= 0.0 && k.gamma < 1.0)) e << "weakly singular kernel needs 0 <= gamma < 1; ";
  } else if (k.kind != K_GENERATORS) {
    if (!(k.delta > 0.0 && k.delta < 0.5)) e << "need 0 < delta < 1/2; ";
  } else if (k.gen == nullptr) {
    e << "AMG_K_GENERATORS needs gen; ";
  }
  if (k.kind == K_FRACTIONAL && !(k.alpha > 0.0 && k.alpha < 0.5))
    e << "fractional kernel needs 0 < alpha < 1/2; ";
  if (k.kind == K_FRACTIONAL_NEAR && !(k.alpha > 0.0 && k.alpha < 1.0))
    e << "fractional kernel with the near-field rule needs 0 < alpha < 1; ";
  if (k.kind == K_WEIGHTED && !(std::isfinite(k.wl) && std::isfinite(k.wr) && k.wl > 0 && k.wr > 0))
    e << "weights must be positive; ";
  if (k.scheme != SCHEME_SHIFTED && k.scheme != SCHEME_STANDARD) e << "unknown scheme; ";
  return e.str();
}

namespace {

// int_0^1 |a - t|^-gamma t^j dt, j = 0, 1, 2, for a = a2 / 2 (the collocation
// point's position in the cell's local coordinate t; a multiple of 1/2).
// The point on the cell's end or at its midpoint: closed forms of the
// end-point singularity; elsewhere the integrand is analytic on [0, 1] with
// its singularity at distance >= 1/2, so Gauss-Legendre is exact to rounding
// (32 points up to distance 4, 12 beyond).
void ws_cell_moments(double gamma, int64_t a2, double J[3]) {
  const double g = gamma;
  if (a2 == 0) {
    for (int j = 0; j < 3; ++j) J[j] = 1.0 / (j + 1 - g);
    return;
  }
  if (a2 == 2) {  // substitute s = 1 - t
    J[0] = 1.0 / (1 - g);
    J[1] = 1.0 / (1 - g) - 1.0 / (2 - g);
    J[2] = 1.0 / (1 - g) - 2.0 / (2 - g) + 1.0 / (3 - g);
    return;
  }
  if (a2 == 1) {  // both halves from the midpoint: (1/2 -+ s)^j, s in [0, 1/2]
    const double M0 = std::pow(0.5, 1 - g) / (1 - g), M2 = std::pow(0.5, 3 - g) / (3 - g);
    J[0] = 2 * M0;
    J[1] = M0;
    J[2] = 0.5 * M0 + 2 * M2;
    return;
  }
  static const GaussLegendre gl32(32), gl12(12);
  const double a = 0.5 * (double)a2;
  const double dist = a < 0 ? -a : a - 1;
  const GaussLegendre& gl = (dist >= 4) ? gl12 : gl32;
  long double s0 = 0, s1 = 0, s2 = 0;
  for (size_t i = 0; i < gl.x.size(); ++i) {
    const double t = gl.x[i];
    const long double f = (long double)gl.w[i] * std::pow(std::fabs(a - t), -g);
    s0 += f;
    s1 += f * t;
    s2 += f * t * t;
  }
  J[0] = (double)s0;
  J[1] = (double)s1;
  J[2] = (double)s2;
}

// Quadratic Lagrange basis on a cell, coefficients of t^0, t^1, t^2.
constexpr double kLeft[3] = {1, -3, 2}, kMidB[3] = {0, 4, -4}, kRight[3] = {0, -1, 2};

double ws_apply(const double J[3], const double* l) { return l[0] * J[0] + l[1] * J[1] + l[2] * J[2]; }

}  // namespace

void ws_stencils(double gamma, int64_t N, std::vector<double>& Wn, std::vector<double>& Wm,
                 int64_t* Sout) {
  // unknown at half-step offset s2 from the collocation point: a node's cells
  // are [s2-2, s2] (it is their right end) and [s2, s2+2] (left end), local
  // a2 = 2 - s2 and -s2; a midpoint's cell is [s2-1, s2+1], a2 = 1 - s2.
  // Node rows see nodes at even s2, midpoint rows at odd s2.  Symmetric in s2.
  const int64_t S = 2 * N;
  const double sc = std::pow(1.0 / (double)N, 1.0 - gamma);
  std::vector<double> J((size_t)(3 * (2 * S + 6)));
  auto Jat = [&](int64_t a2) { return &J[(size_t)(3 * (a2 + S + 2))]; };
  for (int64_t a2 = -S - 2; a2 <= S + 2; ++a2) ws_cell_moments(gamma, a2, Jat(a2));
  Wn.assign((size_t)(2 * S + 1), 0.0);
  Wm.assign((size_t)(2 * S + 1), 0.0);
  for (int64_t s2 = 0; s2 <= S; ++s2) {
    const double wnode = ws_apply(Jat(2 - s2), kRight) + ws_apply(Jat(-s2), kLeft);
    const double wmid = ws_apply(Jat(1 - s2), kMidB);
    const double en = -sc * ((s2 % 2 == 0) ? wnode : wmid);
    const double em = -sc * ((s2 % 2 == 0) ? wmid : wnode);
    Wn[S + s2] = Wn[S - s2] = en;
    Wm[S + s2] = Wm[S - s2] = em;
  }
  *Sout = S;
}

void ws_boundary_coupling(double gamma, int64_t N, double* K0, double* K1) {
  // boundary node x = 0: its right cell only (left end), a2 = c; x = 1: its
  // left cell only (right end), a2 = c - (2N - 2); block order of the rows
  const double sc = std::pow(1.0 / (double)N, 1.0 - gamma);
  const int64_t m = 2 * N - 1;
  for (int64_t idx = 0; idx < m; ++idx) {
    const int64_t c = (idx < N - 1) ? 2 * (idx + 1) : 2 * (idx - (N - 1)) + 1;
    double J[3];
    ws_cell_moments(gamma, c, J);
    K0[idx] = sc * ws_apply(J, kLeft);
    ws_cell_moments(gamma, c - (2 * N - 2), J);
    K1[idx] = sc * ws_apply(J, kRight);
  }
}

namespace {

// The own-point weight int gamma (1 - l_0) equals -sum_{k != 0} W(k): the
// quadratic basis is a partition of unity on every cell, so a row whose
// stencil lies inside the interval sums to zero.  Summed cell by cell in FP64
// it drifts by many units in its last place at large N (tens at N = 2^22 for
// the fractional kernel, 5e7 in size there), which alone moves A x by that
// much times x; it is set from the identity, summed in long double.
void own_weight_from_row_sum(std::vector<double>& W, int64_t S) {
  // four long double partial sums (independent chains), combined pairwise
  long double acc[4] = {0.0L, 0.0L, 0.0L, 0.0L};
  const int64_t m = (int64_t)W.size();
  auto add_range = [&](int64_t lo, int64_t hi) {
    int64_t i = lo;
    for (; i + 3 < hi; i += 4)
      for (int q = 0; q < 4; ++q) acc[q] += (long double)W[(size_t)(i + q)];
    for (int q = 0; i < hi; ++i, ++q) acc[q] += (long double)W[(size_t)i];
  };
  add_range(0, S);
  add_range(S + 1, m);
  W[(size_t)S] = (double)(-((acc[0] + acc[1]) + (acc[2] + acc[3])));
}

}  // namespace

void row_stencil_into(const KernelSpec& k, int64_t N, std::vector<double>& W, int64_t* Sout) {
  const double h = 1.0 / (double)N;
  const double R = k.delta * (double)N;  // exact: N is a power of two
  const int64_t r = (int64_t)std::floor(R);
  const double th_last = R - (double)r;
  const int64_t ncell = r + (th_last > 0.0 ? 1 : 0);
  const int64_t S = 2 * ncell;
  W.assign((size_t)(2 * S + 1), 0.0);
  const double c = kernel_c(k);
  const bool frac = is_fractional(k.kind);
  const bool near = k.kind == K_FRACTIONAL_NEAR;
  const double beta = frac ? -1.0 - 2.0 * k.alpha : 0.0;
  const double scale = frac ? c * std::pow(h, beta + 1.0) : c * h;
  const double wr = (k.kind == K_WEIGHTED) ? k.wr : 1.0;
  const double wl = (k.kind == K_WEIGHTED) ? k.wl : 1.0;
  if (near) {
    // |t| <= rho h, rho = min(1/2, theta_0): the quadratic through the
    // half-grid neighbours x_c -+ h/2 and x_c; its linear term cancels
    // between the sides, its quadratic term 2 t^2 (u_+ - 2 u_c + u_-) / h^2
    // gives the weight m = (4/h^2) int_0^{rho h} gamma t^2 dt of the second
    // difference (both sides together)
    const double th0 = (r > 0) ? 1.0 : th_last;
    const double rho = std::fmin(0.5, th0);
    const double m = 4.0 * scale * std::pow(rho, beta + 3.0) / (beta + 3.0);
    W[S] += 2.0 * m;
    W[S - 1] -= m;
    W[S + 1] -= m;
  }
  // cell k: t in [k h, (k+theta) h]; quadratic through local tau = 0, 1/2, 1:
  //   l_a = 1 - 3 tau + 2 tau^2,  l_b = 4 tau - 4 tau^2,  l_c = 2 tau^2 - tau.
  for (int64_t kc = 0; kc < ncell; ++kc) {
    const double th = (kc < r) ? 1.0 : th_last;
    double J[3];
    if (near && kc == 0) {
      // the cell's own quadratic beyond the near part: tau in [1/2, th]
      frac_cell_from(0.5, th, beta, J);
    } else if (frac) {
      frac_cell(kc, th, beta, J);
    } else {
      J[0] = th;
      J[1] = th * th / 2.0;
      J[2] = th * th * th / 3.0;
    }
    for (double& v : J) v *= scale;
    const double Ib = 4 * J[1] - 4 * J[2];
    const double Ic = 2 * J[2] - J[1];
    const double own = (kc == 0) ? (3 * J[1] - 2 * J[2]) : J[0];  // int gamma (1 - l_0)
    W[S] += (wr + wl) * own;
    if (kc > 0) {
      const double Ia = J[0] - 3 * J[1] + 2 * J[2];
      W[S + 2 * kc] -= wr * Ia;
      W[S - 2 * kc] -= wl * Ia;
    }
    W[S + 2 * kc + 1] -= wr * Ib;
    W[S - 2 * kc - 1] -= wl * Ib;
    W[S + 2 * kc + 2] -= wr * Ic;
    W[S - 2 * kc - 2] -= wl * Ic;
  }
  own_weight_from_row_sum(W, S);
  *Sout = S;
}

std::vector<double> row_stencil(const KernelSpec& k, int64_t N, int64_t* Sout) {
  std::vector<double> W;
  row_stencil_into(k, N, W, Sout);
  return W;
}

std::vector<double> midpoint_stencil_standard(const KernelSpec& k, int64_t N, int64_t* Sout) {
  const double h = 1.0 / (double)N;
  const double R = k.delta * (double)N;  // exact: N is a power of two
  const double c = kernel_c(k) * h;
  const double wr = (k.kind == K_WEIGHTED) ? k.wr : 1.0;
  const double wl = (k.kind == K_WEIGHTED) ? k.wl : 1.0;
  // right side t in [0, delta] in units of h: [0, min(1/2, R)] from the
  // central cell, then [kc - 1/2, min(kc + 1/2, R)], kc = 1, 2, ...
  int64_t klast = 0;
  while ((double)(klast + 1) - 0.5 < R) ++klast;
  const int64_t S = 2 * klast + 1;
  std::vector<double> W(2 * S + 1, 0.0);
  for (int64_t kc = 0; kc <= klast; ++kc) {
    const double a = kc == 0 ? 0.0 : (double)kc - 0.5;
    const double b = std::min((double)kc + 0.5, R);
    // moments in s = tau - kc; quadratic through s = -1/2 (node), 0 (midpoint),
    // +1/2 (node): l_- = 2 s^2 - s, l_0 = 1 - 4 s^2, l_+ = 2 s^2 + s
    const double sa = a - (double)kc, sb = b - (double)kc;
    const double J0 = c * (sb - sa);
    const double J1 = c * (sb * sb - sa * sa) / 2.0;
    const double J2 = c * (sb * sb * sb - sa * sa * sa) / 3.0;
    const double Im = 2 * J2 - J1, I0 = J0 - 4 * J2, Ip = 2 * J2 + J1;
    W[S] += (wr + wl) * J0;
    if (kc == 0) {
      W[S] -= (wr + wl) * I0;
    } else {
      W[S + 2 * kc] -= wr * I0;
      W[S - 2 * kc] -= wl * I0;
    }
    W[S + 2 * kc - 1] -= wr * Im;
    W[S - 2 * kc + 1] -= wl * Im;
    W[S + 2 * kc + 1] -= wr * Ip;
    W[S - 2 * kc - 1] -= wl * Ip;
  }
  own_weight_from_row_sum(W, S);
  *Sout = S;
  return W;
}

namespace {

// node-row and midpoint-row stencils of the kernel's scheme
void both_stencils(const KernelSpec& k, int64_t N, std::vector<double>& Wn, int64_t& Sn,
                   std::vector<double>& Wm, int64_t& Sm) {
  if (k.kind == K_WEAKLY_SINGULAR) {
    ws_stencils(k.gamma, N, Wn, Wm, &Sn);
    Sm = Sn;
    return;
  }
  Wn = row_stencil(k, N, &Sn);
  if (k.scheme == SCHEME_STANDARD) {
    Wm = midpoint_stencil_standard(k, N, &Sm);
  } else {
    Wm = Wn;
    Sm = Sn;
  }
}

}  // namespace

void row_stencils(const KernelSpec& k, int64_t N, std::vector<double>& Wn, int64_t& Sn,
                  std::vector<double>& Wm, int64_t& Sm) {
  both_stencils(k, N, Wn, Sn, Wm, Sm);
}

bool row_stencils_reuse(const KernelSpec& k, int64_t N, std::vector<double>& Wn, int64_t& Sn,
                        std::vector<double>& Wm, int64_t& Sm) {
  if (k.kind != K_WEAKLY_SINGULAR && k.scheme != SCHEME_STANDARD) {
    row_stencil_into(k, N, Wn, &Sn);
    Sm = Sn;
    return true;
  }
  both_stencils(k, N, Wn, Sn, Wm, Sm);
  return false;
}

namespace {

// In-place power-of-two complex FFT (iterative radix 2), twiddles evaluated
// in long double; forward e^{-2 pi i jk/n}, inverse unnormalised.
void fft_pow2(std::vector<std::complex<double>>& a, bool inv) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<std::complex<double>> w;
  for (size_t len = 2; len <= n; len <<= 1) {
    const size_t half = len / 2;
    w.resize(half);
    for (size_t k = 0; k < half; ++k) {
      const long double ang = (inv ? 2.0L : -2.0L) * pi * (long double)k / (long double)len;
      w[k] = {(double)std::cos(ang), (double)std::sin(ang)};
    }
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < half; ++k) {
        const std::complex<double> u = a[i + k], v = a[i + k + half] * w[k];
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
  }
}

// out[m] = sum_{k=0..S} V[m + k] g[k] for m = 0..S (V has S+1 entries,
// zero beyond): a correlation, computed directly for a short reach and as a
// convolution with the reversed g through one complex FFT pair otherwise.
std::vector<double> correlate(const std::vector<double>& V, const double* g, int64_t S) {
  std::vector<double> out((size_t)S + 1, 0.0);
  if ((S + 1) * (S + 1) <= (int64_t(1) << 22)) {
    for (int64_t m = 0; m <= S; ++m) {
      double acc = 0.0;
      for (int64_t k = 0; k <= S && m + k < (int64_t)V.size(); ++k) acc += V[m + k] * g[k];
      out[m] = acc;
    }
    return out;
  }
  size_t n = 1;
  while (n < V.size() + (size_t)S + 1) n <<= 1;
  std::vector<std::complex<double>> x(n), y(n);
  for (size_t i = 0; i < V.size(); ++i) x[i] = V[i];
  for (int64_t i = 0; i <= S; ++i) y[(size_t)i] = g[S - i];  // reversed g
  fft_pow2(x, false);
  fft_pow2(y, false);
  for (size_t i = 0; i < n; ++i) x[i] *= y[i];
  fft_pow2(x, true);
  const double inv_n = 1.0 / (double)n;
  for (int64_t m = 0; m <= S; ++m) out[m] = x[(size_t)(m + S)].real() * inv_n;
  return out;
}

}  // namespace

int64_t volume_reach(const KernelSpec& k, int64_t N) {
  if (k.kind == K_WEAKLY_SINGULAR) return 0;  // the two boundary nodes only
  std::vector<double> Wn, Wm;
  int64_t Sn, Sm;
  both_stencils(k, N, Wn, Sn, Wm, Sm);
  return std::max(Sn, Sm);
}

void volume_correction(const KernelSpec& k, int64_t N, const double* gl, const double* gr,
                       double* b) {
  if (k.kind == K_WEAKLY_SINGULAR) {
    // Dirichlet data u(0) = gl[0], u(1) = gr[0]: b -= E g with E = -(K0 | K1)
    std::vector<double> K0((size_t)(2 * N - 1)), K1((size_t)(2 * N - 1));
    ws_boundary_coupling(k.gamma, N, K0.data(), K1.data());
    for (int64_t i = 0; i < 2 * N - 1; ++i) b[i] += K0[(size_t)i] * gl[0] + K1[(size_t)i] * gr[0];
    return;
  }
  std::vector<double> Wn, Wm;
  int64_t Sn, Sm;
  both_stencils(k, N, Wn, Sn, Wm, Sm);
  const int64_t S = std::max(Sn, Sm);
  const int64_t M = 2 * N - 1;
  // row at interleaved position p (1..M; even: node, odd: midpoint) couples
  // to the left exterior point -k with W(-(p + k)) and to the right one
  // 2N + k with W(2N + k - p); with m = p (left) or m = 2N - p (right) both
  // are sums over k of V[m + k] g[k], V[j] = W(-j) or W(+j).
  for (int side = 0; side < 2; ++side) {
    const double* g = side == 0 ? gl : gr;
    for (int type = 0; type < 2; ++type) {  // 0: node rows, 1: midpoint rows
      const std::vector<double>& W = type == 0 ? Wn : Wm;
      const int64_t Sw = type == 0 ? Sn : Sm;
      std::vector<double> V((size_t)S + 1, 0.0);
      for (int64_t j = 0; j <= Sw; ++j) V[(size_t)j] = W[(size_t)(Sw + (side == 0 ? -j : j))];
      const std::vector<double> corr = correlate(V, g, S);
      for (int64_t m = 1; m <= S; ++m) {
        const int64_t p = side == 0 ? m : 2 * N - m;
        if (p < 1 || p > M || (p % 2 == 0) != (type == 0)) continue;
        // block order: node i at x = i h -> index i - 1; midpoint (j - 1/2) h -> N - 1 + j - 1
        const int64_t idx = (p % 2 == 0) ? p / 2 - 1 : (N - 1) + (p + 1) / 2 - 1;
        b[idx] -= corr[(size_t)m];
      }
    }
  }
}

void shift_level(TpxLevel& t, double shift, double scale) {
  for (auto* v : {&t.a, &t.b, &t.c, &t.d, &t.p, &t.q, &t.xi, &t.zeta, &t.bsub, &t.bmain, &t.bsup})
    for (double& x : *v) x *= scale;
  t.o = t.o * scale + shift;
  t.a[t.n - 1] += shift;
  t.d[t.n - 1] += shift;
}

TpxLevel finest_level(const KernelSpec& k, int64_t N, int64_t near_cut) {
  TpxLevel t;
  const int64_t n = N - 1;
  t.n = n;
  t.a.resize(2 * n - 1);
  t.b.resize(2 * n - 1);
  t.c.resize(2 * n - 1);
  t.d.resize(2 * n - 1);
  t.p.resize(n);
  t.q.resize(n);
  t.xi.resize(n);
  t.zeta.resize(n);
  if (k.kind == K_GENERATORS) {
    // [A | B | C | D] with the layouts of the C ABI.
    const double* gA = k.gen;
    const double* gB = gA + (2 * n - 1);
    const double* gC = gB + 2 * n;
    const double* gD = gC + 2 * n;
    auto B = [&](int64_t off) { return gB[off + n - 1]; };  // -(n-1)..n
    auto C = [&](int64_t off) { return gC[off + n]; };      // -n..n-1
    auto D = [&](int64_t off) { return gD[off + n]; };      // -n..n
    for (int64_t dd = -(n - 1); dd <= n - 1; ++dd) {
      t.a[dd + n - 1] = gA[dd + n - 1];
      t.b[dd + n - 1] = B(dd + 1);   // B_bar = B[:, 1:]
      t.c[dd + n - 1] = C(dd - 1);   // C_bar = C[1:, :]
      t.d[dd + n - 1] = D(dd);       // D_bar = D[1:, 1:]
    }
    for (int64_t i = 0; i < n; ++i) {
      t.p[i] = B(-i);        // B[:, 0]
      t.q[i] = C(i);         // C[0, :]
      t.xi[i] = D(-i - 1);   // D[1:, 0]
      t.zeta[i] = D(i + 1);  // D[0, 1:]
    }
    t.o = D(0);
    return t;
  }
  std::vector<double> Wn, Wm;
  int64_t Sn = 0, Sm = 0;
  both_stencils(k, N, Wn, Sn, Wm, Sm);
  auto node = [&](int64_t s2) {
    return (s2 < -Sn || s2 > Sn || (s2 >= -near_cut && s2 <= near_cut)) ? 0.0 : Wn[s2 + Sn];
  };
  auto mid = [&](int64_t s2) {
    return (s2 < -Sm || s2 > Sm || (s2 >= -near_cut && s2 <= near_cut)) ? 0.0 : Wm[s2 + Sm];
  };
  // Interleaved positions: v_i at 2(i+1), w_o at 1, w_bar_j at 2j+3 (units h/2).
  // Node rows: A, B_bar, p; midpoint rows: C_bar, D_bar, q, xi, zeta, o.
  for (int64_t dd = -(n - 1); dd <= n - 1; ++dd) {
    t.a[dd + n - 1] = node(2 * dd);
    t.b[dd + n - 1] = node(2 * dd + 1);
    t.c[dd + n - 1] = mid(2 * dd - 1);
    t.d[dd + n - 1] = mid(2 * dd);
  }
  for (int64_t i = 0; i < n; ++i) {
    t.p[i] = node(-2 * i - 1);
    t.q[i] = mid(2 * i + 1);
    t.xi[i] = mid(-2 * i - 2);
    t.zeta[i] = mid(2 * i + 2);
  }
  t.o = mid(0);
  if (k.kind == K_WEAKLY_SINGULAR) {
    // variable diagonal int_0^1 |x - y|^-gamma dy at the collocation points
    const int64_t m = 2 * n + 1;
    t.bsub.assign((size_t)m, 0.0);
    t.bsup.assign((size_t)m, 0.0);
    t.bmain.resize((size_t)m);
    for (int64_t idx = 0; idx < m; ++idx) {
      const double x = (idx < n) ? (double)(idx + 1) / (double)N
                                 : ((double)(idx - n) + 0.5) / (double)N;
      t.bmain[(size_t)idx] =
          (std::pow(x, 1 - k.gamma) + std::pow(1 - x, 1 - k.gamma)) / (1 - k.gamma);
    }
  }
  return t;
}

void near_field(const KernelSpec& k, int64_t N, int M, double shift, double scale,
                NearField& nf) {
  std::vector<double> Wn, Wm;
  int64_t Sn = 0, Sm = 0;
  both_stencils(k, N, Wn, Sn, Wm, Sm);
  auto at = [](const std::vector<double>& W, int64_t S, int64_t s2) {
    return (s2 < -S || s2 > S) ? 0.0 : W[s2 + S];
  };
  nf.M = M;
  nf.wn.assign(2 * M + 1, 0.0);
  nf.wm.assign(2 * M + 1, 0.0);
  for (int kk = -M; kk <= M; ++kk) {
    nf.wn[kk + M] = kk == 0 ? 0.0 : scale * at(Wn, Sn, kk);
    nf.wm[kk + M] = kk == 0 ? 0.0 : scale * at(Wm, Sm, kk);
  }
  // The own-point weight int gamma (1 - l_0) equals -sum_{k != 0} W(k) (the
  // quadratic basis is a partition of unity on every cell), so a row's near
  // sum R_s = W(0) + sum_{0<|k|<=M, in range} W(k) is minus the stencil's
  // weight beyond M half-steps and minus its near weight outside 1..2N-1:
  // small numbers, summed in long double, free of the rounding of W(0).
  long double far[2] = {0.0L, 0.0L};
  for (int t = 0; t < 2; ++t) {
    const std::vector<double>& W = t == 0 ? Wn : Wm;
    const int64_t S = t == 0 ? Sn : Sm;
    for (int64_t s2 = -S; s2 <= S; ++s2)
      if (s2 < -M || s2 > M) far[t] += (long double)W[s2 + S];
  }
  const int64_t last = 2 * N - 1;
  auto rsum = [&](int64_t s) {
    const int t = (s % 2 == 0) ? 0 : 1;
    const std::vector<double>& W = t == 0 ? Wn : Wm;
    const int64_t S = t == 0 ? Sn : Sm;
    long double acc = -far[t];
    for (int kk = -M; kk <= M; ++kk)
      if (kk != 0 && (s + kk < 1 || s + kk > last)) acc -= (long double)at(W, S, kk);
    return (double)(acc * (long double)scale + (long double)shift);
  };
  nf.rsum_left.resize(M);
  nf.rsum_right.resize(M);
  for (int64_t s = 1; s <= M; ++s) nf.rsum_left[s - 1] = rsum(s);
  for (int64_t s = last - M + 1; s <= last; ++s) nf.rsum_right[s - (last - M + 1)] = rsum(s);
  for (int t = 0; t < 2; ++t)
    nf.rsum_in[t] = (double)(-far[t] * (long double)scale + (long double)shift);
}

TpxLevel coarsen(const TpxLevel& f) {
  // Galerkin R A P with R = 1/4[1 2 1] (stride 2) on [v; w_o; w_bar] and
  // P = 2 R^T.  The v/w_bar blocks only see the fine Toeplitz blocks, giving
  // t'_i = (t_{2i-2} + 4t_{2i-1} + 6t_{2i} + 4t_{2i+1} + t_{2i+2}) / 8.
  // The coarse w_o column is R (A z) with z = P e_{w_o} = 1/2 e_{v,n-1} +
  // e_{w_o} + 1/2 e_{w_bar,0}; the coarse w_o row is (rho^T A) P with
  // rho = 1/4 e_{v,n-1} + 1/2 e_{w_o} + 1/4 e_{w_bar,0} (Lemma 3.1).
  const int64_t n = f.n, nc = (n - 1) / 2;
  auto g = [n](const std::vector<double>& t, int64_t off) { return t[off + n - 1]; };
  TpxLevel c;
  c.n = nc;
  for (auto* v : {&c.a, &c.b, &c.c, &c.d}) v->assign(2 * nc - 1, 0.0);
  const std::vector<double>* fine[4] = {&f.a, &f.b, &f.c, &f.d};
  std::vector<double>* coarse[4] = {&c.a, &c.b, &c.c, &c.d};
  for (int blk = 0; blk < 4; ++blk) {
    const auto& t = *fine[blk];
    for (int64_t i = -(nc - 1); i <= nc - 1; ++i) {
      (*coarse[blk])[i + nc - 1] = (g(t, 2 * i - 2) + 4 * g(t, 2 * i - 1) + 6 * g(t, 2 * i) +
                                    4 * g(t, 2 * i + 1) + g(t, 2 * i + 2)) / 8.0;
    }
  }
  std::vector<double> colv(n), colw(n), rowv(n), roww(n);
  for (int64_t i = 0; i < n; ++i) {
    colv[i] = 0.5 * g(f.a, n - 1 - i) + f.p[i] + 0.5 * g(f.b, -i);
    colw[i] = 0.5 * g(f.c, n - 1 - i) + f.xi[i] + 0.5 * g(f.d, -i);
    rowv[i] = 0.25 * g(f.a, i - n + 1) + 0.5 * f.q[i] + 0.25 * g(f.c, i);
    roww[i] = 0.25 * g(f.b, i - n + 1) + 0.5 * f.zeta[i] + 0.25 * g(f.d, i);
  }
  const double colo = 0.5 * f.q[n - 1] + f.o + 0.5 * f.zeta[0];
  auto R = [](const std::vector<double>& x, int64_t i) {
    return 0.25 * (x[2 * i] + 2 * x[2 * i + 1] + x[2 * i + 2]);
  };
  c.p.resize(nc);
  c.xi.resize(nc);
  c.q.resize(nc);
  c.zeta.resize(nc);
  for (int64_t i = 0; i < nc; ++i) {
    c.p[i] = R(colv, i);
    c.xi[i] = R(colw, i);
    c.q[i] = 2.0 * R(rowv, i);
    c.zeta[i] = 2.0 * R(roww, i);
  }
  c.o = 0.25 * colv[n - 1] + 0.5 * colo + 0.25 * colw[0];
  if (f.has_band()) {
    // R B P of the tridiagonal part: c[i][j] = sum_{e,f} w_e B[2i+e][2j+f] 2 w_f,
    // w = (1/4, 1/2, 1/4); tridiagonal again
    const int64_t m = 2 * n + 1, mc = n;
    const double w[3] = {0.25, 0.5, 0.25};
    auto Bat = [&](int64_t i, int64_t j) {
      if (j == i) return f.bmain[(size_t)i];
      if (j == i - 1) return f.bsub[(size_t)i];
      if (j == i + 1) return f.bsup[(size_t)i];
      return 0.0;
    };
    c.bsub.assign((size_t)mc, 0.0);
    c.bmain.assign((size_t)mc, 0.0);
    c.bsup.assign((size_t)mc, 0.0);
    for (int64_t i = 0; i < mc; ++i)
      for (int64_t jd = -1; jd <= 1; ++jd) {
        const int64_t j = i + jd;
        if (j < 0 || j >= mc) continue;
        double acc = 0.0;
        for (int e = 0; e < 3; ++e)
          for (int ff = 0; ff < 3; ++ff) {
            const int64_t r = 2 * i + e, q = 2 * j + ff;
            if (r < m && q < m) acc += w[e] * Bat(r, q) * 2.0 * w[ff];
          }
        (jd < 0 ? c.bsub : (jd == 0 ? c.bmain : c.bsup))[(size_t)i] = acc;
      }
  }
  if (f.symmetric()) {
    // The Galerkin image of a symmetric level is symmetric, but the
    // recurrences above give mirror entries that agree only up to rounding.
    // Averaging them keeps every coarse level exactly symmetric, so it keeps
    // the compact real spectra and the SPD kernels on the device.
    const int64_t m = 2 * nc - 1;
    std::vector<double> a(m), b(m);
    for (int64_t i = 0; i < m; ++i) {
      a[i] = 0.5 * (c.a[i] + c.a[m - 1 - i]);
      b[i] = 0.5 * (c.b[i] + c.c[m - 1 - i]);
    }
    c.a = a;
    c.d = a;
    c.b = b;
    for (int64_t i = 0; i < m; ++i) c.c[i] = b[m - 1 - i];
    for (int64_t i = 0; i < nc; ++i) {
      c.p[i] = c.q[i] = 0.5 * (c.p[i] + c.q[i]);
      c.xi[i] = c.zeta[i] = 0.5 * (c.xi[i] + c.zeta[i]);
    }
  }
  return c;
}

std::vector<double> densify(const TpxLevel& t) {
  const int64_t n = t.n, m = 2 * n + 1;
  std::vector<double> M(m * m, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      const int64_t off = j - i + n - 1;
      M[i * m + j] = t.a[off];
      M[i * m + (n + 1 + j)] = t.b[off];
      M[(n + 1 + i) * m + j] = t.c[off];
      M[(n + 1 + i) * m + (n + 1 + j)] = t.d[off];
    }
    M[i * m + n] = t.p[i];
    M[n * m + i] = t.q[i];
    M[(n + 1 + i) * m + n] = t.xi[i];
    M[n * m + (n + 1 + i)] = t.zeta[i];
  }
  M[n * m + n] = t.o;
  if (t.has_band())
    for (int64_t i = 0; i < m; ++i) {
      M[i * m + i] += t.bmain[(size_t)i];
      if (i > 0) M[i * m + i - 1] += t.bsub[(size_t)i];
      if (i + 1 < m) M[i * m + i + 1] += t.bsup[(size_t)i];
    }
  return M;
}

bool lu_factor(std::vector<double>& A, int m, std::vector<int>& piv) {
  piv.assign(m, 0);
  for (int k = 0; k < m; ++k) {
    int pr = k;
    double best = std::fabs(A[k * m + k]);
    for (int i = k + 1; i < m; ++i)
      if (std::fabs(A[i * m + k]) > best) best = std::fabs(A[i * m + k]), pr = i;
    piv[k] = pr;
    if (best == 0.0) return false;
    if (pr != k)
      for (int j = 0; j < m; ++j) std::swap(A[k * m + j], A[pr * m + j]);
    const double inv = 1.0 / A[k * m + k];
    for (int i = k + 1; i < m; ++i) {
      const double l = A[i * m + k] * inv;
      A[i * m + k] = l;
      for (int j = k + 1; j < m; ++j) A[i * m + j] -= l * A[k * m + j];
    }
  }
  return true;
}

void lu_inverse(const std::vector<double>& LU, int m, const std::vector<int>& piv,
                std::vector<double>& inv) {
  inv.assign((size_t)m * m, 0.0);
  std::vector<double> x(m);
  for (int col = 0; col < m; ++col) {
    std::fill(x.begin(), x.end(), 0.0);
    x[col] = 1.0;
    for (int k = 0; k < m; ++k) std::swap(x[k], x[piv[k]]);  // P e_col
    for (int i = 0; i < m; ++i)                               // L y = P e
      for (int k = 0; k < i; ++k) x[i] -= LU[(size_t)i * m + k] * x[k];
    for (int i = m - 1; i >= 0; --i) {                        // U x = y
      for (int k = i + 1; k < m; ++k) x[i] -= LU[(size_t)i * m + k] * x[k];
      x[i] /= LU[(size_t)i * m + i];
    }
    for (int i = 0; i < m; ++i) inv[(size_t)col * m + i] = x[i];
  }
}

void manufactured_rhs(const KernelSpec& k, int64_t N, double* out) {
  // f(x) = int_{|t|<=delta} gamma(t) (u(x) - u~(x+t)) dt, u = x^2 (1-x)^2 on
  // (0,1), u~ = 0 outside.  Constant/weighted kernels: antiderivative
  // U(y) = y^3/3 - y^4/2 + y^5/5.  Fractional kernel: Taylor expansion of u
  // about x (exact, degree 4) where x + t stays in (0,1), u(x) times the
  // kernel mass where it leaves.
  const double d = k.delta, c = kernel_c(k);
  const double wl = (k.kind == K_WEIGHTED) ? k.wl : 1.0;
  const double wr = (k.kind == K_WEIGHTED) ? k.wr : 1.0;
  auto u = [](double x) { return x * x * (1 - x) * (1 - x); };
  auto U = [](double y) { return y * y * y * (1.0 / 3 - y / 2 + y * y / 5); };
  const int64_t m = 2 * N - 1;
  for (int64_t idx = 0; idx < m; ++idx) {
    const double x = (idx < N - 1) ? (double)(idx + 1) / (double)N
                                   : ((double)(idx - (N - 1)) + 0.5) / (double)N;
    const double ux = u(x);
    double f;
    if (!is_fractional(k.kind)) {
      const double right = ux * d - (U(std::fmin(x + d, 1.0)) - U(x));
      const double left = ux * d - (U(x) - U(std::fmax(x - d, 0.0)));
      f = c * (wr * right + wl * left);
    } else {
      const double be = -1.0 - 2.0 * k.alpha;
      const double tr = std::fmin(d, 1.0 - x), tl = std::fmin(d, x);
      const double du[4] = {2 * x - 6 * x * x + 4 * x * x * x, 2 - 12 * x + 12 * x * x,
                            -12 + 24 * x, 24.0};
      const double fact[4] = {1, 2, 6, 24};
      f = 0.0;
      for (int p = 1; p <= 4; ++p) {
        // int_{-tl}^{tr} t^p |t|^be dt (a principal value for p = 1 when
        // be + 2 <= 0, the near-field kernel; log(tr/tl) at be + 2 = 0)
        const double e = be + p + 1;
        const double sgn = (p % 2) ? -1.0 : 1.0;
        const double Mp = (e == 0.0) ? std::log(tr / tl)
                                     : (std::pow(tr, e) + sgn * std::pow(tl, e)) / e;
        f -= du[p - 1] / fact[p - 1] * Mp;
      }
      for (double a : {1.0 - x, x})
        if (a < d) f += ux * (std::pow(d, be + 1) - std::pow(a, be + 1)) / (be + 1);
      f *= c;
    }
    out[idx] = f;
  }
}

std::vector<double> twiddles(int64_t M, int64_t count, int64_t stride) {
  std::vector<double> t(2 * count);
  const long double two_pi = 2.0L * acosl(-1.0L);
  for (int64_t m = 0; m < count; ++m) {
    const int64_t e = (m * stride) % M;
    const long double ang = two_pi * (long double)e / (long double)M;
    t[2 * m] = (double)cosl(ang);
    t[2 * m + 1] = (double)(-sinl(ang));
  }
  return t;
}

}  // namespace amg
