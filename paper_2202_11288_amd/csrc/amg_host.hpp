// Host-side (CPU, FP64) numerics of the library: finest-level generators by
// product integration, Galerkin coarsening of Toeplitz-plus-Cross levels,
// coarsest LU, twiddle tables.  Internal header (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace amg {

enum KernelKind { K_CONST = 0, K_WEIGHTED = 1, K_FRACTIONAL = 2, K_GENERATORS = 3,
                  K_WEAKLY_SINGULAR = 4, K_FRACTIONAL_NEAR = 5 };

// c |s|^(-1-2 alpha): product integration throughout (0 < alpha < 1/2), or
// with the symmetric near-field rule on |t| <= h/2 (0 < alpha < 1)
inline bool is_fractional(int kind) { return kind == K_FRACTIONAL || kind == K_FRACTIONAL_NEAR; }

enum Scheme { SCHEME_SHIFTED = 0, SCHEME_STANDARD = 1 };

struct KernelSpec {
  int kind = K_CONST;
  double delta = 0.25;
  double alpha = 0.0;
  double wl = 1.0, wr = 1.0;
  const double* gen = nullptr;
  int scheme = SCHEME_SHIFTED;
  double gamma = 0.0;  // K_WEAKLY_SINGULAR: |x - y|^-gamma on (0, 1)
  // the standard rule is set up for the constant and weighted kernels
  bool supported() const { return !(scheme == SCHEME_STANDARD && is_fractional(kind)); }
};

// One level in the Toeplitz-like-plus-Cross form (eq. (split01)):
// n x n Toeplitz blocks A, B_bar, C_bar, D_bar with T[i][j] = t[j-i+n-1],
// Cross vectors p, q, xi, zeta (length n) and the scalar o.
struct TpxLevel {
  int64_t n = 0;
  std::vector<double> a, b, c, d;
  std::vector<double> p, q, xi, zeta;
  double o = 0.0;
  // Optional tridiagonal part on the block-ordered vector (empty: none):
  // bsub[i] couples i to i-1, bmain[i] to i, bsup[i] to i+1 (bsub[0] =
  // bsup[2n] = 0).  The variable diagonal of the weakly singular model
  // (eq. (3system)) at the finest level; its Galerkin images below.
  std::vector<double> bsub, bmain, bsup;
  bool has_band() const { return !bmain.empty(); }
  // true when A = D_bar symmetric and C_bar = B_bar^T exactly (and no band):
  // the packed spectra are then real / imaginary and stored compactly.
  bool symmetric() const;
};

// Validation of the public arguments; returns an empty string when valid.
std::string validate(const KernelSpec& k, int64_t N, int coarsest_log2);

// Row stencil W[s2 + S], s2 in [-S, S], in half-grid offsets (shifted-symmetric
// collocation: every row has this stencil).
std::vector<double> row_stencil(const KernelSpec& k, int64_t N, int64_t* S);

// Midpoint-row stencil of the standard collocation (eq. (ccs2.6)): the row at
// a midpoint integrates over the mesh cells [(k-1/2)h, (k+1/2)h] around it,
// the central one holding the point as its midpoint, the last one cut at the
// horizon.  W[s2 + S], s2 in [-S, S] (odd s2: nodes, even: midpoints).
std::vector<double> midpoint_stencil_standard(const KernelSpec& k, int64_t N, int64_t* S);

// Weakly singular model (eq. (3system), kernel |x - y|^-gamma on (0, 1)):
// node- and midpoint-row stencils W[s2 + S] = -h^(1-gamma) * product-
// integration weight of the unknown at half-step offset s2 (S = 2N); the
// couplings K0, K1 (2N-1 each, block order) of the boundary nodes x = 0, 1.
void ws_stencils(double gamma, int64_t N, std::vector<double>& Wn, std::vector<double>& Wm,
                 int64_t* S);
void ws_boundary_coupling(double gamma, int64_t N, double* K0, double* K1);

// Node-row and midpoint-row stencils of the kernel's collocation scheme
// (equal under the shifted-symmetric rule); W[s2 + S], s2 in [-S, S].
void row_stencils(const KernelSpec& k, int64_t N, std::vector<double>& Wn, int64_t& Sn,
                  std::vector<double>& Wm, int64_t& Sm);
// The same into vectors whose storage is reused (no fresh pages for a
// caller that keeps them); returns true when the midpoint-row stencil equals
// the node-row one (shifted-symmetric rule), in which case Wm is untouched.
bool row_stencils_reuse(const KernelSpec& k, int64_t N, std::vector<double>& Wn, int64_t& Sn,
                        std::vector<double>& Wm, int64_t& Sm);
// Row stencil into W (its storage reused).
void row_stencil_into(const KernelSpec& k, int64_t N, std::vector<double>& W, int64_t* S);

// Reach S (half-grid steps) of the node- and midpoint-row stencils.
int64_t volume_reach(const KernelSpec& k, int64_t N);

// b -= E g for the volume data g_left[k] = g(-k h/2), g_right[k] = g(1 + k h/2),
// k = 0..S (block-ordered b).  Direct sums for a short reach, FFT convolution
// beyond.
void volume_correction(const KernelSpec& k, int64_t N, const double* g_left,
                       const double* g_right, double* b);

// t <- shift*I + scale*t (generators and Cross data times scale, shift on
// the diagonal entries a_0, d_0 and o).
void shift_level(TpxLevel& t, double shift, double scale);

// Finest level from the kernel stencil or from caller generators.
// near_cut >= 0 (stencil kernels only): the stencil entries at half-step
// offsets |s2| <= near_cut are left out (the far field of the split residual
// below).
TpxLevel finest_level(const KernelSpec& k, int64_t N, int64_t near_cut = -1);

// Near field of the finest level for the split evaluation of A x (stencil
// kernels).  In the interleaved order of the collocation points (position s
// = 1..2N-1 in units of h/2: nodes at even s, midpoints at odd s) row s of
// the finest matrix is the row stencil of its point type, W(s' - s), cut to
// the columns 1..2N-1 (eq. (ccs2.6); under the shifted rule both types share
// one stencil).  With the near offsets |k| <= M applied in difference form,
//   (A x)_s = sum_{0<|k|<=M} W(k) (x_{s+k} - x_s) + R_s x_s + far_s(x),
//   R_s = sum_{|k|<=M, 1<=s+k<=2N-1} W(k)   (+ shift),
// the products that cancel in a smooth x meet only differences of
// neighbouring values, and the far field (all |k| > M) is a Toeplitz-plus-
// Cross level of small entries.  The own-point weight W(0) = int gamma
// (1 - l_0) is taken as -sum_{k != 0} W(k) (the basis is a partition of
// unity), so R_s = -(stencil weight beyond M) - (near weight outside
// 1..2N-1), summed in long double without the rounding of W(0).
// w[k + M] = scale * W(k) per row type (w[M] = 0); rsum_left[s-1] (s =
// 1..M), rsum_right[s-(2N-M)] (s = 2N-M..2N-1) and rsum_in[type] (every
// other s) hold scale * R_s + shift.
struct NearField {
  int M = 0;
  std::vector<double> wn, wm;            // node rows, midpoint rows (2M+1 each)
  std::vector<double> rsum_left, rsum_right;
  double rsum_in[2] = {0.0, 0.0};        // [0] node rows, [1] midpoint rows
};
void near_field(const KernelSpec& k, int64_t N, int M, double shift, double scale, NearField& nf);

// Galerkin coarse level R A P (Lemma 3.1), O(n).
TpxLevel coarsen(const TpxLevel& f);

// Dense (2n+1)^2 matrix of a level, row-major.
std::vector<double> densify(const TpxLevel& t);

// LU with partial pivoting, in place (row-major m x m); piv[i] = row swapped
// with i at step i.  Returns false if a zero pivot is met.
bool lu_factor(std::vector<double>& A, int m, std::vector<int>& piv);

// Inverse from the factors of lu_factor: inv (column-major m x m) solves
// A inv = I column by column (P, unit-lower L, upper U).
void lu_inverse(const std::vector<double>& LU, int m, const std::vector<int>& piv,
                std::vector<double>& inv);

// Manufactured right-hand side f(x_c) for u = x^2 (1-x)^2, block order.
void manufactured_rhs(const KernelSpec& k, int64_t N, double* b);

// Twiddle e^{-2 pi i m / M} for m = 0..count-1 (interleaved re, im), computed
// in long double and rounded once.
std::vector<double> twiddles(int64_t M, int64_t count, int64_t stride = 1);

}  // namespace amg
