"""CPU FP64 oracle for the fast block-structured AMG of Chen, Cao and
Serra-Capizzano (arXiv 2202.11288).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP/C++ library (``paper_2202_11288_amd``), and neither imports the other.

Contents (each function cites the passage of the paper it follows):

* ``discretize`` -- product-integration weights of the piecewise-quadratic
  collocation (Sec. 2.2, shifted-symmetric form eq. (system1)), the dense
  (2N-1)x(2N-1) block system assembled row by row, the manufactured
  right-hand side.
* ``dense`` -- simple restriction/prolongation (Sec. 3.1), dense Galerkin
  coarse operators (eq. (5 Galerkin) / (block Galerkin)), damped Jacobi
  (eq. (7 Jacobi)), the block V-cycle (Algorithm 2), the stationary outer
  iteration with the stopping rule of Sec. 5, the two-grid error operator
  (Theorem 4.1).
* ``tpx`` -- the Toeplitz-like-plus-Cross representation (eq. (split01)),
  Lemma 3.1's coarse recurrences, circulant-embedded FFT matvecs (Sec. 3.2,
  eq. (ccs3.4)), and the same V-cycle / outer iteration on that representation
  for large N.

Every floating-point computation here is FP64.  Parity status per function is
stated in its docstring; functions without an independent pin say
"parity unpinned".
"""
