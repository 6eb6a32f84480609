"""CPU FP64 oracle for the filtered-AIM 2D EFIE (test infrastructure).

This package is test infrastructure.  Only the tests, the smoke check of the
package entry file and the CPU-baseline leg of the benchmark may import it.
It shares no code with the HIP library: every function here is written from
the paper's definitions (Sec. II eqs. (1)-(6), Sec. III eqs. (7)-(10) and the
self-term rule of Sec. III-C) and from textbook closed forms, in plain NumPy /
SciPy double precision.

Modules
  geometry   segments, tangents, normals, Gauss-Legendre nodes (Sec. II, eq. (7))
  green      g = -j/4 H0^(2)(kR) (Sec. II), its log/regular split, the
             analytically filtered kernel g^alpha of eq. (6) in two forms
  galerkin   dense Galerkin S (eq. (4)), N (eq. (2), Maue form), Gram G
  aim        grid, anterpolation weights, grid kernel, numerical filter,
             near-field correction and the AIM operators of eqs. (8) and (10)
             applied by direct (non-FFT) sums over active grid points
  mie        circle eigenvalues and Mie-series currents / RCS (closed forms)
  solver     restarted GMRES and mixed-precision iterative refinement
  excitation plane-wave right-hand sides (Sec. II) and monostatic RCS

Parity status of each function is stated in its module header.
"""
