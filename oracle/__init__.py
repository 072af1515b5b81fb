"""CPU oracle for the Green-function-preconditioned fixed-point solvers.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 numpy
implementation of what the paper's algorithms compute, written to be checked
against the paper by eye.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the GPU library never does, and
the two share no code.

Modules
-------
fourier   TD / PCD discrete Fourier transforms (Sec. 3.1 eqs. (9)-(10),
          Sec. 3.2 eqs. (20)-(21), Sec. 5.2 eq. (31), Sec. 5.4 eq. (47)),
          plus a brute-force DFT used as a pin.
fdd       effective wavenumbers of the finite-difference discretisations
          (Sec. 3.1 eqs. (12)-(14), (18); Sec. 5.3 eqs. (36)-(45)).
green     the Green-function inverse of Sec. 5.2 eq. (34), the isotropic
          Green tensor and Lippmann-Schwinger operator of Sec. 5.4 eq. (48),
          and the discrete Green operator (DGO) image sum of Sec. 5.4.
solve3d   the 3D fixed-point algorithms (Sec. 5.2 TD, Sec. 5.4 PCD and DGO).
solve1d   the 1D algorithms of Sec. 3 and the analytic solution of Sec. 2.1.
bounds    laminate closed form, Voigt / Reuss / Hashin-Shtrikman bounds,
          effective stiffness assembly.
direct    independent routes to the same discrete solution: dense LU for
          tiny grids and preconditioned conjugate gradients.

Parity status of each function is stated in its docstring; everything here is
pinned by the `-m "not gpu"` tests except where a docstring says
"parity unpinned".
"""
