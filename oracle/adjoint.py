"""Adjoint sensitivity of an effective-stiffness objective, FP64.  TEST
INFRASTRUCTURE ONLY.

For macroscopic tensor strains A and B (Voigt tensor components), the
objective is J = A : C_eff : B = A : <sigma[B]>, where sigma[B] is the stress of
the converged fixed point of Sec. 5.2 under Ebar = B.  BASIC, FB and AFB solve
a variational problem: the fixed point minimises <(Ebar + eps~) : C : (Ebar +
eps~)> over the compatible fluctuations eps~ of the scheme, the discrete
gradient and divergence being adjoint (q^b the conjugate of q^a up to the
scalar phase of AFB).  Hence J = <eps[A] : C : eps[B]> and, by the envelope
property of a minimum, its derivative with respect to the moduli of voxel x
is the partial derivative at the solution:
    dJ/dlambda(x) = tr eps[A] tr eps[B] / N,   dJ/dmu(x) = 2 eps[A] : eps[B] / N.
At fixed Poisson ratio, lambda and mu scale with E, so
    dJ/dE(x) = (lambda dJ/dlambda + mu dJ/dmu) / E.
The adjoint field of the load A is the primal solution under A.

The DGO of Sec. 5.4 (D3, polarisation form eps = Ebar + G (C - C_H) eps with
G = F^{c+} Gamma^c F^{c-}) is not derived from an energy, but G is
self-adjoint: Gamma^c is a real symmetric 6 x 6 per frequency (Mandel
metric; sums of Gamma_H) and even in xi (symmetric image window), and it
annihilates uniform fields (Gamma^c_0 = 0).  Differentiating eps[B] and
solving the adjoint equation w - dC G w = C A (dC = C - C_H) gives
dJ = <(A + G w) : dC : eps[B]>, and A + G w solves the primal equation under
A: so the same formula holds with the DGO's own eps[A], eps[B].
"""
from __future__ import annotations

import numpy as np

from . import solve3d

W = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])   # Voigt weights of a double contraction


def contract(a, b):
    """a : b for Voigt tensor-component arrays (leading axis 6)."""
    return np.tensordot(W, np.asarray(a) * np.asarray(b), axes=(0, 0))


def objective(lam, mu, A, B, lam0, mu0, scheme="AFB", tol=1e-12, maxit=5000, Gc=None):
    """(J, eps[A], eps[B]) with J = A : <sigma[B]>.  scheme="DGO" iterates D3
    with the discrete Green operator Gc (green.dgo_voigt)."""
    def solve(Eb):
        if scheme == "DGO":
            return solve3d.solve_dgo(lam, mu, Eb, lam0, mu0, Gc, tol=tol, maxit=maxit)
        return solve3d.solve_gfp(lam, mu, Eb, lam0, mu0, scheme=scheme, tol=tol, maxit=maxit)
    rb = solve(B)
    ra = rb if np.array_equal(np.asarray(A), np.asarray(B)) else solve(A)
    return float(contract(A, rb.sig_mean)), ra.eps, rb.eps


def modulus_gradient(lam, mu, eps_a, eps_b):
    """(dJ/dlambda, dJ/dmu, dJ/dE) per voxel, each shaped like lam."""
    N = lam.size
    tra = eps_a[0] + eps_a[1] + eps_a[2]
    trb = eps_b[0] + eps_b[1] + eps_b[2]
    gl = tra * trb / N
    gm = 2.0 * contract(eps_a, eps_b) / N
    E = mu * (3.0 * lam + 2.0 * mu) / (lam + mu)
    return gl, gm, (lam * gl + mu * gm) / E
