"""Effective stiffness as a differentiable function of the Young's modulus field.

`effective_stiffness(E, nu, A, B, ...)` returns J = A : C_eff : B for the
periodic cell with per-voxel Young's modulus E (a torch tensor shaped
(n3, n2, n1)) and uniform Poisson ratio nu, and back-propagates dJ/dE(x)
through the adjoint of the fixed point: BASIC, FB and AFB are self-adjoint
(the fixed point minimises a quadratic energy), and so is the DGO of Sec. 5.4
(its Green map is a real symmetric, even operator that annihilates uniform
fields), so the adjoint field of the load A is the primal solution under A and
the gradient is the pointwise product computed by lsfft_stiffness_gradient.
Every solve and the gradient run in the HIP library; this module marshals
arguments and holds the handles.
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs, lsfft

_W = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])


class _EffectiveStiffness(torch.autograd.Function):
    @staticmethod
    def forward(ctx, young, nu, A, B, lambda0, mu0, scheme, prec, tol, maxit, f64_warmup, dgo):
        E = young.detach().to("cpu", torch.float64).numpy()
        lam, mu = inputs.lame_from_young(E, nu)
        if lambda0 is None or mu0 is None:
            # reference medium: mean of the Lame moduli of the extreme Young's
            # moduli.  The converged BASIC / FB / AFB solution does not depend
            # on C0, so letting it follow E changes no derivative; the DGO's
            # does, and there the caller fixes C0 (checked in the wrapper).
            l_lo, m_lo = inputs.lame_from_young(E.min(), nu)
            l_hi, m_hi = inputs.lame_from_young(E.max(), nu)
            lambda0, mu0 = 0.5 * (float(l_lo) + float(l_hi)), 0.5 * (float(m_lo) + float(m_hi))
        extra = {"disc": "pcd", "dgo_images": dgo[0], "dgo_weight_power": dgo[1]} if scheme.lower() == "dgo" else {}
        s = lsfft.Solver(lam, mu, lambda0, mu0, scheme=scheme, prec=prec, f64_warmup=f64_warmup, **extra)
        dt = torch.float32 if prec == "f32" else torch.float64
        shape = (6,) + tuple(E.shape)
        eps_b = torch.empty(shape, dtype=dt, device="cuda")
        rb = s.solve_device(B, tol=tol, maxit=maxit, eps_dev=eps_b)
        if rb["status"] < 0 or rb["status"] == lsfft.EDIVERGED:
            s.close()
            raise lsfft.LsfftError(rb["status"], "effective_stiffness (load B)")
        if np.array_equal(A, B):
            eps_a, ra = eps_b, rb
        else:
            eps_a = torch.empty(shape, dtype=dt, device="cuda")
            ra = s.solve_device(A, tol=tol, maxit=maxit, eps_dev=eps_a)
            if ra["status"] < 0 or ra["status"] == lsfft.EDIVERGED:
                s.close()
                raise lsfft.LsfftError(ra["status"], "effective_stiffness (load A)")
        ctx.solver = s
        ctx.eps = (eps_a, eps_b)
        ctx.young_meta = (young.dtype, young.device)
        ctx.info = {"iters": (ra["iters"], rb["iters"]), "residual": (ra["residual"], rb["residual"]),
                    "status": (ra["status"], rb["status"])}
        J = float(np.dot(_W * A, rb["sig_mean"]))
        return torch.tensor(J, dtype=torch.float64, device=young.device)

    @staticmethod
    def backward(ctx, gJ):
        s = ctx.solver
        eps_a, eps_b = ctx.eps
        de = torch.empty(eps_a.shape[1:], dtype=eps_a.dtype, device="cuda")
        lsfft.stiffness_gradient(s.handle, eps_a, eps_b, dj_dyoung=de)
        s.close()
        ctx.eps = None
        dtype, device = ctx.young_meta
        grad = gJ.to(device=device, dtype=torch.float64) * de.to(device=device, dtype=torch.float64)
        return grad.to(dtype), None, None, None, None, None, None, None, None, None, None, None


def effective_stiffness(young, nu, A, B=None, lambda0=None, mu0=None, scheme="afb", prec="f64", tol=1e-8,
                        maxit=5000, f64_warmup=0, dgo_images=4, dgo_weight_power=1):
    """J = A : C_eff : B (A, B Voigt tensor-component 6-vectors; B = A by
    default) for Young's modulus field `young` and Poisson ratio `nu`.
    Differentiable with respect to `young` for every scheme (the DGO runs on
    the PCD grid with the given image window and weight power, and needs an
    explicit reference medium, which the gradient holds fixed).  Raises
    LsfftError when either solve fails or diverges."""
    if scheme.lower() == "dgo" and (lambda0 is None or mu0 is None):
        # the DGO's discrete solution depends on C0 (Sec. 5.4); the gradient
        # returned holds C0 fixed, so it must not be derived from E
        raise ValueError("scheme='dgo' needs an explicit reference medium (lambda0, mu0)")
    A = np.asarray(A, dtype=np.float64)
    B = A if B is None else np.asarray(B, dtype=np.float64)
    if A.shape != (6,) or B.shape != (6,):
        raise ValueError("A and B must be Voigt 6-vectors of tensor components")
    return _EffectiveStiffness.apply(young, float(nu), A, B, lambda0, mu0, scheme, prec, float(tol), int(maxit),
                                     int(f64_warmup), (int(dgo_images), int(dgo_weight_power)))
