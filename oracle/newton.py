"""Smoothed Newton-CG ("CG-Newton") on the pseudo-Huber problem (8).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2 replaces ||x||_1 by the pseudo-Huber function
psi_mu(x) = sum_i (sqrt(mu^2 + x_i^2) - mu)  (eq. (7)) and minimises
f_mu(x) = tau*psi_mu(x) + 0.5*||A x - b||^2  (problem (8)) with the Newton
model (9).  Section 8.1 (item pdNCG) solves the Newton system
grad^2 f_mu(x) d = -grad f_mu(x) inexactly by preconditioned CG with the
inverse diagonal of grad^2 f_mu as preconditioner; section 8.3 fixes
mu = 1e-5, stops PCG at relative residual 1e-1 and caps the backtracking
line search at 50 steps.

The primal-dual mechanics of the cited pdNCG paper are not part of this
paper.  ``hessian="primal"`` uses the exact Hessian of (8):
d_i = tau * mu^2 / w_i^3 with w_i = sqrt(mu^2 + x_i^2).
``hessian="primal_dual"`` linearises the pair (tau*g + A^T(Ax - b) = 0,
w*g - x = 0) in (x, g) and eliminates dg, which gives the same system with
d_i = tau * (1 - x_i g_i / w_i) / w_i, followed by g <- proj_[-1,1](g + dg).
Both variants are written out here from that derivation.
"""
import numpy as np


def pseudo_huber(x, mu):
    """psi_mu(x) of eq. (7)."""
    return float(np.sum(np.sqrt(mu * mu + x * x) - mu))


def smoothed_objective(A_mv, b, tau, mu, x):
    """f_tau^mu(x) of problem (8)."""
    r = A_mv(x) - b
    return tau * pseudo_huber(x, mu) + 0.5 * float(r @ r)


def pcg(H_mv, rhs, Minv, rtol, maxit):
    """Preconditioned CG on H d = rhs from d = 0; stop at ||r|| <= rtol ||rhs||."""
    d = np.zeros_like(rhs)
    r = rhs.copy()
    z = Minv * r
    p = z.copy()
    rz = float(r @ z)
    stop = rtol * float(np.linalg.norm(rhs))
    it = 0
    while it < maxit and float(np.linalg.norm(r)) > stop:
        Hp = H_mv(p)
        alpha = rz / float(p @ Hp)
        d += alpha * p
        r -= alpha * Hp
        z = Minv * r
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return d, it


def newton_cg(A_mv, At_mv, colnorm2, b, tau, mu=1e-5, x0=None,
              max_newton=200, pcg_rtol=0.1, pcg_maxit=1000, max_backtrack=50,
              armijo=1e-4, grad_tol=None, hessian="primal_dual"):
    """Returns (x, stats) with stats = dict(newton=, pcg=, grad_inf=)."""
    n = colnorm2.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    gd = np.zeros(n)
    grad_tol = 1e-9 * tau if grad_tol is None else grad_tol
    f = lambda v: smoothed_objective(A_mv, b, tau, mu, v)
    total_pcg = 0
    k = 0
    gnorm = np.inf
    for k in range(max_newton):
        w = np.sqrt(mu * mu + x * x)
        grad = tau * x / w + At_mv(A_mv(x) - b)
        gnorm = float(np.abs(grad).max())
        if gnorm <= grad_tol:
            break
        if hessian == "primal":
            d = tau * mu * mu / (w ** 3)
        else:
            d = tau * (1.0 - x * gd / w) / w
        H_mv = lambda p: At_mv(A_mv(p)) + d * p
        dx, it = pcg(H_mv, -grad, 1.0 / (colnorm2 + d), pcg_rtol, pcg_maxit)
        total_pcg += it
        f0 = f(x)
        slope = float(grad @ dx)
        alpha = 1.0
        for _ in range(max_backtrack):
            if f(x + alpha * dx) <= f0 + armijo * alpha * slope:
                break
            alpha *= 0.5
        if hessian != "primal":
            dg = -gd + x / w + (1.0 - x * gd / w) * dx / w
            gd = np.clip(gd + dg, -1.0, 1.0)
        x = x + alpha * dx
    return x, dict(newton=k, pcg=total_pcg, grad_inf=gnorm)
