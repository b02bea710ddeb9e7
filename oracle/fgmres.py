"""Flexible GMRES with right preconditioning (Saad 1993), as used in Sec. 7.1
and 7.2 of the paper as the FP64 outer iteration, and the non-flexible
right-preconditioned GMRES it is compared with (Sec. 7.2, the robustness
argument for FGMRES).

Readings: Arnoldi by modified Gram-Schmidt; x0 = 0; the iteration stops once
the Arnoldi residual estimate |g_{j+1}| <= rtol * ||b||_2 (the paper stops on
a relative l2 residual reduction); restart after m steps from the true
residual.  The returned info holds the true relative residual.
"""
import numpy as np


def fgmres(apply_A, b, precond, rtol=1e-10, restart=30, max_iters=300, x0=None,
           on_iteration=None, on_estimate=None, flexible=True):
    """Solve A x = b.  ``precond(v)`` may change from step to step (flexible).

    ``flexible=False`` is right-preconditioned GMRES: the same Arnoldi process
    on A M, but only the basis V is kept and the update is x += M(V y), one
    more preconditioner application, which equals the flexible update only
    when M is the same linear map in every step.

    Returns (x, info) with info = dict(iterations, rel_res_est, rel_res_true,
    history, converged).  ``on_iteration(j, z)`` may inspect (and replace) the
    preconditioned vector; used for failure-injection tests.  ``on_estimate(
    history)`` sees the residual history after every Arnoldi step (the learned
    stage's fallback rule reads it)."""
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    history = []
    if nb == 0.0:
        return x, dict(iterations=0, rel_res_est=0.0, rel_res_true=0.0,
                       history=[0.0], converged=True)
    tol = rtol * nb
    it = 0
    converged = False
    while it < max_iters and not converged:
        r = b - apply_A(x)
        beta = float(np.linalg.norm(r))
        history.append(beta / nb)
        if beta <= tol:
            converged = True
            break
        m = restart
        V = np.zeros((m + 1, b.size))
        Z = np.zeros((m, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            z = precond(V[j])
            if on_iteration is not None:
                z = on_iteration(it, z)
            Z[j] = z
            w = apply_A(z)
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            history.append(abs(g[j + 1]) / nb)
            if on_estimate is not None:
                on_estimate(history)
            if abs(g[j + 1]) <= tol or it >= max_iters or H[j, j] == 0.0:
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:]) / H[i, i]
        if flexible:
            x = x + Z[:j_done].T @ y
        else:
            x = x + precond(V[:j_done].T @ y)
        if abs(g[j_done]) <= tol:
            converged = True
    rel_true = float(np.linalg.norm(b - apply_A(x)) / nb)
    return x, dict(iterations=it, rel_res_est=history[-1], rel_res_true=rel_true,
                   history=history, converged=converged)
