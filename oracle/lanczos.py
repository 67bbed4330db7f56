"""Lanczos eigensolver for the smallest eigenpair (oracle; test infrastructure only).

Step 1 of the site update (Sec. 5) needs only a solver for the lowest
eigenpair of H_eff.  This is the textbook Lanczos three-term recurrence with
full re-orthogonalisation against all previous Krylov vectors (classical
Gram-Schmidt applied twice), a Krylov basis of at most `kmax` vectors and an
explicit restart from the current Ritz vector.  Convergence: the residual
norm of the Ritz pair, |beta_k y_k|, falls below tol * max(1, |theta|).
"""
import numpy as np


def lanczos_ground(matvec, v0, tol=1e-12, kmax=40, max_restarts=200):
    """Return (theta, x, n_matvec, converged) for the smallest eigenpair."""
    shape = v0.shape
    v = np.asarray(v0, dtype=np.float64).ravel().copy()
    n = v.size
    nv = np.linalg.norm(v)
    if nv == 0.0:
        v = np.ones(n)
        nv = np.linalg.norm(v)
    v /= nv
    nmv = 0
    theta = None
    for _ in range(max_restarts):
        V = [v]
        alphas, betas = [], []
        converged = False
        y = np.array([1.0])
        for k in range(min(kmax, n)):
            w = matvec(V[k].reshape(shape)).ravel()
            nmv += 1
            a = float(np.dot(V[k], w))
            alphas.append(a)
            w = w - a * V[k]
            if k > 0:
                w = w - betas[k - 1] * V[k - 1]
            Vm = np.array(V)
            for _ in range(2):
                w = w - Vm.T @ (Vm @ w)
            b = float(np.linalg.norm(w))
            T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
            ev, Y = np.linalg.eigh(T)
            theta = float(ev[0])
            y = Y[:, 0]
            resid = abs(b * y[-1])
            scale = max(1.0, abs(theta))
            if resid <= tol * scale or b <= 1e-15 * scale or k + 1 == n:
                converged = True
                break
            betas.append(b)
            V.append(w / b)
        x = np.array(V[: len(y)]).T @ y
        x /= np.linalg.norm(x)
        if converged:
            return theta, x.reshape(shape), nmv, True
        v = x
    return theta, x.reshape(shape), nmv, False
