"""Adjoint of H_eff with respect to the MPO tensor (oracle; test infrastructure only).

H_eff psi is linear in W, so the vector-Jacobian product of y = H_eff(W) psi
with a cotangent ybar is, by definition,
  Wbar[w, v, s, t] = sum_{a,b,x,y} ybar[a, s, b] L[a, w, x] psi[x, t, y] R[b, v, y].
With ybar = psi (unit norm) this is dE/dW_i of E = <psi|H_eff|psi>.  Summing
<dE/dW_i, dW_i/dJ> over all sites, each taken in the mixed-canonical gauge
centred on that site, gives dE/dJ = <Psi|dH/dJ|Psi> (product rule over the
MPO tensors; Hellmann-Feynman at an eigenstate).
"""
import numpy as np

from . import contract as C
from .mps import left_canonicalize


def heff_grad_W(L, R, psi, ybar):
    return np.einsum("asb,awx,xty,bvy->wvst", ybar, L, psi, R)


def energy_gradients(mpo, tensors):
    """dE/dW_i for every site of the (normalised) state `tensors`."""
    l = len(mpo)
    M = left_canonicalize(tensors)
    # right-canonicalise towards site 0, building the right environments
    Renv = [None] * (l + 1)
    Renv[l] = np.ones((1, 1, 1))
    for i in range(l - 1, 0, -1):
        ml, d, mr = M[i].shape
        Q, Rf = np.linalg.qr(M[i].reshape(ml, d * mr).T)   # M^T = Q R  ->  M = R^T Q^T
        k = Q.shape[1]
        M[i] = Q.T.reshape(k, d, mr)
        prev = M[i - 1]
        M[i - 1] = (prev.reshape(-1, ml) @ Rf.T).reshape(prev.shape[0], prev.shape[1], k)
        Renv[i] = C.update_right(Renv[i + 1], mpo[i], M[i])
    M[0] = M[0] / np.linalg.norm(M[0])
    grads = []
    Lenv = np.ones((1, 1, 1))
    for i in range(l):
        grads.append(heff_grad_W(Lenv, Renv[i + 1], M[i], M[i]))
        if i + 1 < l:
            ml, d, mr = M[i].shape
            Q, Rf = np.linalg.qr(M[i].reshape(ml * d, mr))
            k = Q.shape[1]
            M[i] = Q.reshape(ml, d, k)
            nxt = M[i + 1]
            M[i + 1] = (Rf @ nxt.reshape(mr, -1)).reshape(k, nxt.shape[1], nxt.shape[2])
            Lenv = C.update_left(Lenv, mpo[i], M[i])
    return grads


def mpo_expectation(mpo, tensors):
    """<Psi|H|Psi> / <Psi|Psi> by a left-to-right environment contraction."""
    Lenv = np.ones((1, 1, 1))
    norm = np.ones((1, 1))
    for W, M in zip(mpo, tensors):
        Lenv = C.update_left(Lenv, W, M)
        norm = np.einsum("ax,asb,xsy->by", norm, M, M)
    return float(Lenv[0, 0, 0] / norm[0, 0])
