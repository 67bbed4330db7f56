"""MPS helpers (oracle; test infrastructure only).

A site tensor is M[a, s, b] with shape (m_{i-1}, d, m_i); the paper writes
(d, m_{i-1}, m_i) (Sec. 2), a permutation of it.
"""
import numpy as np


def bond_budget(l, d, mmax):
    """Largest useful bond dimension of every bond 0..l: min(m, d^b, d^(l-b))."""
    return [int(min(mmax, d ** b, d ** (l - b))) for b in range(l + 1)]


def left_canonicalize(tensors):
    """QR sweep from the left: every tensor but the last becomes left-normalised
    (sum_s A^s+ A^s = 1, Sec. 2); the last one carries the norm, which is then
    divided out so that the state has unit norm."""
    out = [np.array(t, dtype=np.float64) for t in tensors]
    for i in range(len(out) - 1):
        ml, d, mr = out[i].shape
        Q, Rf = np.linalg.qr(out[i].reshape(ml * d, mr))
        k = Q.shape[1]
        out[i] = Q.reshape(ml, d, k)
        nxt = out[i + 1]
        out[i + 1] = (Rf @ nxt.reshape(mr, -1)).reshape(k, nxt.shape[1], nxt.shape[2])
    out[-1] = out[-1] / np.linalg.norm(out[-1])
    return out


def state_vector(tensors):
    """Contract an open MPS into the d^l coefficient vector (site 1 is the most
    significant digit), eq. psi-as-mps-general."""
    v = tensors[0]                                  # (1, d, m)
    v = v.reshape(v.shape[1], v.shape[2])
    for t in tensors[1:]:
        v = np.tensordot(v, t, axes=([1], [0]))     # (D, d, m)
        v = v.reshape(-1, t.shape[2])
    return v.ravel()


def is_left_normalised(A, tol=1e-12):
    ml, d, mr = A.shape
    M = A.reshape(ml * d, mr)
    return np.allclose(M.T @ M, np.eye(mr), atol=tol)


def is_right_normalised(B, tol=1e-12):
    ml, d, mr = B.shape
    M = B.reshape(ml, d * mr)
    return np.allclose(M @ M.T, np.eye(ml), atol=tol)
