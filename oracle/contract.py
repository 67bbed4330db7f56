"""Local contractions of DMRG3S (oracle; test infrastructure only).

Layouts (row-major, real):
  L[a, w, x]    (m_l, w_l, m_l)  left environment;  a bra, x ket
  W[w, v, s, t] (w_l, w_r, d, d) MPO tensor;         s out, t in
  psi[x, t, y]  (m_l, d, m_r)   site tensor
  R[b, v, y]    (m_r, w_r, m_r)  right environment; b bra, y ket
  out[a, s, b]  (m_l, d, m_r)
"""
import numpy as np


def apply_heff(L, W, R, psi):
    """H_eff psi = L_{i-1} R_{i+1} W_i M_i (eq. es-iter), contracted in the
    order ((( L M ) W ) R) given in Sec. 5:
      1. L with M over the left MPS bond,
      2. W over the physical index of M and the left MPO bond,
      3. R over the right MPO and MPS bonds."""
    T1 = np.tensordot(L, psi, axes=([2], [0]))            # [a, w, t, y]
    T2 = np.tensordot(T1, W, axes=([1, 2], [0, 3]))       # [a, y, v, s]
    return np.tensordot(T2, R, axes=([2, 1], [1, 2]))     # [a, s, b]


def heff_matrix(L, W, R):
    """The explicit (d m_l m_r)^2 matrix of H_eff, row index (a, s, b),
    column index (x, t, y)."""
    H = np.einsum("awx,wvst,bvy->asbxty", L, W, R)
    n = L.shape[0] * W.shape[2] * R.shape[0]
    return H.reshape(n, n)


def update_left(L, W, A):
    """L_i = L_{i-1} A_i^dagger W_i A_i (Sec. 2): new[b, v, y]."""
    X = np.tensordot(L, A, axes=([2], [0]))               # [a, w, t, y]
    X = np.tensordot(X, W, axes=([1, 2], [0, 3]))         # [a, y, v, s]
    return np.tensordot(A, X, axes=([0, 1], [0, 3])).transpose(0, 2, 1)  # A[a,s,b] -> [b, y, v] -> [b, v, y]


def update_right(R, W, B):
    """R_i = R_{i+1} B_i^dagger W_i B_i (Sec. 2): new[a, w, x]."""
    X = np.tensordot(B, R, axes=([2], [2]))               # B[x,t,y] R[b,v,y] -> [x, t, b, v]
    X = np.tensordot(X, W, axes=([1, 3], [3, 1]))         # [x, b, w, s]
    return np.tensordot(B, X, axes=([1, 2], [3, 1])).transpose(0, 2, 1)  # B[a,s,b] -> [a, x, w] -> [a, w, x]


def expansion_term_l2r(L, W, psi, alpha):
    """P_i = alpha L_{i-1} M_i W_i (eq. subexp-ourt) for a left-to-right sweep,
    as P[a, s, v, y] with shape (m_l, d, w_r, m_r)."""
    X = np.tensordot(L, psi, axes=([2], [0]))             # [a, w, t, y]
    X = np.tensordot(X, W, axes=([1, 2], [0, 3]))         # [a, y, v, s]
    return alpha * X.transpose(0, 3, 2, 1)


def expansion_term_r2l(R, W, psi, alpha):
    """P_i = alpha R_{i+1} M_i W_i for a right-to-left sweep, as P[w, a, s, b]
    with shape (w_l, m_l, d, m_r)."""
    X = np.tensordot(psi, R, axes=([2], [2]))             # [a, t, b, v]
    X = np.tensordot(X, W, axes=([1, 3], [3, 1]))         # [a, b, w, s]
    return alpha * X.transpose(2, 0, 3, 1)


def expanded_tensor_l2r(psi, P):
    """M~ = [M  P] (Sec. 4.1) as the (m_l d) x (m_r + w_r m_r) matrix."""
    ml, d, mr = psi.shape
    return np.hstack([psi.reshape(ml * d, mr), P.reshape(ml * d, -1)])


def expanded_tensor_r2l(psi, P):
    """M~ = [M ; P] (Sec. 4.1) as the (m_l + w_l m_l) x (d m_r) matrix."""
    ml, d, mr = psi.shape
    return np.vstack([psi.reshape(ml, d * mr), P.reshape(-1, d * mr)])


def truncation_size(s, kmax, eps):
    """Number of singular values kept: at most kmax, and only s_j > eps s_0."""
    if s.size == 0 or s[0] == 0.0:
        return 0
    return int(min(kmax, np.count_nonzero(s > eps * s[0])))


def truncate_l2r(Mt, psi, nbr, kmax, eps):
    """Steps 4-5 of the site update (Sec. 5), left to right.

    SVD of M~, keep k singular triplets; the new site tensor is U_k and the
    remainder S V^T meets the zero-padded neighbour [B; 0], so only its first
    m_r columns matter: B~ = (U_k^T M*) B.  Returns (A, B~, s, discarded)."""
    ml, d, mr = psi.shape
    U, s, Vt = np.linalg.svd(Mt, full_matrices=False)
    k = truncation_size(s, kmax, eps)
    A = U[:, :k].reshape(ml, d, k)
    X = U[:, :k].T @ psi.reshape(ml * d, mr)              # (k, m_r)
    nb = X @ nbr.reshape(mr, -1)
    discarded = float(np.sum(s[k:] ** 2))
    return A, nb.reshape(k, nbr.shape[1], nbr.shape[2]), s, discarded


def truncate_r2l(Mt, psi, nbr, kmax, eps):
    """Mirror of truncate_l2r for a right-to-left sweep: the new site tensor is
    V_k^T, the neighbour A~ = A (M* V_k)."""
    ml, d, mr = psi.shape
    U, s, Vt = np.linalg.svd(Mt, full_matrices=False)
    k = truncation_size(s, kmax, eps)
    B = Vt[:k].reshape(k, d, mr)
    X = psi.reshape(ml, d * mr) @ Vt[:k].T                # (m_l, k)
    na = nbr.reshape(-1, ml) @ X
    discarded = float(np.sum(s[k:] ** 2))
    return B, na.reshape(nbr.shape[0], nbr.shape[1], k), s, discarded


def energy(L, W, R, psi):
    """<psi|H_eff|psi> / <psi|psi>."""
    return float(np.vdot(psi, apply_heff(L, W, R, psi)) / np.vdot(psi, psi))


# --- comparison methods (two-site DMRG of Sec. 7.2, CWF of Sec. 3.3) --------

def apply_heff_two_site(L, W1, W2, R, psi2):
    """Two-site H_eff psi2 for psi2[x, t1, t2, y] of shape (m_l, d, d, m_r)
    (the two-site DMRG local problem, compared with in Sec. 7.2), contracted like the single-site
    one: L over the left MPS bond, W1 over (w, t1), W2 over (v1, t2), R over
    the right MPO and MPS bonds.  out[a, s1, s2, b]."""
    T = np.tensordot(L, psi2, axes=([2], [0]))            # [a, w, t1, t2, y]
    T = np.tensordot(T, W1, axes=([1, 2], [0, 3]))        # [a, t2, y, v1, s1]
    T = np.tensordot(T, W2, axes=([3, 1], [0, 3]))        # [a, y, s1, v2, s2]
    return np.tensordot(T, R, axes=([3, 1], [1, 2]))      # [a, s1, s2, b]


def cwf_environment(L, W):
    """The enlarged left environment of the centre-matrix formalism (Sec. 3.3):
    Lt[(a, s), v, (x, t)] = sum_w L[a, w, x] W[w, v, s, t], shape
    (m_l d, w_r, m_l d)."""
    ml, d, wr = L.shape[0], W.shape[2], W.shape[1]
    Lt = np.einsum("awx,wvst->asvxt", L, W)
    return Lt.reshape(ml * d, wr, ml * d)


def apply_cwf(Lt, R, C):
    """H applied to the centre matrix C[(x, t), y] of shape (m_l d, m_r) with the
    enlarged environment: out[(a, s), b] = sum Lt[(a,s), v, (x,t)] C[(x,t), y]
    R[b, v, y] (Sec. 3.3); 2 w m^3 d (d + 1) flops against 4 w m^3 d (plus the
    W-map) for the three-step single-site order of Sec. 5, a ratio (d + 1)/2."""
    T = np.tensordot(Lt, C, axes=([2], [0]))              # [(a,s), v, y]
    return np.tensordot(T, R, axes=([1, 2], [1, 2]))      # [(a,s), b]


def two_site_split(psi2, kmax, eps):
    """Truncated SVD split of a two-site tensor psi2 (m_l, d, d, m_r) as the
    (m_l d) x (d m_r) matrix, as two-site DMRG does after its eigensolver:
    A = U_k (m_l, d, k) and the right factor S_k V_k^T (k, d, m_r).  Returns
    (A, SVt, s, discarded)."""
    ml, d, d2, mr = psi2.shape
    U, s, Vt = np.linalg.svd(psi2.reshape(ml * d, d2 * mr), full_matrices=False)
    k = truncation_size(s, kmax, eps)
    A = U[:, :k].reshape(ml, d, k)
    SVt = (s[:k, None] * Vt[:k]).reshape(k, d2, mr)
    return A, SVt, s, float(np.sum(s[k:] ** 2))
