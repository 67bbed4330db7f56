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


# --- exact-residual expansion term (the residual Z = H Psi - E Psi of the
# Sec. 4 opening, in place of the cheap term of eq. subexp-ourt) ------------
#
# At site i of a left-to-right sweep the residual is kept with its left part
# projected onto the current left basis A_{<i} (those rows are what the
# expanded tensor's left bond can take up) and its right part exact.  Its
# coefficients on |A_a s> are then spread over the right-side vectors
# |B_y> (from -E Psi) and H_{>i,v} |B_y> (from H Psi, the local H Psi
# coefficients being L M W), which are not orthonormal: the metric between
# them needs <H_v B_y | H_v' B_y'>, the right environment of the channel
# pairs of H^2.  Right-to-left is the mirror.

def update_left_h2(G, W, A):
    """G_new[b, v, u, y] = <H_v A_b | H_u A_y> for the left-part MPO
    operators H_v (channel v of the bond right of the site):
    sum G[a, w, c, x] A[a, t, b] W[w, v, s, t] W[c, u, s, e] A[x, e, y]."""
    X = np.tensordot(G, A, axes=([3], [0]))               # [a, w, c, e, y]
    X = np.tensordot(X, W, axes=([2, 3], [0, 3]))         # [a, w, y, u, s]
    X = np.tensordot(X, W, axes=([1, 4], [0, 2]))         # [a, y, u, v, t]
    X = np.tensordot(A, X, axes=([0, 1], [0, 4]))         # [b, y, u, v]
    return X.transpose(0, 3, 2, 1)


def update_right_h2(G, W, B):
    """G_new[y, v, z, x] = <H_v B_y | H_z B_x> for the right-part MPO
    operators H_v (channel v of the bond left of the site):
    sum B[y, t, b] W[v, u, s, t] W[z, c, s, e] B[x, e, q] G[b, u, c, q]."""
    X = np.tensordot(B, G, axes=([2], [3]))               # [x, e, b, u, c]
    X = np.tensordot(X, W, axes=([1, 4], [3, 1]))         # [x, b, u, z, s]
    X = np.tensordot(X, W, axes=([2, 4], [1, 2]))         # [x, b, z, v, t]
    X = np.tensordot(B, X, axes=([1, 2], [4, 1]))         # [y, x, z, v]
    return X.transpose(0, 3, 2, 1)


def residual_gram_l2r(L, W, R, Gr, psi, E, alpha):
    """Left Gram matrix (m_l d) x (m_l d) of the expanded tensor [M | alpha Z]
    whose expansion part is the exact residual: M M^T + alpha^2 <z|z>, with
    z_{(a,s)} = sum_y (-E M[a,s,y]) |B_y> + sum_{v,y} (L M W)[a,s,v,y] H_v|B_y>.
    R is the right environment of the site and Gr the H^2 one (bond right
    of the site)."""
    ml, d, mr = psi.shape
    wr = W.shape[1]
    Mm = psi.reshape(ml * d, mr)
    Pm = expansion_term_l2r(L, W, psi, 1.0).reshape(ml * d, wr * mr)
    Zc = np.hstack([-E * Mm, Pm])
    G = residual_metric_l2r(R, Gr)
    return Mm @ Mm.T + alpha ** 2 * (Zc @ G @ Zc.T)


def residual_gram_r2l(L, W, R, Gl, psi, E, alpha):
    """Right Gram matrix (d m_r) x (d m_r) of [M ; alpha Z] (mirror of
    residual_gram_l2r): z_{(s,b)} = sum_a (-E M[a,s,b]) |A_a> +
    sum_{w,a} (W M R)[w,a,s,b] H_w|A_a>, with the metric <A_a'|H_w A_a> =
    L[a', w, a] and <H_w A_a | H_w' A_a'> = Gl[a, w, w', a']."""
    ml, d, mr = psi.shape
    wl = W.shape[0]
    Mm = psi.reshape(ml, d * mr)
    Pm = expansion_term_r2l(R, W, psi, 1.0).reshape(wl * ml, d * mr)
    Zc = np.vstack([-E * Mm, Pm])
    G = residual_metric_r2l(L, Gl)
    return Mm.T @ Mm + alpha ** 2 * (Zc.T @ G @ Zc)


def _metric_factor(G):
    """F (n x r) with G = F F^T for the metric G of the residual's
    vectors, from the eigen-decomposition of G.  Those vectors are linearly
    dependent (the far-side operator of the completed MPO channel is the
    identity, so it repeats |B_y>); eigenvalues of G at or below
    n u lambda_max are such exact dependences and are taken as zero."""
    lam, Q = np.linalg.eigh(G)
    keep = lam > G.shape[0] * np.finfo(np.float64).eps * lam.max()
    return Q[:, keep] * np.sqrt(lam[keep])


def residual_metric_l2r(R, Gr):
    """Metric of |B_y> and H_v|B_y> (the right-side vectors of a left-to-right
    residual): [[1, R], [R^T, Gr]] with <B_y'|H_v B_y> = R[y', v, y]."""
    mr, wr = R.shape[0], R.shape[1]
    Rm = R.reshape(mr, wr * mr)
    Ghh = Gr.transpose(1, 0, 2, 3).reshape(wr * mr, wr * mr)
    return np.block([[np.eye(mr), Rm], [Rm.T, Ghh]])


def residual_metric_r2l(L, Gl):
    """Mirror of residual_metric_l2r for |A_a> and H_w|A_a>."""
    ml, wl = L.shape[0], L.shape[1]
    Lm = L.reshape(ml, wl * ml)
    Ghh = Gl.transpose(1, 0, 2, 3).reshape(wl * ml, wl * ml)
    return np.block([[np.eye(ml), Lm], [Lm.T, Ghh]])


def residual_expanded_l2r(L, W, R, Gr, psi, E, alpha):
    """The expanded tensor [M | alpha Z] with the exact residual as its
    expansion part, written on an orthonormal basis of the span of the
    residual's right-side vectors: [M | alpha Z_c F] with G = F F^T, an
    (m_l d) x (m_r + r) matrix whose SVD is the truncation's (its Gram
    matrix is residual_gram_l2r)."""
    ml, d, mr = psi.shape
    wr = W.shape[1]
    Mm = psi.reshape(ml * d, mr)
    Pm = expansion_term_l2r(L, W, psi, 1.0).reshape(ml * d, wr * mr)
    Zc = np.hstack([-E * Mm, Pm])
    F = _metric_factor(residual_metric_l2r(R, Gr))
    return np.hstack([Mm, alpha * (Zc @ F)])


def residual_expanded_r2l(L, W, R, Gl, psi, E, alpha):
    """Mirror of residual_expanded_l2r: [M ; alpha F^T Z_c], an
    (m_l + r) x (d m_r) matrix."""
    ml, d, mr = psi.shape
    wl = W.shape[0]
    Mm = psi.reshape(ml, d * mr)
    Pm = expansion_term_r2l(R, W, psi, 1.0).reshape(wl * ml, d * mr)
    Zc = np.vstack([-E * Mm, Pm])
    F = _metric_factor(residual_metric_r2l(L, Gl))
    return np.vstack([Mm, alpha * (F.T @ Zc)])
