"""Exact diagonalisation built WITHOUT any MPO (oracle; test infrastructure only).

Spin chains: bit-string basis, matrix elements from the spin-flip rule.
Fermions: occupation-number basis over modes ordered site-major with the up
mode before the down mode (mode 2i = (i, up), 2i+1 = (i, dn)); a basis state
is prod_{modes in increasing order} (c+_mode)^{n_mode} |vac>, so
c+_p c_q carries the sign (-1)^{number of occupied modes strictly between}.
These basis states coincide with the Jordan-Wigner product states used by the
MPO builders, which is what lets the two be compared element by element.
The product-basis index has site 1 as the most significant digit; the local
fermion digit is 0 = empty, 1 = up, 2 = dn, 3 = updn.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def spin_chain_hamiltonian(l, couplings, field=None):
    """Sparse H = sum J_ij S_i.S_j + sum h_i Sz_i on 2^l states.
    Digit of site i (0-based) is bit (l-1-i); digit 0 = up, 1 = down."""
    dim = 1 << l
    rows, cols, vals = [], [], []
    h = field if field is not None else [0.0] * l
    for s in range(dim):
        def up(i):
            return ((s >> (l - 1 - i)) & 1) == 0
        diag = 0.0
        for (i, j), J in couplings.items():
            si = 0.5 if up(i) else -0.5
            sj = 0.5 if up(j) else -0.5
            diag += J * si * sj
            if up(i) != up(j):
                s2 = s ^ (1 << (l - 1 - i)) ^ (1 << (l - 1 - j))
                rows.append(s2)
                cols.append(s)
                vals.append(0.5 * J)
        for i in range(l):
            diag += h[i] * (0.5 if up(i) else -0.5)
        rows.append(s)
        cols.append(s)
        vals.append(diag)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


def _fock_to_product_index(occ, l):
    """occupation bits (mode 2i = up_i, 2i+1 = dn_i) -> product-basis index."""
    idx = 0
    for i in range(l):
        nu = (occ >> (2 * i)) & 1
        nd = (occ >> (2 * i + 1)) & 1
        digit = {(0, 0): 0, (1, 0): 1, (0, 1): 2, (1, 1): 3}[(nu, nd)]
        idx = idx * 4 + digit
    return idx


def hubbard_hamiltonian(l, hoppings, U=0.0, mu=None):
    """Sparse H = -sum t_ij (c+_is c_js + h.c.) + U sum n_up n_dn - sum mu n
    on the full 4^l product basis (all particle numbers)."""
    dim = 4 ** l
    nmodes = 2 * l
    m = mu if mu is not None else [0.0] * l
    rows, cols, vals = [], [], []
    for occ in range(1 << nmodes):
        col = _fock_to_product_index(occ, l)
        diag = 0.0
        for i in range(l):
            nu = (occ >> (2 * i)) & 1
            nd = (occ >> (2 * i + 1)) & 1
            diag += U * nu * nd - m[i] * (nu + nd)
        rows.append(col)
        cols.append(col)
        vals.append(diag)
        for (i, j), t in hoppings.items():
            for s in (0, 1):
                for p, q in ((2 * i + s, 2 * j + s), (2 * j + s, 2 * i + s)):
                    # c+_p c_q |occ>
                    if not (occ >> q) & 1 or ((occ >> p) & 1 and p != q):
                        continue
                    lo, hi = min(p, q), max(p, q)
                    between = occ & (((1 << hi) - 1) ^ ((1 << (lo + 1)) - 1))
                    sign = -1.0 if bin(between).count("1") % 2 else 1.0
                    new = (occ ^ (1 << q)) | (1 << p)
                    rows.append(_fock_to_product_index(new, l))
                    cols.append(col)
                    vals.append(-t * sign)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


def particle_numbers(l):
    """(N, 2Sz) of every product-basis state of the Hubbard chain."""
    n_of = np.array([0, 1, 1, 2])
    sz_of = np.array([0, 1, -1, 0])
    N = np.zeros(4 ** l, dtype=np.int64)
    S = np.zeros(4 ** l, dtype=np.int64)
    for i in range(l):
        digit = (np.arange(4 ** l) // 4 ** (l - 1 - i)) % 4
        N += n_of[digit]
        S += sz_of[digit]
    return N, S


def spin_sz(l):
    """2Sz of every spin product-basis state."""
    tot = np.zeros(1 << l, dtype=np.int64)
    for i in range(l):
        bit = (np.arange(1 << l) >> (l - 1 - i)) & 1
        tot += 1 - 2 * bit
    return tot


def ground_energy(H, mask=None):
    """Smallest eigenvalue of sparse symmetric H, optionally restricted to
    the basis states where mask is True."""
    if mask is not None:
        idx = np.nonzero(mask)[0]
        H = H[idx][:, idx]
    n = H.shape[0]
    if n <= 2048:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    vals = spla.eigsh(H, k=1, which="SA", tol=1e-14)[0]
    return float(vals[0])


def free_fermion_energy(l, hoppings, n_up, n_dn):
    """Closed form for U = 0: sum of the lowest single-particle levels."""
    h = np.zeros((l, l))
    for (i, j), t in hoppings.items():
        h[i, j] -= t
        h[j, i] -= t
    eps = np.linalg.eigvalsh(h)
    return float(eps[:n_up].sum() + eps[:n_dn].sum())
