"""MPO builders (oracle; test infrastructure only).

An MPO tensor is stored as W[w, w', s, t] with shape (w_{i-1}, w_i, d, d):
w / w' are the left / right MPO bonds, s the output (bra) and t the input
(ket) physical index.  The paper writes the same tensor as (d, d, w, w)
(Sec. 2); this is a permutation of it.

Construction: finite-state form with channel 0 = "no operator placed yet",
channel w-1 = "term complete", and for every operator type `op` and range
r = 1..R a channel "op was placed r sites to the left".  The first site keeps
only row 0, the last site only column w-1.  The paper only prints the
two-site example (Sec. 4.3); the finite-state form is the textbook one.

A pair term  c_ij * A_i B_j  (i < j <= i + R) is written as
  W_i[0, (A,1)] = A,   W_k[(A,r), (A,r+1)] = S  (string, r = k - i),
  W_j[(A, j-i), w-1] = c_ij * B.
"""
import numpy as np

from .local_ops import spin_half, spin_half_pauli_like, fermion_site


def _finite_state_mpo(l, d, starts, strings, finishers, coupling, onsite, R):
    """Generic finite-state MPO.

    starts[k]    operator placed at the first site of a pair term (type k)
    strings[k]   operator on the sites strictly between the two partners
    finishers[k] operator at the second site (multiplied by the coupling)
    coupling(i, j) -> float   amplitude of the pair (i, j), i < j
    onsite[i]    (d, d) operator on site i (may be zero)
    """
    nk = len(starts)
    w = 2 + nk * R
    final = w - 1
    ident = np.eye(d)

    def ch(k, r):
        return 1 + (r - 1) * nk + k

    mpo = []
    for j in range(l):
        Wb = np.zeros((w, w, d, d))
        Wb[0, 0] = ident
        Wb[final, final] = ident
        Wb[0, final] = onsite[j]
        for k in range(nk):
            Wb[0, ch(k, 1)] = starts[k]
            for r in range(1, R):
                Wb[ch(k, r), ch(k, r + 1)] = strings[k]
            for r in range(1, R + 1):
                i = j - r
                if i >= 0:
                    c = coupling(i, j)
                    if c != 0.0:
                        Wb[ch(k, r), final] = c * finishers[k]
        mpo.append(Wb)
    if l == 1:
        return [mpo[0][0:1, final:final + 1].copy()]
    mpo[0] = mpo[0][0:1].copy()
    mpo[-1] = mpo[-1][:, final:final + 1].copy()
    return mpo


def spin_exchange_mpo(l, couplings, field=None):
    """H = sum_{i<j} J_ij (Sz_i Sz_j + (S+_i S-_j + S-_i S+_j)/2) + sum h_i Sz_i.

    couplings: dict {(i, j): J_ij} with 0 <= i < j < l (0-based sites).
    """
    ops = spin_half()
    R = max(j - i for (i, j) in couplings) if couplings else 1
    starts = [ops["Sp"], ops["Sm"], ops["Sz"]]
    strings = [ops["I"]] * 3
    finishers = [0.5 * ops["Sm"], 0.5 * ops["Sp"], ops["Sz"]]
    h = field if field is not None else [0.0] * l
    onsite = [h[i] * ops["Sz"] for i in range(l)]
    return _finite_state_mpo(l, 2, starts, strings, finishers,
                             lambda i, j: couplings.get((i, j), 0.0), onsite, R)


def heisenberg_mpo(l, J=1.0):
    """Spin-1/2 Heisenberg chain, open boundaries, w = 5."""
    return spin_exchange_mpo(l, {(i, i + 1): J for i in range(l - 1)})


def j1j2_mpo(l, J1=1.0, J2=0.0):
    """J1-J2 chain, open boundaries, w = 8 (range-2 finite-state form)."""
    c = {(i, i + 1): J1 for i in range(l - 1)}
    for i in range(l - 2):
        c[(i, i + 2)] = J2
    return spin_exchange_mpo(l, c)


def fermion_hopping_mpo(l, hoppings, U=0.0, mu=None):
    """H = -sum_{i<j} t_ij sum_s (c+_is c_js + h.c.) + U sum n_up n_dn - sum mu_i n_i.

    hoppings: dict {(i, j): t_ij}.  Jordan-Wigner strings F between the
    partners; the starting operator on site i is c+_s F (for c+_i c_j) or
    F c_s (for c+_j c_i), as follows from c_i = F_1...F_{i-1} c_i^loc.
    """
    ops = fermion_site()
    F = ops["F"]
    R = max(j - i for (i, j) in hoppings) if hoppings else 1
    starts = [ops["cd_up"] @ F, ops["cd_dn"] @ F, F @ ops["c_up"], F @ ops["c_dn"]]
    strings = [F] * 4
    finishers = [-ops["c_up"], -ops["c_dn"], -ops["cd_up"], -ops["cd_dn"]]
    m = mu if mu is not None else [0.0] * l
    onsite = [U * ops["n_updn"] - m[i] * (ops["n_up"] + ops["n_dn"]) for i in range(l)]
    return _finite_state_mpo(l, 4, starts, strings, finishers,
                             lambda i, j: hoppings.get((i, j), 0.0), onsite, R)


def hubbard_chain_mpo(l, t=1.0, U=0.0):
    """Fermi-Hubbard chain, open boundaries, w = 6."""
    return fermion_hopping_mpo(l, {(i, i + 1): t for i in range(l - 1)}, U=U)


def cylinder_bonds(width, length):
    """Nearest-neighbour bonds of a width x length cylinder (periodic across
    the width, open along the length), sites numbered column by column:
    s = x * width + y.  Every column is traversed in the same direction, so
    the longest bond spans `width` sites."""
    bonds = []
    for x in range(length):
        for y in range(width):
            s = x * width + y
            if width > 1 and (y + 1 < width or width > 2):
                s2 = x * width + (y + 1) % width
                bonds.append((min(s, s2), max(s, s2)))
            if x + 1 < length:
                bonds.append((s, s + width))
    return sorted(set(bonds))


def hubbard_cylinder_mpo(width, length, t=1.0, U=0.0):
    """Fermi-Hubbard cylinder; w = 2 + 4*width (18 for width 4)."""
    return fermion_hopping_mpo(width * length,
                               {b: t for b in cylinder_bonds(width, length)}, U=U)


def worked_example_mpo():
    """The two-spin MPO printed in Sec. 4.3, with the operators as printed:
    W_1 = [S+/sqrt2, S-/sqrt2, Sz] (row), W_2 = [S-/sqrt2, S+/sqrt2, Sz]^T."""
    ops = spin_half_pauli_like()
    r2 = np.sqrt(2.0)
    W1 = np.zeros((1, 3, 2, 2))
    W1[0, 0] = ops["Sp"] / r2
    W1[0, 1] = ops["Sm"] / r2
    W1[0, 2] = ops["Sz"]
    W2 = np.zeros((3, 1, 2, 2))
    W2[0, 0] = ops["Sm"] / r2
    W2[1, 0] = ops["Sp"] / r2
    W2[2, 0] = ops["Sz"]
    return [W1, W2]


def mpo_apply(mpo, v):
    """H v for the operator of an open-boundary MPO without forming its
    matrix (v has d^l entries, site 1 the most significant digit): the sites
    are applied one at a time to the not yet reached digits of v, keeping the
    open MPO channel as the leading index."""
    d = mpo[0].shape[2]
    X = np.asarray(v, dtype=np.float64).reshape(1, 1, -1)      # [w, done digits, remaining digits]
    for W in mpo:
        w, n_done, n_rest = X.shape
        X = X.reshape(w, n_done, d, n_rest // d)                 # [w, O, t, rest]
        Y = np.tensordot(W, X, axes=([0, 3], [0, 2]))            # [v, s, O, rest]
        X = Y.transpose(0, 2, 1, 3).reshape(W.shape[1], n_done * d, n_rest // d)
    assert X.shape[0] == 1 and X.shape[2] == 1
    return X.reshape(-1)


def mpo_to_dense(mpo):
    """Contract an open-boundary MPO into the full d^l x d^l matrix
    (site 1 is the most significant digit of the basis index)."""
    T = mpo[0][0]                       # (w, d, d)
    T = np.transpose(T, (0, 1, 2))      # T[w, out, in]
    for W in mpo[1:]:
        # T_new[w', (O,s), (I,t)] = sum_w T[w, O, I] W[w, w', s, t]
        n = T.shape[1]
        d = W.shape[2]
        Tn = np.einsum("wOI,wvst->vOsIt", T, W)
        T = Tn.reshape(W.shape[1], n * d, n * d)
    assert T.shape[0] == 1
    return T[0]
