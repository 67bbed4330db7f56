"""Single-site operators (oracle; test infrastructure only).

Spin-1/2: basis (|up>, |down>); Sz = diag(1/2, -1/2), S+ = |up><down|.
Spinful fermions (d = 4): basis (|0>, |up>, |dn>, |updn>) with
|updn> = c+_up c+_dn |0>, i.e. within a site the up mode precedes the down
mode.  Jordan-Wigner: c_{i,s} = F_1 ... F_{i-1} c_{i,s}^loc with
F = (-1)^n = diag(1, -1, -1, 1); the on-site ordering puts an F_up factor
into the local down annihilator.
"""
import numpy as np


def spin_half():
    sz = np.diag([0.5, -0.5])
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    sm = sp.T.copy()
    ident = np.eye(2)
    return {"I": ident, "Sz": sz, "Sp": sp, "Sm": sm}


def spin_half_pauli_like():
    """Operators exactly as printed in the two-spin example (Sec. 4.3).

    The printed expansion term needs Sz = diag(1, -1) with S+ = |up><down|
    (with Sz = diag(1/2, -1/2) its third column would carry a factor 1/2).
    """
    ops = spin_half()
    ops["Sz"] = np.diag([1.0, -1.0])
    return ops


def fermion_site():
    # basis index: 0 = |0>, 1 = |up>, 2 = |dn>, 3 = |updn> = c+_up c+_dn |0>
    c_up = np.zeros((4, 4))
    c_up[0, 1] = 1.0    # c_up |up>   = |0>
    c_up[2, 3] = 1.0    # c_up |updn> = c_up c+_up c+_dn |0> = |dn>
    c_dn = np.zeros((4, 4))
    c_dn[0, 2] = 1.0    # c_dn |dn>   = |0>
    c_dn[1, 3] = -1.0   # c_dn |updn> = -c+_up c_dn c+_dn |0> = -|up>
    ops = {
        "I": np.eye(4),
        "F": np.diag([1.0, -1.0, -1.0, 1.0]),
        "c_up": c_up,
        "c_dn": c_dn,
        "cd_up": c_up.T.copy(),
        "cd_dn": c_dn.T.copy(),
    }
    ops["n_up"] = ops["cd_up"] @ c_up
    ops["n_dn"] = ops["cd_dn"] @ c_dn
    ops["n_updn"] = ops["n_up"] @ ops["n_dn"]
    return ops
