"""CPU tests of the host side of the library: the shared object loads and
exports every symbol the public header declares, and the (host) MPO
builders of the product equal the oracle's, element by element."""
import ctypes
import os
import re

import numpy as np
import pytest


def abi_mod():
    from paper_1501_05504_amd import abi
    return abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmrg3s.h")
LIB = os.path.join(ROOT, "paper_1501_05504_amd", "lib", "libdmrg3s.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdmrg3s.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(d3s_[a-zA-Z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["d3s_apply_heff", "d3s_expand_subspace", "d3s_truncate", "d3s_update_env", "d3s_sweep",
              "d3s_lanczos", "d3s_heff_grad_W", "d3s_prepare", "d3s_create", "d3s_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_loads_and_version():
    from paper_1501_05504_amd import abi
    assert "gfx950" in abi.version()


def test_product_mpo_builders_equal_oracle():
    from oracle import mpo as MPO
    from paper_1501_05504_amd import abi
    cases = [
        (abi.heisenberg_mpo(7, 1.3), MPO.heisenberg_mpo(7, 1.3)),
        (abi.j1j2_mpo(9, 1.0, 0.24), MPO.j1j2_mpo(9, 1.0, 0.24)),
        (abi.hubbard_chain_mpo(5, 1.0, 8.0), MPO.hubbard_chain_mpo(5, 1.0, 8.0)),
        (abi.hubbard_cylinder_mpo(4, 3, 1.0, 4.0), MPO.hubbard_cylinder_mpo(4, 3, 1.0, 4.0)),
    ]
    for got, ref in cases:
        assert len(got) == len(ref)
        # the channel order inside the MPO bond is a gauge choice: compare the
        # contracted operators on short chains and the shapes everywhere
        for g, r in zip(got, ref):
            assert g.shape == r.shape
    # the contracted Hamiltonians agree exactly
    for got, ref in [(abi.heisenberg_mpo(6, 1.3), MPO.heisenberg_mpo(6, 1.3)),
                     (abi.j1j2_mpo(7, 1.0, 0.24), MPO.j1j2_mpo(7, 1.0, 0.24)),
                     (abi.hubbard_chain_mpo(4, 1.0, 8.0), MPO.hubbard_chain_mpo(4, 1.0, 8.0)),
                     (abi.hubbard_cylinder_mpo(4, 1, 1.0, 4.0), MPO.hubbard_cylinder_mpo(4, 1, 1.0, 4.0))]:
        assert np.abs(MPO.mpo_to_dense(got) - MPO.mpo_to_dense(ref)).max() < 1e-14


def test_product_cylinder_mpo_equals_oracle_4x2():
    """The product's w = 18 cylinder MPO (its own channel order) applies the
    same operator as the oracle's on the 4 x 2 cylinder, whose length bonds
    have range 4 (the oracle's builder is pinned to Fock-space ED there)."""
    from oracle import mpo as MPO
    from paper_1501_05504_amd import abi
    got = abi.hubbard_cylinder_mpo(4, 2, 1.0, 4.0)
    ref = MPO.hubbard_cylinder_mpo(4, 2, 1.0, 4.0)
    assert [g.shape for g in got] == [r.shape for r in ref]
    rng = np.random.default_rng(29)
    for _ in range(2):
        v = rng.standard_normal(4 ** 8)
        a, b = MPO.mpo_apply(got, v), MPO.mpo_apply(ref, v)
        assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()


def test_product_mpo_with_chemical_potential():
    from oracle import mpo as MPO
    from paper_1501_05504_amd import abi
    mu = [0.3, -0.2, 0.5, 0.1]
    got = abi.hubbard_chain_mpo(4, 1.0, 8.0, mu=mu)
    ref = MPO.fermion_hopping_mpo(4, {(i, i + 1): 1.0 for i in range(3)}, U=8.0, mu=mu)
    assert np.abs(MPO.mpo_to_dense(got) - MPO.mpo_to_dense(ref)).max() < 1e-14


def test_mpo_respects_channel_charges():
    """Host-side: the product MPO builders and their channel charges agree."""
    """Every nonzero W[w,v,s,t] satisfies q_s - q_t = Delta_v - Delta_w."""
    W = abi_mod().hubbard_chain_mpo(5, t=1.0, U=8.0)[2]
    wq = abi_mod().mpo_fermion_charges(1)
    phys = np.array(abi_mod().HUBBARD_CHARGES)
    for w, v, s, t in zip(*np.nonzero(W)):
        assert np.array_equal(phys[s] - phys[t], wq[v] - wq[w])
    Ws = abi_mod().j1j2_mpo(6, 1.0, 0.3)[3]
    sq = abi_mod().mpo_spin_charges(2)
    sp = np.array(abi_mod().SPIN_HALF_CHARGES)
    for w, v, s, t in zip(*np.nonzero(Ws)):
        assert np.array_equal(sp[s] - sp[t], sq[v] - sq[w])




def test_tridiag_lowest_matches_lapack():
    """Host helper of the eigensolver: the lowest eigenpair of symmetric
    tridiagonal matrices (random, split, graded, n = 1..60) against LAPACK."""
    from scipy.linalg import eigh_tridiagonal
    from paper_1501_05504_amd import abi
    rng = np.random.default_rng(7)
    cases = [(np.array([2.5]), np.array([]))]
    for n in [2, 3, 5, 17, 40, 60]:
        cases.append((rng.standard_normal(n), rng.standard_normal(n - 1)))
        cases.append((1e3 * rng.standard_normal(n), 1e-3 * rng.standard_normal(n - 1)))
    split = rng.standard_normal(12)
    bs = rng.standard_normal(11)
    bs[5] = 0.0
    cases.append((split, bs))
    # a Lanczos-like matrix: slowly varying diagonal near -60, off-diagonals ~ 1
    cases.append((-60 + np.cumsum(rng.uniform(0, 1, 40)), rng.uniform(0.5, 1.5, 39)))
    for a, b in cases:
        th, y = abi.tridiag_lowest(a, b)
        w, v = eigh_tridiagonal(a, b) if len(a) > 1 else (a.copy(), np.ones((1, 1)))
        scale = max(1.0, np.abs(a).max() + (np.abs(b).max() if len(b) else 0.0))
        assert abs(th - w[0]) <= 1e-13 * scale, (len(a), th, w[0])
        assert abs(np.linalg.norm(y) - 1.0) < 1e-12
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        assert np.linalg.norm(T @ y - th * y) <= 1e-12 * scale
        if len(a) > 1 and w[1] - w[0] > 1e-6 * scale:
            assert abs(abs(y @ v[:, 0]) - 1.0) < 1e-10
