"""GPU parity of the exact-residual expansion (the residual H Psi - E Psi in
place of the cheap expansion term) against the CPU FP64 oracle: the H^2
channel-pair environments, the Gram matrix of the expanded tensor, the
truncation from a Gram matrix, and whole sweeps.
Tolerances: FP64 contractions 1e-12 relative to the largest entry; the
Gram truncation's singular values 1e-10 s_0 (eigenvalues of a Gram matrix
carry absolute errors near n u s_0^2); energies 1e-10.
"""
import numpy as np
import pytest
import torch

from oracle import contract as C
from oracle import ed, mpo as MPO
from oracle.dmrg3s import DMRG3S
from paper_1501_05504_amd import synth

pytestmark = pytest.mark.gpu

abi = pytest.importorskip("paper_1501_05504_amd.abi")

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = abi.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device=DEV).contiguous()


def rel_err(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def _mpo_site(model):
    if model == "heisenberg":
        return np.asarray(MPO.heisenberg_mpo(5)[2])          # w = 5, d = 2: LDS W-map
    return np.asarray(MPO.hubbard_chain_mpo(5, t=1.0, U=4.0)[2])   # w = 6, d = 4: wide W-map


H2_SHAPES = [(1, 1), (3, 5), (17, 9), (40, 33)]


@pytest.mark.parametrize("model", ["heisenberg", "hubbard"])
@pytest.mark.parametrize("ml,mr", H2_SHAPES, ids=[str(s) for s in H2_SHAPES])
def test_update_env_h2(ctx, model, ml, mr):
    W = _mpo_site(model)
    wl, wr, d = W.shape[0], W.shape[1], W.shape[2]
    site = synth.gaussian((ml, d, mr), 501)
    Gl = synth.gaussian((ml, wl, wl, ml), 502)
    Gr = synth.gaussian((mr, wr, wr, mr), 503)
    out = torch.full((mr * wr * wr * mr,), float("nan"), dtype=torch.float64, device=DEV)
    ctx.update_env_h2(abi.L2R, dev(Gl), dev(W), dev(site), out)
    torch.cuda.synchronize()
    ref = C.update_left_h2(Gl, W, site)
    assert rel_err(out.cpu().numpy().reshape(ref.shape), ref) < 1e-12
    out = torch.full((ml * wl * wl * ml,), float("nan"), dtype=torch.float64, device=DEV)
    ctx.update_env_h2(abi.R2L, dev(Gr), dev(W), dev(site), out)
    torch.cuda.synchronize()
    ref = C.update_right_h2(Gr, W, site)
    assert rel_err(out.cpu().numpy().reshape(ref.shape), ref) < 1e-12


GRAM_SHAPES = [(1, 2), (4, 7), (20, 13), (33, 40)]


@pytest.mark.parametrize("model", ["heisenberg", "hubbard"])
@pytest.mark.parametrize("ml,mr", GRAM_SHAPES, ids=[str(s) for s in GRAM_SHAPES])
def test_residual_gram(ctx, model, ml, mr):
    W = _mpo_site(model)
    wl, wr, d = W.shape[0], W.shape[1], W.shape[2]
    L = synth.gaussian((ml, wl, ml), 511)
    R = synth.gaussian((mr, wr, mr), 512)
    psi = synth.gaussian((ml, d, mr), 513)
    Gr = synth.gaussian((mr, wr, wr, mr), 514)
    Gl = synth.gaussian((ml, wl, wl, ml), 515)
    E, alpha = -3.25, 0.07
    gram = torch.full(((ml * d) ** 2,), float("nan"), dtype=torch.float64, device=DEV)
    ctx.residual_gram(abi.L2R, dev(L), dev(R), dev(Gr), dev(W), dev(psi), E, alpha, gram)
    torch.cuda.synchronize()
    ref = C.residual_gram_l2r(L, W, R, Gr, psi, E, alpha)
    assert rel_err(gram.cpu().numpy().reshape(ref.shape), ref) < 1e-12
    gram = torch.full(((d * mr) ** 2,), float("nan"), dtype=torch.float64, device=DEV)
    ctx.residual_gram(abi.R2L, dev(L), dev(R), dev(Gl), dev(W), dev(psi), E, alpha, gram)
    torch.cuda.synchronize()
    ref = C.residual_gram_r2l(L, W, R, Gl, psi, E, alpha)
    assert rel_err(gram.cpu().numpy().reshape(ref.shape), ref) < 1e-12


@pytest.mark.parametrize("direction", ["l2r", "r2l"])
def test_truncate_gram(ctx, direction):
    """Truncation from the Gram matrix of an expanded tensor: same k,
    singular values, kept subspace and (sign-aligned) neighbour as the
    oracle."""
    ml, d, mr, kmax = 12, 2, 15, 9
    psi = synth.gaussian((ml, d, mr), 521)
    if direction == "l2r":
        Mt = np.hstack([psi.reshape(ml * d, mr), 0.3 * synth.gaussian((ml * d, 30), 522)])
        Gm = Mt @ Mt.T
        nbr = synth.gaussian((mr, d, 7), 523)
        A, B, s, disc = C.truncate_gram_l2r(Gm, psi, nbr, kmax, 1e-14)
        k_ref = A.shape[2]
        site = torch.empty(ml * d * kmax, dtype=torch.float64, device=DEV)
        nout = torch.empty(kmax * d * 7, dtype=torch.float64, device=DEV)
        k, dd, sg = ctx.truncate_gram(abi.L2R, dev(Gm), dev(psi), kmax, 1e-14, dev(nbr), site, nout,
                                      renormalize=False)
        U = site[:ml * d * k].view(ml * d, k).cpu().numpy()
        X = nout[:k * d * 7].view(k, -1).cpu().numpy()
        Ur, Xr = A.reshape(ml * d, k_ref), B.reshape(k_ref, -1)
    else:
        Mt = np.vstack([psi.reshape(ml, d * mr), 0.3 * synth.gaussian((25, d * mr), 524)])
        Gm = Mt.T @ Mt
        nbr = synth.gaussian((5, d, ml), 525)
        Bt, A, s, disc = C.truncate_gram_r2l(Gm, psi, nbr, kmax, 1e-14)
        k_ref = Bt.shape[0]
        site = torch.empty(kmax * d * mr, dtype=torch.float64, device=DEV)
        nout = torch.empty(5 * d * kmax, dtype=torch.float64, device=DEV)
        k, dd, sg = ctx.truncate_gram(abi.R2L, dev(Gm), dev(psi), kmax, 1e-14, dev(nbr), site, nout,
                                      renormalize=False)
        U = site[:k * d * mr].view(k, d * mr).cpu().numpy().T
        X = nout[:5 * d * k].view(5 * d, k).cpu().numpy().T
        Ur, Xr = Bt.reshape(k_ref, -1).T, A.reshape(-1, k_ref).T
    assert k == k_ref
    assert np.allclose(np.array(sg[:k]), s[:k], atol=1e-10 * s[0])
    assert abs(dd - disc) < 1e-10 * float(np.sum(s ** 2))
    assert np.allclose(U @ U.T, Ur @ Ur.T, atol=1e-10)
    sign = np.sign(np.sum(U * Ur, axis=0))
    assert np.allclose(X * sign[:, None], Xr, atol=1e-9 * np.abs(Xr).max())


def _run_gpu(ctx, mpo, tensors, m, expansion, sweeps, tol=1e-12):
    st = abi.State(mpo, tensors, m, device=DEV)
    e0 = ctx.prepare(st)
    params = abi.sweep_params(alpha=1e-3, e_before=e0, expansion=expansion)
    prev, energies = None, []
    for _ in range(sweeps):
        _, stats, recs = ctx.sweep(st, params)
        energies.append(stats.energy)
        if prev is not None and abs(stats.energy - prev) / abs(stats.energy) < tol:
            break
        prev = stats.energy
    return energies, st, recs


def test_residual_sweep_heisenberg12(ctx):
    """Heisenberg l = 12: with the exact-residual expansion the GPU sweeps
    reach ED at the exact bond (m = 64) and the oracle's converged energy at
    m = 16, where the cheap term gives the same energy."""
    l = 12
    e_ed = ed.ground_energy(ed.spin_chain_hamiltonian(l, {(i, i + 1): 1.0 for i in range(l - 1)}))
    es, _, _ = _run_gpu(ctx, abi.heisenberg_mpo(l), synth.random_mps(l, 2, 64), 64, "residual", 12)
    assert abs(es[-1] - e_ed) < 1e-10
    tensors = synth.random_mps(l, 2, 16)
    es, st, _ = _run_gpu(ctx, abi.heisenberg_mpo(l), tensors, 16, "residual", 30)
    run = DMRG3S(MPO.heisenberg_mpo(l), tensors, mmax=16, alpha0=1e-3, expansion="residual")
    E, _ = run.run(tol=1e-12, max_sweeps=30)
    assert abs(es[-1] - E) < 1e-10
    assert max(st.m) <= 16
    es_h, _, _ = _run_gpu(ctx, abi.heisenberg_mpo(l), tensors, 16, "heuristic", 30)
    assert abs(es[-1] - es_h[-1]) < 1e-6


def test_residual_sweep_hubbard_half_filling(ctx):
    """Hubbard l = 6, U = 8, mu = U/2, exact bond m = 64: the wide channel-pair
    MPO (w^2 = 36, d = 4) path; the energy equals Fock ED of the half-filled
    sector."""
    l, U = 6, 8.0
    mpo = abi.hubbard_chain_mpo(l, t=1.0, U=U, mu=[U / 2] * l)
    es, _, _ = _run_gpu(ctx, mpo, synth.random_mps(l, 4, 64, seed=8), 64, "residual", 12)
    H = ed.hubbard_hamiltonian(l, {(i, i + 1): 1.0 for i in range(l - 1)}, U=U)
    N, S = ed.particle_numbers(l)
    e_ed = ed.ground_energy(H, mask=(N == l) & (S == 0))
    assert abs(es[-1] + U / 2 * l - e_ed) < 1e-9


def test_residual_sweep_rejected_for_blocks(ctx):
    l = 4
    mpo = abi.hubbard_chain_mpo(l, t=1.0, U=4.0, mu=[2.0] * l)
    tensors, secs = synth.random_symmetric_mps(l, abi.HUBBARD_CHARGES, [l, 0], 8)
    st = abi.State(mpo, tensors, 8, device=DEV)
    sym = abi.Symmetry(abi.HUBBARD_CHARGES, abi.mpo_bond_charges(mpo, abi.mpo_fermion_charges(1)), secs)
    e0 = ctx.prepare_blocks(st, sym)
    with pytest.raises(abi.D3SError):
        ctx.sweep_blocks(st, sym, abi.sweep_params(alpha=1e-3, e_before=e0, expansion="residual"))
