"""GPU parity of the block-sparse (U(1) x U(1)) H_eff against the dense CPU
oracle on charge-conserving inputs: the grouped launches must reproduce the
dense contraction exactly (an exact reorganisation of the sum), leave the
forbidden blocks zero, and give the same result when replayed from a
captured hipGraph."""
import numpy as np
import pytest
import torch

from oracle import contract as C
from paper_1501_05504_amd import synth

pytestmark = pytest.mark.gpu

abi = pytest.importorskip("paper_1501_05504_amd.abi")

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = abi.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device=DEV).to(dtype).contiguous()


def rel_err(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def hubbard_block_case(ml, mr, seed, sigma=1.5, span=4):
    """Charge-conserving L, W, R, psi for the Hubbard MPO bulk tensor."""
    qL, dL = synth.gaussian_sectors((6, 0), (sigma, sigma), ml, (span, span))
    qR, dR = synth.gaussian_sectors((7, 1), (sigma, sigma), mr, (span, span))
    W = abi.hubbard_chain_mpo(3, t=1.0, U=8.0)[1]
    wq = abi.mpo_fermion_charges(1)
    phys = np.array(abi.HUBBARD_CHARGES)
    sl, sr = synth.expand_charges(qL, dL), synth.expand_charges(qR, dR)
    ml, mr = len(sl), len(sr)
    L = synth.gaussian((ml, W.shape[0], ml), seed) * synth.mask_env(sl, wq)
    R = synth.gaussian((mr, W.shape[1], mr), seed + 1) * synth.mask_env(sr, wq)
    psi = synth.gaussian((ml, 4, mr), seed + 2) * synth.mask_site(sl, phys, sr)
    return dict(qL=qL, dL=dL, qR=qR, dR=dR, W=W, wq=wq, phys=phys, L=L, R=R, psi=psi,
                mask=synth.mask_site(sl, phys, sr))


def make_plan(ctx, case):
    W = case["W"]
    return abi.BlockPlan(ctx, 2, 4, W.shape[0], W.shape[1], case["qL"], case["dL"], case["qR"], case["dR"],
                         case["phys"], case["wq"], case["wq"])


@pytest.mark.parametrize("ml,mr,seed", [(40, 52, 1), (96, 80, 2), (300, 257, 3)])
def test_block_heff_equals_dense_oracle(ctx, ml, mr, seed):
    case = hubbard_block_case(ml, mr, seed)
    ref = C.apply_heff(case["L"], case["W"], case["R"], case["psi"])
    assert np.abs(ref[~case["mask"]]).max() < 1e-12 * np.abs(ref).max()     # symmetry of the oracle result
    plan = make_plan(ctx, case)
    out = torch.full(case["psi"].shape, float("nan"), dtype=torch.float64, device=DEV)
    plan.apply(dev(case["L"]), dev(case["W"]), dev(case["R"]), dev(case["psi"]), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert rel_err(got, ref) < 1e-12
    assert np.all(got[~case["mask"]] == 0.0)
    assert plan.ntasks > 10 and plan.flops > 0
    plan.close()


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4, 5])
def test_block_heff_every_grouped_tile(cfg):
    """Every grouped tile configuration gives the oracle's result in FP64,
    FP32 and BF16 (the low-precision products run on the padded twin; BF16
    against the oracle on rounded operands with the rounding model of the
    dense tests)."""
    from tests.test_gpu_parity import bf16_bound, bf16_round
    case = hubbard_block_case(150, 130, 17)
    ref = C.apply_heff(case["L"], case["W"], case["R"], case["psi"])
    Lb, Rb, pb = bf16_round(case["L"]), bf16_round(case["R"]), bf16_round(case["psi"])
    Wf = np.asarray(case["W"], dtype=np.float32).astype(np.float64)
    ref_b = C.apply_heff(Lb, Wf, Rb, pb)
    bound_b = bf16_bound(Lb, Wf, Rb, pb)
    c = abi.Context(0)
    try:
        c.set_grouped_tile(cfg)
        plan = make_plan(c, case)
        for dt, tol in ((torch.float64, 1e-12), (torch.float32, 3e-5)):
            out = torch.empty(case["psi"].shape, dtype=dt, device=DEV)
            plan.apply(dev(case["L"], dt), dev(case["W"], dt), dev(case["R"], dt), dev(case["psi"], dt), out)
            torch.cuda.synchronize()
            assert rel_err(out.double().cpu().numpy(), ref) < tol
        out = torch.empty(case["psi"].shape, dtype=torch.float32, device=DEV)
        plan.apply(dev(Lb, torch.bfloat16), dev(Wf, torch.float32), dev(Rb, torch.bfloat16), dev(pb, torch.bfloat16),
                   out)
        torch.cuda.synchronize()
        assert np.all(np.abs(out.double().cpu().numpy() - ref_b) <= bound_b)
        plan.close()
    finally:
        c.close()


def test_block_heff_f32(ctx):
    case = hubbard_block_case(120, 100, 5)
    f = torch.float32
    L, W, R, psi = [np.asarray(x, dtype=np.float32).astype(np.float64)
                    for x in (case["L"], case["W"], case["R"], case["psi"])]
    ref = C.apply_heff(L, W, R, psi)
    plan = make_plan(ctx, case)
    out = torch.empty(psi.shape, dtype=f, device=DEV)
    plan.apply(dev(L, f), dev(W, f), dev(R, f), dev(psi, f), out)
    torch.cuda.synchronize()
    assert rel_err(out.double().cpu().numpy(), ref) < 3e-5
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("ml,mr,seed", [(20, 17, 13), (40, 52, 11), (300, 257, 12)])
def test_block_heff_low_precision_transposed_psi(ctx, prec, ml, mr, seed):
    """FP32 / BF16 block products against the oracle on the rounded operands
    (FP32 3e-5; BF16 the element-wise model of the rounding of T2 to 8 bits,
    test_gpu_parity.bf16_bound),
    eager and replayed from a captured graph; the forbidden blocks stay
    zero.  The product runs on the plan's twin over sectors padded to
    multiples of 8 (operands moved in and the product moved back), whose
    first GEMM reads the block-transposed psi; odd sector dimensions make
    the padding non-trivial (with ml = 20 the sectors hold 1-3 states and
    the padded blocks are mostly zeros)."""
    case = hubbard_block_case(ml, mr, seed)
    t = torch.float32 if prec == "f32" else torch.bfloat16
    Lt, Rt, pt = dev(case["L"], t), dev(case["R"], t), dev(case["psi"], t)
    Wf = dev(case["W"], torch.float32)
    ref = C.apply_heff(Lt.double().cpu().numpy(), Wf.double().cpu().numpy(), Rt.double().cpu().numpy(),
                       pt.double().cpu().numpy())
    from tests.test_gpu_parity import bf16_bound
    plan = make_plan(ctx, case)
    bound = None if prec == "f32" else bf16_bound(Lt.double().cpu().numpy(), Wf.double().cpu().numpy(),
                                                  Rt.double().cpu().numpy(), pt.double().cpu().numpy())
    forbidden = case["mask"] == 0
    for use_graph in (False, True, True):
        out = torch.full(tuple(pt.shape), float("nan"), dtype=torch.float32, device=DEV)
        plan.apply(Lt, Wf, Rt, pt, out, use_graph=use_graph)
        torch.cuda.synchronize()
        o = out.double().cpu().numpy()
        if bound is None:
            assert rel_err(o, ref) < 3e-5, use_graph
        else:
            assert np.all(np.abs(o - ref) <= bound), use_graph
        assert np.all(o[forbidden] == 0.0)
    plan.close()


def test_block_heff_graph_replays(ctx):
    """Captured once, replayed several times with eager work (and a changed
    input in place) between the replays; every replay equals the eager
    result of the same inputs."""
    case = hubbard_block_case(96, 88, 7)
    plan = make_plan(ctx, case)
    L, W, R = dev(case["L"]), dev(case["W"]), dev(case["R"])
    x = dev(case["psi"])
    out_g = torch.empty_like(x)
    out_e = torch.empty_like(x)
    for rep in range(4):
        plan.apply(L, W, R, x, out_g, use_graph=True)
        torch.cuda.synchronize()
        plan.apply(L, W, R, x, out_e, use_graph=False)
        torch.cuda.synchronize()
        assert torch.equal(out_g, out_e), rep
        ref = C.apply_heff(case["L"], case["W"], case["R"], x.cpu().numpy())
        assert rel_err(out_g.cpu().numpy(), ref) < 1e-12
        x.mul_(0.5).add_(out_e / (1.0 + out_e.abs().max()))      # eager work, new input in place
        x.mul_(dev(case["mask"].astype(np.float64)))
    plan.close()


def test_block_heff_autotuned_plan(tmp_path):
    """A plan built with autotuning on (both grouped tile sizes timed) gives
    the oracle's result."""
    case = hubbard_block_case(160, 150, 9)
    ref = C.apply_heff(case["L"], case["W"], case["R"], case["psi"])
    c = abi.Context(0)
    try:
        c.set_autotune(True, tmp_path / "tune.txt")
        plan = make_plan(c, case)
        out = torch.empty(case["psi"].shape, dtype=torch.float64, device=DEV)
        plan.apply(dev(case["L"]), dev(case["W"]), dev(case["R"]), dev(case["psi"]), out)
        torch.cuda.synchronize()
        assert rel_err(out.cpu().numpy(), ref) < 1e-12
        plan.close()
    finally:
        c.close()


@pytest.mark.parametrize("ml,mr,seed", [(40, 52, 11), (300, 257, 12)])
def test_block_expand_equals_dense_oracle(ctx, ml, mr, seed):
    """[psi | alpha P] and [psi ; alpha P] from the grouped launches equal the
    oracle's dense expansion entry by entry (zeros outside the blocks)."""
    case = hubbard_block_case(ml, mr, seed)
    L, W, R, psi = case["L"], case["W"], case["R"], case["psi"]
    ml, mr = psi.shape[0], psi.shape[2]
    wl, wr = W.shape[0], W.shape[1]
    alpha = 0.43
    plan = make_plan(ctx, case)
    Mt = torch.full((ml * 4, (1 + wr) * mr), float("nan"), dtype=torch.float64, device=DEV)
    plan.expand_subspace(abi.L2R, dev(L), dev(W), dev(psi), alpha, Mt)
    Mt2 = torch.full(((1 + wl) * ml, 4 * mr), float("nan"), dtype=torch.float64, device=DEV)
    plan.expand_subspace(abi.R2L, dev(R), dev(W), dev(psi), alpha, Mt2)
    torch.cuda.synchronize()
    ref = C.expanded_tensor_l2r(psi, C.expansion_term_l2r(L, W, psi, alpha))
    ref2 = C.expanded_tensor_r2l(psi, C.expansion_term_r2l(R, W, psi, alpha))
    assert rel_err(Mt.cpu().numpy(), ref) < 1e-12
    assert rel_err(Mt2.cpu().numpy(), ref2) < 1e-12
    plan.close()


def _sector_spectrum_case(case, direction, seed):
    """An expanded tensor with the block structure of [psi | P] (L2R) or
    [psi ; P] (R2L) on the case's bonds: every charge Q of the new bond gets
    a block of rank about half its size with singular values
    scale_Q * geomspace(1, 1e-12, r_Q), scale_Q spread over 1 ... 1e-3, and
    zeros elsewhere.  Returns (Mt, psi, expected kept dims by charge key)."""
    rng = np.random.default_rng(seed)
    sl = synth.expand_charges(case["qL"], case["dL"])
    sr = synth.expand_charges(case["qR"], case["dR"])
    phys, wq = case["phys"], case["wq"]
    ml, mr, d, w = len(sl), len(sr), phys.shape[0], wq.shape[0]
    key = lambda q: (int(q[0]), int(q[1]))
    if direction == "l2r":
        side = [key(sl[a] + phys[s]) for a in range(ml) for s in range(d)]
        other = [key(sr[y]) for y in range(mr)] + [key(sr[y] + wq[v]) for v in range(w) for y in range(mr)]
        Mt = np.zeros((ml * d, (1 + w) * mr))
    else:
        side = [key(sr[b] - phys[s]) for s in range(d) for b in range(mr)]
        other = [key(sl[a]) for a in range(ml)] + [key(sl[a] + wq[v]) for v in range(w) for a in range(ml)]
        Mt = np.zeros(((1 + w) * ml, d * mr))
    side, other = np.array(side), np.array(other)
    charges = sorted(set(map(tuple, side)) & set(map(tuple, other)))
    values = {}
    for qi, Q in enumerate(charges):
        ri = np.nonzero(np.all(side == Q, axis=1))[0]
        ci = np.nonzero(np.all(other == Q, axis=1))[0]
        r = max(1, min(len(ri), len(ci)) // 2)
        sv = 10.0 ** (-3.0 * qi / max(1, len(charges) - 1)) * np.geomspace(1.0, 1e-12, r)
        U = np.linalg.qr(rng.standard_normal((len(ri), r)))[0]
        V = np.linalg.qr(rng.standard_normal((len(ci), r)))[0]
        blk = (U * sv) @ V.T
        if direction == "l2r":
            Mt[np.ix_(ri, ci)] = blk
        else:
            Mt[np.ix_(ci, ri)] = blk.T
        values[Q] = sv
    if direction == "l2r":
        psi = Mt[:, :mr].reshape(ml, d, mr).copy()
    else:
        psi = Mt[:ml].reshape(ml, d, mr).copy()
    s0 = max(v[0] for v in values.values())
    kept = {Q: int(np.count_nonzero(v > 1e-14 * s0)) for Q, v in values.items()}
    return Mt, psi, kept


@pytest.mark.parametrize("direction", ["l2r", "r2l"])
@pytest.mark.parametrize("ml,mr,seed", [(40, 52, 31), (300, 257, 32)])
def test_block_truncate_keeps_every_value_above_eps(ctx, direction, ml, mr, seed):
    """d3s_truncate_blocks on a block-structured expanded tensor whose sectors
    hold spectra reaching 1e-15 s_0: every value above 1e-14 s_0 is kept (most
    lie far below what one FP64 Gram matrix resolves), sector by sector; the
    dense LAPACK truncation of the same matrix keeps as many; the kept
    subspace, the site tensor's isometry and the neighbour agree with it."""
    case = hubbard_block_case(ml, mr, seed)
    ml, mr = case["psi"].shape[0], case["psi"].shape[2]
    d = 4
    Mt, psi, kept = _sector_spectrum_case(case, direction, seed + 100)
    plan = make_plan(ctx, case)
    rng = np.random.default_rng(seed)
    n = ml * d if direction == "l2r" else d * mr
    site = torch.empty(n * n, dtype=torch.float64, device=DEV)
    if direction == "l2r":
        nbr = rng.standard_normal((mr, d, 3))
        nout = torch.empty(n * d * 3, dtype=torch.float64, device=DEV)
        k, disc, q, dims = plan.truncate(abi.L2R, dev(Mt), dev(psi), n, 1e-14, dev(nbr), site, nout,
                                         renormalize=False)
        A, B, s, disc_ref = C.truncate_l2r(Mt, psi, nbr, n, 1e-14)
        U = site[: n * k].view(n, k).cpu().numpy()
        X = nout[: k * d * 3].view(k, -1).cpu().numpy()
        Ur, Xr = A.reshape(n, -1), B.reshape(A.shape[2], -1)
    else:
        nbr = rng.standard_normal((3, d, ml))
        nout = torch.empty(3 * d * n, dtype=torch.float64, device=DEV)
        k, disc, q, dims = plan.truncate(abi.R2L, dev(Mt), dev(psi), n, 1e-14, dev(nbr), site, nout,
                                         renormalize=False)
        Bs, A, s, disc_ref = C.truncate_r2l(Mt, psi, nbr, n, 1e-14)
        U = site[: k * n].view(k, n).cpu().numpy().T
        X = nout[: 3 * d * k].view(-1, k).cpu().numpy().T
        Ur, Xr = Bs.reshape(Bs.shape[0], -1).T, A.reshape(-1, Bs.shape[0]).T
    plan.close()
    assert k == sum(kept.values()) == Ur.shape[1]
    got = {(int(a), int(b)): int(m) for (a, b), m in zip(q, dims)}
    assert got == {Q: v for Q, v in kept.items() if v > 0}
    # sectors are ordered by charge and the site tensor is an isometry
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-13
    assert np.abs(U @ U.T - Ur @ Ur.T).max() < 1e-3
    assert rel_err(U @ X, Ur @ Xr) < 1e-9
    assert abs(disc - disc_ref) < 1e-14 * float(np.sum(s ** 2))


@pytest.mark.parametrize("direction", ["l2r", "r2l"])
def test_block_truncate_concurrent_solves_equal_serial(direction):
    """The sector eigensolves of one truncation run concurrently (four
    shares: the calling thread on the context's stream and three worker
    threads with their own streams) or one after the other: same kept states
    per sector, the same kept subspace and discarded weight to rounding."""
    case = hubbard_block_case(300, 257, 41)
    ml, mr, d = case["psi"].shape[0], case["psi"].shape[2], 4
    Mt, psi, kept = _sector_spectrum_case(case, direction, 141)
    n = ml * d if direction == "l2r" else d * mr
    res = []
    for workers in (1, 4):
        c = abi.Context(0)
        try:
            c.set_eig_workers(workers)
            plan = make_plan(c, case)
            site = torch.empty(n * n, dtype=torch.float64, device=DEV)
            if direction == "l2r":
                nbr = np.ones((mr, d, 3))
                nout = torch.empty(n * d * 3, dtype=torch.float64, device=DEV)
                k, disc, q, dims = plan.truncate(abi.L2R, dev(Mt), dev(psi), n, 1e-14, dev(nbr), site, nout,
                                                 renormalize=False)
                U = site[: n * k].view(n, k).cpu().numpy()
            else:
                nbr = np.ones((3, d, ml))
                nout = torch.empty(3 * d * n, dtype=torch.float64, device=DEV)
                k, disc, q, dims = plan.truncate(abi.R2L, dev(Mt), dev(psi), n, 1e-14, dev(nbr), site, nout,
                                                 renormalize=False)
                U = site[: k * n].view(k, n).cpu().numpy().T
            res.append((k, disc, [tuple(x) for x in np.asarray(q).tolist()], list(dims), U @ U.T))
            plan.close()
        finally:
            c.close()
    (k1, d1, q1, m1, P1), (k4, d4, q4, m4, P4) = res
    assert k1 == k4 == sum(kept.values())
    assert q1 == q4 and m1 == m4
    assert abs(d1 - d4) < 1e-14 * float(np.sum(Mt ** 2))
    assert np.abs(P1 - P4).max() < 1e-8


@pytest.mark.parametrize("ml,mr,seed", [(40, 52, 21), (300, 257, 22)])
def test_block_update_env_equals_dense_oracle(ctx, ml, mr, seed):
    """Both environment updates from the grouped launches equal the oracle's
    dense ones entry by entry (zeros outside the allowed blocks)."""
    case = hubbard_block_case(ml, mr, seed)
    L, W, R, psi = case["L"], case["W"], case["R"], case["psi"]
    ml, mr = psi.shape[0], psi.shape[2]
    wl, wr = W.shape[0], W.shape[1]
    plan = make_plan(ctx, case)
    out = torch.full((mr, wr, mr), float("nan"), dtype=torch.float64, device=DEV)
    plan.update_env(abi.L2R, dev(L), dev(W), dev(psi), out)
    out2 = torch.full((ml, wl, ml), float("nan"), dtype=torch.float64, device=DEV)
    plan.update_env(abi.R2L, dev(R), dev(W), dev(psi), out2)
    torch.cuda.synchronize()
    assert rel_err(out.cpu().numpy(), C.update_left(L, W, psi)) < 1e-12
    assert rel_err(out2.cpu().numpy(), C.update_right(R, W, psi)) < 1e-12
    plan.close()


@pytest.mark.parametrize("kind", [1, 2, 3])
@pytest.mark.parametrize("n,batch", [(1, 3), (7, 5), (40, 2), (96, 40), (128, 3), (130, 3)])
def test_eig_batched_equals_lapack(kind, n, batch):
    """The batched eigensolvers of the truncation against LAPACK:
    eigenvalues, eigenvectors through A V = V L, and V orthonormal.  Kind 1
    runs rocSOLVER divide and conquer, kind 2 rocSOLVER Jacobi, kind 3 the
    LDS solver up to n = 128 (divide and conquer above)."""
    c = abi.Context(0)
    try:
        c.set_eigensolver(kind)
        rng = np.random.default_rng(n * 10 + batch)
        X = rng.standard_normal((batch, n, n + 3))
        G = X @ X.transpose(0, 2, 1)
        A = torch.tensor(G, device=DEV)
        W = torch.empty((batch, n), dtype=torch.float64, device=DEV)
        c.eig_batched(A, W)
        torch.cuda.synchronize()
        for b in range(batch):
            w_ref = np.linalg.eigvalsh(G[b])
            scale = max(1.0, np.abs(w_ref).max())
            assert np.abs(W[b].cpu().numpy() - w_ref).max() < 1e-12 * scale
            V = A[b].cpu().numpy()          # row j = eigenvector j
            assert np.abs(G[b] @ V.T - V.T * W[b].cpu().numpy()).max() < 1e-11 * scale
            assert np.abs(V @ V.T - np.eye(n)).max() < 1e-12 * n
    finally:
        c.close()


def test_eig_small_solver_degenerate_and_padded():
    """The LDS eigensolver on what the truncation hands it: rank-deficient
    Gram matrices padded with zero rows and columns, and exactly repeated
    eigenvalues; eigenvalues against LAPACK, A V = V L and V orthonormal."""
    c = abi.Context(0)
    try:
        c.set_eigensolver(3)
        rng = np.random.default_rng(5)
        n = 72
        mats = []
        X = rng.standard_normal((50, 20))
        G = np.zeros((n, n))
        G[:50, :50] = X @ X.T                          # rank 20, 22 padded zero rows
        mats.append(G)
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam = np.repeat([0.0, 1.0, 2.5, 7.0], n // 4)  # four eigenvalues, 18 times each
        mats.append((Q * lam) @ Q.T)
        mats.append(np.zeros((n, n)))
        Gs = np.stack(mats)
        A = torch.tensor(Gs, device=DEV)
        W = torch.empty((len(mats), n), dtype=torch.float64, device=DEV)
        c.eig_batched(A, W)
        torch.cuda.synchronize()
        for b in range(len(mats)):
            w_ref = np.linalg.eigvalsh(Gs[b])
            scale = max(1.0, np.abs(w_ref).max())
            w = W[b].cpu().numpy()
            assert np.abs(w - w_ref).max() < 1e-12 * scale
            V = A[b].cpu().numpy()
            assert np.abs(Gs[b] @ V.T - V.T * w).max() < 1e-11 * scale
            assert np.abs(V @ V.T - np.eye(n)).max() < 1e-12 * n
    finally:
        c.close()
