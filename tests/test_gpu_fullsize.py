"""Parity at the measured sizes, in the launch configuration bench.py times
(default tile rule: 256x128 tiles, the steady-state K loop), on output rows
the CPU FP64 oracle computes one left index at a time; and the argument
checks at the edges of the accepted sizes.
Tolerances as for the small shapes: FP64 1e-12, FP32 3e-5 relative to the
largest entry of the sampled rows, BF16 the element-wise rounding model of
test_gpu_parity.bf16_bound.  64 rows are sampled: the first and last, both
sides of GEMM tile boundaries (256-row tiles of the (a, w) rows of the first
GEMM and of the (a, s) rows of the second), and seeded random ones.
The block H_eff the benchmark times at the 4096-state cylinder site is
checked the same way on 16 sampled rows.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import contract as C

pytestmark = pytest.mark.gpu

abi = pytest.importorskip("paper_1501_05504_amd.abi")

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = abi.Context(0)
    yield c
    c.close()


def rel_err(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def sampled_rows(m, w, n=64, seed=0):
    """n left indices: 0, m-1, both sides of GEMM-1 tile boundaries (its rows
    are (a, w); 256-row tiles), then seeded random ones."""
    rows = {0, m - 1}
    for step in (256 // w, 256 // 4):        # GEMM-1 rows (a, w); GEMM-2 rows (a, s), d = 4
        b = step
        while len(rows) < n // 2 and b < m:
            rows.update({b - 1, b})
            b += 11 * step
    rng = np.random.default_rng(seed)
    while len(rows) < n:
        rows.add(int(rng.integers(0, m)))
    return np.array(sorted(rows))


@pytest.mark.parametrize("m,prec", [(2048, "f64"), (2048, "f32"), (2048, "bf16"), (4096, "f64"), (4096, "f32")])
def test_heff_full_size_sampled_rows(ctx, m, prec):
    """Hubbard MPO shape (d = 4, w = 6) at the benchmark's bond dimensions, in
    the precisions the benchmark times, on 64 sampled output rows."""
    from tests.test_gpu_parity import bf16_bound
    d, w = 4, 6
    g = torch.Generator(device="cpu").manual_seed(900 + m)
    L = torch.randn((m, w, m), generator=g, dtype=torch.float64) / m
    W = torch.randn((w, w, d, d), generator=g, dtype=torch.float64)
    R = torch.randn((m, w, m), generator=g, dtype=torch.float64) / m
    psi = torch.randn((m, d, m), generator=g, dtype=torch.float64)
    t = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[prec]
    tw = torch.float64 if prec == "f64" else torch.float32
    to = torch.float64 if prec == "f64" else torch.float32
    Lt, Wt, Rt, pt = L.to(t), W.to(tw), R.to(t), psi.to(t)
    out = torch.full((m, d, m), float("nan"), dtype=to, device=DEV)
    ctx.set_tile_config(-1)
    ctx.apply_heff(Lt.to(DEV), Wt.to(DEV), Rt.to(DEV), pt.to(DEV), out)
    torch.cuda.synchronize()
    rows = sampled_rows(m, w, 64, seed=m)
    got = out[torch.tensor(rows, device=DEV)].double().cpu().numpy()
    del out
    assert np.isfinite(got).all()
    Lh, Wh, Rh, ph = (x.double().numpy() for x in (Lt, Wt, Rt, pt))
    ref = C.apply_heff(Lh[rows], Wh, Rh, ph)
    if prec == "bf16":
        assert np.all(np.abs(got - ref) <= bf16_bound(Lh[rows], Wh, Rh, ph))
    else:
        assert rel_err(got, ref) < (1e-12 if prec == "f64" else 3e-5)


def _raw_apply(ctx, dims, ptr=None):
    ml, d, mr, wl, wr = dims
    p = ctypes.c_void_p(ptr)
    return abi._apply_heff(ctx.h, abi.F64, ml, d, mr, wl, wr, p, p, p, p, ctypes.c_void_p(ptr + 8 if ptr else None))


@pytest.mark.parametrize("dims", [(0, 4, 8, 6, 6), (8, 0, 8, 6, 6), (8, 4, 0, 6, 6), (8, 4, 8, 0, 6),
                                  (8, 4, 8, 6, -1), (8, 4, 8, 21, 6), (8, 4, 8, 6, 21),
                                  (1 << 20, 4, 1 << 20, 6, 6)],
                         ids=["ml0", "d0", "mr0", "wl0", "wr-1", "wl*d>80", "wr*d>80", "too-large"])
def test_apply_heff_rejects_sizes_outside_the_accepted_range(ctx, dims):
    """Empty, negative and oversized dimensions are refused on the host with
    EINVAL before any pointer is touched (null pointers are passed)."""
    st = _raw_apply(ctx, dims)
    assert st == abi.EINVAL, abi._last_error(ctx.h)


def test_apply_heff_largest_mpo_bond(ctx):
    """w d = 80, the largest MPO bond the register W-map takes (w = 20,
    d = 4), against the oracle."""
    ml, d, mr, wl, wr = 24, 4, 31, 20, 20
    rng = np.random.default_rng(77)
    L, W, R, psi = (rng.standard_normal(s) for s in ((ml, wl, ml), (wl, wr, d, d), (mr, wr, mr), (ml, d, mr)))
    out = torch.empty((ml, d, mr), dtype=torch.float64, device=DEV)
    tt = lambda a: torch.tensor(a, dtype=torch.float64, device=DEV)
    ctx.apply_heff(tt(L), tt(W), tt(R), tt(psi), out)
    torch.cuda.synchronize()
    assert rel_err(out.cpu().numpy(), C.apply_heff(L, W, R, psi)) < 1e-12


def test_apply_heff_rejects_null_pointers(ctx):
    st = _raw_apply(ctx, (8, 4, 8, 6, 6))
    assert st == abi.EINVAL and b"null" in abi._last_error(ctx.h)


def _site_case():
    """The block H_eff of bench.py's cylinder_site: the w = 18 bulk MPO of
    the 4 x 16 Hubbard cylinder, 45 Gaussian U(1)xU(1) sectors per bond
    normalised to m = 4096, packed layout, seeded Gaussian entries."""
    from paper_1501_05504_amd import synth
    m = 4096
    qL, dL = synth.gaussian_sectors((28, 0), (1.5, 1.5), m, (8, 8))
    qR, dR = synth.gaussian_sectors((29, 1), (1.5, 1.5), m, (8, 8))
    mpo = abi.hubbard_cylinder_mpo(4, 16, t=1.0, U=4.0)
    W = np.asarray(mpo[len(mpo) // 2])
    wq = np.asarray(abi.mpo_fermion_charges(4))
    phys = np.asarray(abi.HUBBARD_CHARGES)
    return m, np.asarray(qL), np.asarray(dL), np.asarray(qR), np.asarray(dR), W, wq, phys


def _sector(qs, q):
    hit = np.nonzero(np.all(qs == q, axis=1))[0]
    return int(hit[0]) if len(hit) else -1


def _env_blocks(q, dims, wq):
    """(i, w, i', offset) of the packed environment blocks, in order."""
    out, off = [], 0
    for i in range(len(dims)):
        for w in range(len(wq)):
            ip = _sector(q, q[i] - wq[w])
            if ip >= 0:
                out.append((i, w, ip, off))
                off += int(dims[i]) * int(dims[ip])
    return out, off


def _site_blocks(qL, dL, qR, dR, phys):
    out, off = [], 0
    for i in range(len(dL)):
        for s in range(len(phys)):
            j = _sector(qR, qL[i] + phys[s])
            if j >= 0:
                out.append((i, s, j, off))
                off += int(dL[i]) * int(dR[j])
    return out, off


def test_block_site_full_size_sampled_rows(ctx):
    """The benchmark's block H_eff at the 4096-state cylinder site, in the
    launch configuration it times (packed layout, graph replay; FP64
    product, and the bound FP32 / BF16 products with their default tiles),
    against the dense oracle on 16 sampled output rows (first and last rows
    of the largest sectors, seeded random ones): FP64 1e-12, FP32 3e-5 of
    the largest sampled entry on operands rounded to FP32, BF16 the
    element-wise rounding model of test_gpu_parity.bf16_bound on operands
    rounded to BF16."""
    from paper_1501_05504_amd import synth
    from tests.test_gpu_parity import bf16_bound, bf16_round
    m, qL, dL, qR, dR, W, wq, phys = _site_case()
    w, d = W.shape[0], 4
    plan = abi.BlockPlan(ctx, 2, d, w, w, qL, dL, qR, dR, phys, wq, wq, layout=abi.LAYOUT_PACKED)
    lb, nl = _env_blocks(qL, dL, wq)
    rbk, nr = _env_blocks(qR, dR, wq)
    sb, ns = _site_blocks(qL, dL, qR, dR, phys)
    assert (plan.nl, plan.nr, plan.npsi) == (nl, nr, ns)
    Lp = synth.gaussian((nl,), synth.SEED_LEFT) / m
    Rp = synth.gaussian((nr,), synth.SEED_RIGHT) / m
    pp = synth.gaussian((ns,), synth.SEED_PSI)
    tt = lambda a: torch.tensor(a, dtype=torch.float64, device=DEV)
    Ld, Rd, pd, Wd = tt(Lp), tt(Rp), tt(pp), tt(W)
    outs = {}
    y = torch.empty(ns, dtype=torch.float64, device=DEV)
    for _ in range(2):
        plan.apply(Ld, Wd, Rd, pd, y, use_graph=True)
    torch.cuda.synchronize()
    outs["f64"] = y.cpu().numpy().copy()
    for name, prec in (("f32", abi.F32), ("bf16", abi.BF16)):
        plan.bind(Ld, Wd, Rd, prec)
        for _ in range(2):
            plan.apply_bound(pd, y, use_graph=True)
        torch.cuda.synchronize()
        outs[name] = y.cpu().numpy().copy()
    plan.close()
    del Ld, Rd, pd, y
    oL = np.concatenate([[0], np.cumsum(dL)])
    oR = np.concatenate([[0], np.cumsum(dR)])
    big = np.argsort(-dL)[:3]
    rows = sorted({int(oL[i]) for i in big} | {int(oL[i + 1] - 1) for i in big} |
                  set(np.random.default_rng(4096).integers(0, m, 10).tolist()))
    # dense R and psi, sampled rows of L and of the outputs
    R = np.zeros((m, w, m))
    for j, v, jp, off in rbk:
        R[oR[j]:oR[j + 1], v, oR[jp]:oR[jp + 1]] = Rp[off:off + dR[j] * dR[jp]].reshape(dR[j], dR[jp])
    psi = np.zeros((m, d, m))
    for i, s, j, off in sb:
        psi[oL[i]:oL[i + 1], s, oR[j]:oR[j + 1]] = pp[off:off + dL[i] * dR[j]].reshape(dL[i], dR[j])
    row_sec = np.searchsorted(oL, np.asarray(rows), side="right") - 1
    Lr = np.zeros((len(rows), w, m))
    for r, (a, i) in enumerate(zip(rows, row_sec)):
        for ii, ww, ip, off in lb:
            if ii == i:
                blk = Lp[off:off + dL[i] * dL[ip]].reshape(dL[i], dL[ip])
                Lr[r, ww, oL[ip]:oL[ip + 1]] = blk[a - oL[i]]

    def out_rows(v):
        o = np.zeros((len(rows), d, m))
        for r, (a, i) in enumerate(zip(rows, row_sec)):
            for ii, s, j, off in sb:
                if ii == i:
                    o[r, s, oR[j]:oR[j + 1]] = v[off:off + dL[i] * dR[j]].reshape(dL[i], dR[j])[a - oL[i]]
        return o
    ref = C.apply_heff(Lr, W, R, psi)
    assert rel_err(out_rows(outs["f64"]), ref) < 1e-12
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    Wf = r32(W)
    ref32 = C.apply_heff(r32(Lr), Wf, r32(R), r32(psi))
    assert rel_err(out_rows(outs["f32"]), ref32) < 3e-5
    Lb, Rb, pb = bf16_round(Lr), bf16_round(R), bf16_round(psi)
    del R
    got = out_rows(outs["bf16"])
    refb = C.apply_heff(Lb, Wf, Rb, pb)
    assert np.all(np.abs(got - refb) <= bf16_bound(Lb, Wf, Rb, pb))
