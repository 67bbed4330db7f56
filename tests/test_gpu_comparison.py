"""GPU parity of the comparison methods' local operations against the CPU
FP64 oracle: the two-site H_eff, its truncated SVD split, and the
centre-matrix (CWF) H application with its enlarged environment.
Tolerances as for the single-site product: FP64 1e-12 relative to the
largest output, FP32 3e-5 (sums of at most a few 10^4 terms at 6e-8 unit
roundoff).
"""
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


TWO_SITE = [  # (ml, d, mr, wl, wc, wr): tiny, boundary MPO bonds, ragged tails, several tiles
    (1, 2, 1, 1, 5, 1),
    (3, 2, 5, 5, 5, 5),
    (17, 4, 9, 6, 6, 6),
    (40, 2, 33, 5, 5, 1),
    (33, 4, 40, 1, 6, 6),
    (130, 4, 70, 6, 6, 6),
    (64, 3, 64, 8, 8, 8),
    (20, 4, 20, 18, 18, 18),
]


def _two_site_inputs(ml, d, mr, wl, wc, wr, seed=0):
    return (synth.gaussian((ml, wl, ml), 10 + seed), synth.gaussian((wl, wc, d, d), 20 + seed),
            synth.gaussian((wc, wr, d, d), 30 + seed), synth.gaussian((mr, wr, mr), 40 + seed),
            synth.gaussian((ml, d, d, mr), 50 + seed))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", TWO_SITE, ids=[str(s) for s in TWO_SITE])
def test_apply_heff_two_site(ctx, shape, prec):
    ml, d, mr, wl, wc, wr = shape
    L, W1, W2, R, psi2 = _two_site_inputs(*shape)
    ref = C.apply_heff_two_site(L, W1, W2, R, psi2)
    t = torch.float64 if prec == "f64" else torch.float32
    out = torch.full((ml, d, d, mr), float("nan"), dtype=t, device=DEV)
    ctx.apply_heff_two_site(dev(L, t), dev(W1, t), dev(W2, t), dev(R, t), dev(psi2, t), out)
    torch.cuda.synchronize()
    assert rel_err(out.double().cpu().numpy(), ref) < (1e-12 if prec == "f64" else 3e-5)


def test_apply_heff_two_site_rejects_bad_calls(ctx):
    L, W1, W2, R, psi2 = _two_site_inputs(4, 2, 4, 5, 5, 5)
    psi_d = dev(psi2)
    with pytest.raises(abi.D3SError):
        ctx.apply_heff_two_site(dev(L), dev(W1), dev(W2), dev(R), psi_d, psi_d)     # aliasing
    with pytest.raises(ValueError):
        ctx.apply_heff_two_site(dev(L, torch.bfloat16), dev(W1), dev(W2), dev(R), dev(psi2, torch.bfloat16),
                                torch.empty_like(psi_d))


CWF = [  # (ml, d, mr, wl, wr)
    (1, 2, 1, 1, 5),
    (5, 2, 7, 5, 5),
    (37, 4, 53, 6, 6),
    (70, 4, 130, 1, 6),
    (130, 4, 70, 6, 1),
    (64, 2, 64, 8, 8),
    (40, 4, 40, 18, 18),
]


@pytest.mark.parametrize("shape", CWF, ids=[str(s) for s in CWF])
def test_cwf_environment_and_application(ctx, shape):
    ml, d, mr, wl, wr = shape
    L = synth.gaussian((ml, wl, ml), 61)
    W = synth.gaussian((wl, wr, d, d), 62)
    R = synth.gaussian((mr, wr, mr), 63)
    Cm = synth.gaussian((ml * d, mr), 64)
    Lt_ref = C.cwf_environment(L, W)
    Lt = torch.full((ml * d, wr, ml * d), float("nan"), dtype=torch.float64, device=DEV)
    ctx.cwf_environment(dev(L), dev(W), Lt)
    torch.cuda.synchronize()
    assert rel_err(Lt.cpu().numpy(), Lt_ref) < 1e-13
    ref = C.apply_cwf(Lt_ref, R, Cm)
    for t, tol in ((torch.float64, 1e-12), (torch.float32, 3e-5)):
        out = torch.full((ml * d, mr), float("nan"), dtype=t, device=DEV)
        ctx.apply_cwf(Lt.to(t).contiguous(), dev(R, t), dev(Cm, t), out)
        torch.cuda.synchronize()
        assert rel_err(out.double().cpu().numpy(), ref) < tol


def test_cwf_equals_single_site_product_at_full_size(ctx):
    """The CWF application and the single-site product are the same operator
    (a property that holds at any size), checked at the measured size of the
    comparison (Fermi-Hubbard MPO shape d = 4, w = 6, m = 1024), and sampled
    output rows against the oracle's single-site product."""
    ml = mr = 1024
    d, w = 4, 6
    g = torch.Generator(device="cpu").manual_seed(71)
    L = torch.randn((ml, w, ml), generator=g, dtype=torch.float64).to(DEV)
    W = torch.randn((w, w, d, d), generator=g, dtype=torch.float64).to(DEV)
    R = torch.randn((mr, w, mr), generator=g, dtype=torch.float64).to(DEV)
    psi = torch.randn((ml, d, mr), generator=g, dtype=torch.float64).to(DEV)
    Lt = torch.empty((ml * d, w, ml * d), dtype=torch.float64, device=DEV)
    ctx.cwf_environment(L, W, Lt)
    out_cwf = torch.empty((ml * d, mr), dtype=torch.float64, device=DEV)
    ctx.apply_cwf(Lt, R, psi.view(ml * d, mr), out_cwf)
    out = torch.empty((ml, d, mr), dtype=torch.float64, device=DEV)
    ctx.apply_heff(L, W, R, psi, out)
    torch.cuda.synchronize()
    a, b = out_cwf.cpu().numpy(), out.view(ml * d, mr).cpu().numpy()
    assert rel_err(a, b) < 1e-12
    Lh, Wh, Rh, ph = (t.cpu().numpy() for t in (L, W, R, psi))
    for row in (0, 517, ml - 1):
        ref = C.apply_heff(Lh[row:row + 1], Wh, Rh, ph).reshape(d, mr)
        assert rel_err(a[row * d:(row + 1) * d], ref) < 1e-12


def test_two_site_full_size_sampled_rows(ctx):
    """Two-site product at the measured size (d = 4, w = 6, m = 1024) on rows
    the oracle computes one left index at a time."""
    ml = mr = 1024
    d, w = 4, 6
    g = torch.Generator(device="cpu").manual_seed(72)
    L = torch.randn((ml, w, ml), generator=g, dtype=torch.float64)
    W1 = torch.randn((w, w, d, d), generator=g, dtype=torch.float64)
    W2 = torch.randn((w, w, d, d), generator=g, dtype=torch.float64)
    R = torch.randn((mr, w, mr), generator=g, dtype=torch.float64)
    psi2 = torch.randn((ml, d, d, mr), generator=g, dtype=torch.float64)
    out = torch.empty((ml, d, d, mr), dtype=torch.float64, device=DEV)
    ctx.apply_heff_two_site(L.to(DEV), W1.to(DEV), W2.to(DEV), R.to(DEV), psi2.to(DEV), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    Lh, W1h, W2h, Rh, ph = (t.numpy() for t in (L, W1, W2, R, psi2))
    for a in (0, 389, ml - 1):
        ref = C.apply_heff_two_site(Lh[a:a + 1], W1h, W2h, Rh, ph)
        assert rel_err(got[a:a + 1], ref) < 1e-12


@pytest.mark.parametrize("shape", [(6, 2, 5, 3), (40, 4, 33, 50), (64, 2, 64, 200)],
                         ids=["tiny", "ragged", "kmax"])
def test_two_site_split(ctx, shape):
    """The split of a two-site tensor through d3s_truncate without a
    neighbour: the singular values, the kept product (unique: the rank-k
    approximation) and the isometry, in both directions."""
    ml, d, mr, kmax = shape
    psi2 = synth.gaussian((ml, d, d, mr), 81)
    A_ref, SVt_ref, s_ref, disc_ref = C.two_site_split(psi2, kmax, 0.0)
    k_ref = A_ref.shape[2]
    approx_ref = A_ref.reshape(ml * d, k_ref) @ SVt_ref.reshape(k_ref, d * mr)
    mat = dev(psi2.reshape(ml * d, d * mr))
    n = ml * d
    site = torch.empty(n * min(kmax, n), dtype=torch.float64, device=DEV)
    right = torch.empty(min(kmax, n) * d * mr, dtype=torch.float64, device=DEV)
    k, disc, s = ctx.truncate(abi.L2R, mat, mat.view(ml, d, d * mr), kmax, 0.0, None, site, right,
                              renormalize=False)
    assert k == k_ref
    assert np.allclose(s[:min(n, d * mr)], s_ref, rtol=0, atol=1e-10 * s_ref[0])
    assert abs(disc - disc_ref) <= 1e-10 * float(np.sum(s_ref ** 2))
    A = site[:n * k].view(n, k).cpu().numpy()
    SVt = right[:k * d * mr].view(k, d * mr).cpu().numpy()
    assert np.allclose(A.T @ A, np.eye(k), atol=1e-10)
    assert rel_err(A @ SVt, approx_ref) < 1e-9
    # right to left: the new site is V_k^T, the left part U_k S_k
    nr = d * mr
    site_r = torch.empty(nr * min(kmax, nr), dtype=torch.float64, device=DEV)
    left = torch.empty(ml * d * min(kmax, nr), dtype=torch.float64, device=DEV)
    k2, _, _ = ctx.truncate(abi.R2L, mat, mat.view(ml * d, d, mr), kmax, 0.0, None, site_r, left,
                            renormalize=False)
    assert k2 == k_ref
    B = site_r[:k2 * nr].view(k2, nr).cpu().numpy()
    US = left[:ml * d * k2].view(ml * d, k2).cpu().numpy()
    assert np.allclose(B @ B.T, np.eye(k2), atol=1e-10)
    assert rel_err(US @ B, approx_ref) < 1e-9
