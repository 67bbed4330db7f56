"""Parity at the measured sizes, in the launch configuration bench.py times
(default tile rule: 256x128 tiles, the steady-state K loop), on output rows
the CPU FP64 oracle computes one left index at a time; and the argument
checks at the edges of the accepted sizes.
Tolerances as for the small shapes: FP64 1e-12, FP32 3e-5 relative to the
largest entry of the sampled rows, BF16 the element-wise rounding model of
test_gpu_parity.bf16_bound.  64 rows are sampled: the first and last, both
sides of GEMM tile boundaries (256-row tiles of the (a, w) rows of the first
GEMM and of the (a, s) rows of the second), and seeded random ones.
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
