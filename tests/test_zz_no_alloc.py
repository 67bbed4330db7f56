"""The allocation-free H_eff entry point (d3s_apply_heff_noalloc) through the
C-ABI against d3s_apply_heff on the same inputs: two calls in a row on one
context, the second on a smaller problem (the scratch array keeps the first
call's contents), every precision, a product too large for the scratch
rejected before any launch, and no device memory taken by the call."""
import numpy as np
import pytest
import torch

from paper_1501_05504_amd import synth

pytestmark = pytest.mark.gpu

abi = pytest.importorskip("paper_1501_05504_amd.abi")

DEV = torch.device("cuda:0")

# FP64: sums of <= 1e4 unit-scale products; FP32: K <= 2e3 terms at 6e-8;
# BF16: both calls round the same BF16 operands (FP32 accumulation), so only
# the split-K order can differ
TOL = {torch.float64: 1e-12, torch.float32: 3e-5, torch.bfloat16: 1e-5}


def _case(ml, d, mr, wl, wr, seed, dtype):
    L = synth.gaussian((ml, wl, ml), seed)
    W = synth.gaussian((wl, wr, d, d), seed + 1)
    R = synth.gaussian((mr, wr, mr), seed + 2)
    psi = synth.gaussian((ml, d, mr), seed + 3)
    t = lambda a, dt: torch.tensor(a, dtype=torch.float64, device=DEV).to(dt).contiguous()
    wdt = torch.float64 if dtype == torch.float64 else torch.float32
    odt = torch.float64 if dtype == torch.float64 else torch.float32
    return t(L, dtype), t(W, wdt), t(R, dtype), t(psi, dtype), odt


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_noalloc_equals_apply_heff_twice(dtype):
    ctx = abi.Context(0)
    for shape, seed in [((300, 4, 257, 6, 6), 7), ((37, 4, 53, 6, 6), 8)]:
        ml, d, mr, wl, wr = shape
        L, W, R, psi, odt = _case(ml, d, mr, wl, wr, seed, dtype)
        ref = torch.empty((ml, d, mr), dtype=odt, device=DEV)
        got = torch.full((ml, d, mr), float("nan"), dtype=odt, device=DEV)
        ctx.apply_heff(L, W, R, psi, ref)
        ctx.apply_heff_noalloc(L, W, R, psi, got)
        torch.cuda.synchronize()
        r, g = ref.cpu().double().numpy(), got.cpu().double().numpy()
        assert np.isfinite(g).all()
        assert np.abs(g - r).max() <= TOL[dtype] * np.abs(r).max()
    ctx.close()


def test_noalloc_rejects_products_beyond_the_scratch():
    ctx = abi.Context(0)
    ml = mr = 512        # FP64, d = 4, w = 6: about 104 MiB of intermediates
    L, W, R, psi, odt = _case(ml, 4, mr, 6, 6, 3, torch.float64)
    out = torch.zeros((ml, 4, mr), dtype=odt, device=DEV)
    with pytest.raises(abi.D3SError) as e:
        ctx.apply_heff_noalloc(L, W, R, psi, out)
    assert e.value.status == abi.EINVAL
    assert "scratch" in str(e.value)
    assert float(out.abs().max()) == 0.0
    ctx.close()


def test_noalloc_takes_no_device_memory():
    """A fresh context whose only work is the allocation-free product leaves
    the device's free memory unchanged (the kernels were loaded by a product
    on another context first)."""
    warm = abi.Context(0)
    ml, d, mr, wl, wr = 200, 4, 200, 6, 6
    L, W, R, psi, odt = _case(ml, d, mr, wl, wr, 11, torch.float64)
    ref = torch.empty((ml, d, mr), dtype=odt, device=DEV)
    out = torch.empty((ml, d, mr), dtype=odt, device=DEV)
    warm.apply_heff(L, W, R, psi, ref)
    warm.apply_heff_noalloc(L, W, R, psi, out)
    torch.cuda.synchronize()
    ctx = abi.Context(0)
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        ctx.apply_heff_noalloc(L, W, R, psi, out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    # the intermediates alone would take ~30 MiB
    assert abs(free0 - free1) < (2 << 20)
    assert np.abs(out.cpu().numpy() - ref.cpu().numpy()).max() <= 1e-12 * np.abs(ref.cpu().numpy()).max()
    ctx.close()
    warm.close()
