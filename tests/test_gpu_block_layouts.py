"""Block plans of the packed layout (only the allowed blocks, the layout of
the block sweeps) and the bound low-precision product of the eigensolver
(d3s_block_plan_bind / d3s_apply_heff_blocks_bound), against the dense CPU
oracle.  The packing below is written from the layout's definition in the
header (blocks in the order of the left sector, then the physical state or
channel; each block row-major)."""
import numpy as np
import pytest
import torch

from oracle import contract as C

from tests.test_gpu_blocks import dev, hubbard_block_case, rel_err

pytestmark = pytest.mark.gpu

abi = pytest.importorskip("paper_1501_05504_amd.abi")

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    c = abi.Context(0)
    yield c
    c.close()


def offsets(dims):
    return np.concatenate([[0], np.cumsum(dims)]).astype(int)


def sector_of(qs, q):
    for k, x in enumerate(qs):
        if tuple(x) == tuple(q):
            return k
    return -1


def pack_site(psi, qL, dL, qR, dR, phys):
    oL, oR = offsets(dL), offsets(dR)
    out = []
    for i in range(len(dL)):
        for s in range(len(phys)):
            j = sector_of(qR, np.add(qL[i], phys[s]))
            if j >= 0:
                out.append(psi[oL[i]:oL[i + 1], s, oR[j]:oR[j + 1]].ravel())
    return np.concatenate(out)


def unpack_site(v, shape, qL, dL, qR, dR, phys):
    oL, oR = offsets(dL), offsets(dR)
    out = np.zeros(shape)
    p = 0
    for i in range(len(dL)):
        for s in range(len(phys)):
            j = sector_of(qR, np.add(qL[i], phys[s]))
            if j >= 0:
                n = dL[i] * dR[j]
                out[oL[i]:oL[i + 1], s, oR[j]:oR[j + 1]] = v[p:p + n].reshape(dL[i], dR[j])
                p += n
    assert p == len(v)
    return out


def pack_env(E, q, dims, wq):
    o = offsets(dims)
    out = []
    for i in range(len(dims)):
        for w in range(len(wq)):
            ip = sector_of(q, np.subtract(q[i], wq[w]))
            if ip >= 0:
                out.append(E[o[i]:o[i + 1], w, o[ip]:o[ip + 1]].ravel())
    return np.concatenate(out)


def packed_case(ml, mr, seed):
    case = hubbard_block_case(ml, mr, seed)
    qL, dL, qR, dR = case["qL"], case["dL"], case["qR"], case["dR"]
    case["Lp"] = pack_env(case["L"], qL, dL, case["wq"])
    case["Rp"] = pack_env(case["R"], qR, dR, case["wq"])
    case["psip"] = pack_site(case["psi"], qL, dL, qR, dR, case["phys"])
    return case


def make_plan(ctx, case, layout):
    W = case["W"]
    return abi.BlockPlan(ctx, 2, 4, W.shape[0], W.shape[1], case["qL"], case["dL"], case["qR"], case["dR"],
                         case["phys"], case["wq"], case["wq"], layout=layout)


@pytest.mark.parametrize("ml,mr,seed", [(40, 52, 21), (300, 257, 22)])
def test_packed_plan_equals_dense_oracle(ctx, ml, mr, seed):
    """FP64 product of a packed-layout plan: the packed blocks of the
    oracle's dense result, to 1e-12; the sizes match the packing."""
    case = packed_case(ml, mr, seed)
    ref = C.apply_heff(case["L"], case["W"], case["R"], case["psi"])
    plan = make_plan(ctx, case, abi.LAYOUT_PACKED)
    assert (plan.nl, plan.nr, plan.npsi) == (len(case["Lp"]), len(case["Rp"]), len(case["psip"]))
    out = torch.full((plan.npsi,), float("nan"), dtype=torch.float64, device=DEV)
    for use_graph in (False, True):
        plan.apply(dev(case["Lp"]), dev(case["W"]), dev(case["Rp"]), dev(case["psip"]), out, use_graph=use_graph)
        torch.cuda.synchronize()
        got = unpack_site(out.cpu().numpy(), case["psi"].shape, case["qL"], case["dL"], case["qR"], case["dR"],
                          case["phys"])
        assert rel_err(got, ref) < 1e-12
    plan.close()


@pytest.mark.parametrize("layout", ["dense", "packed"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("ml,mr,seed", [(20, 17, 23), (300, 257, 24)])
def test_bound_product_equals_oracle(ctx, layout, prec, ml, mr, seed):
    """The bound low-precision product (FP64 in and out) against the oracle on
    operands rounded as the product rounds them (L, R, psi to the product's
    type, W to FP32): FP32 3e-5 of the largest entry, BF16 the element-wise
    rounding model of test_gpu_parity.bf16_bound; eager and replayed from a
    captured graph; forbidden entries of the dense layout are zero."""
    from tests.test_gpu_parity import bf16_bound, bf16_round
    case = packed_case(ml, mr, seed)
    rnd = bf16_round if prec == "bf16" else (lambda a: np.asarray(a, dtype=np.float32).astype(np.float64))
    Lr, Rr, pr = rnd(case["L"]), rnd(case["R"]), rnd(case["psi"])
    Wf = np.asarray(case["W"], dtype=np.float32).astype(np.float64)
    ref = C.apply_heff(Lr, Wf, Rr, pr)
    lay = abi.LAYOUT_PACKED if layout == "packed" else abi.LAYOUT_DENSE
    plan = make_plan(ctx, case, lay)
    if layout == "packed":
        L, R, psi = case["Lp"], case["Rp"], case["psip"]
    else:
        L, R, psi = case["L"], case["R"], case["psi"]
    plan.bind(dev(L), dev(case["W"]), dev(R), abi.F32 if prec == "f32" else abi.BF16)
    bound = bf16_bound(Lr, Wf, Rr, pr) if prec == "bf16" else None
    for use_graph in (False, True, True):
        out = torch.full((plan.npsi,), float("nan"), dtype=torch.float64, device=DEV)
        plan.apply_bound(dev(psi), out, use_graph=use_graph)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        if layout == "packed":
            o = unpack_site(o, case["psi"].shape, case["qL"], case["dL"], case["qR"], case["dR"], case["phys"])
        else:
            o = o.reshape(case["psi"].shape)
            assert np.all(o[case["mask"] == 0] == 0.0)
        if bound is None:
            assert rel_err(o, ref) < 3e-5, use_graph
        else:
            assert np.all(np.abs(o - ref) <= bound), use_graph
    plan.close()


def test_autotuned_twin_switches_precision():
    """With the autotuner on, the padded twin built for FP32 products is
    timed again in BF16 when BF16 products follow (its tiles are re-picked
    for that precision); both products still meet their bounds against the
    oracle on rounded operands, and so does FP32 again afterwards."""
    from tests.test_gpu_parity import bf16_bound, bf16_round
    case = packed_case(300, 257, 27)
    c = abi.Context(0)
    try:
        c.set_autotune(True)
        plan = make_plan(c, case, abi.LAYOUT_PACKED)
        Wf = np.asarray(case["W"], dtype=np.float32).astype(np.float64)
        f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
        for prec in ("f32", "bf16", "f32"):
            rnd = bf16_round if prec == "bf16" else f32
            Lr, Rr, pr = rnd(case["L"]), rnd(case["R"]), rnd(case["psi"])
            ref = C.apply_heff(Lr, Wf, Rr, pr)
            plan.bind(dev(case["Lp"]), dev(case["W"]), dev(case["Rp"]), abi.F32 if prec == "f32" else abi.BF16)
            out = torch.full((plan.npsi,), float("nan"), dtype=torch.float64, device=DEV)
            plan.apply_bound(dev(case["psip"]), out)
            torch.cuda.synchronize()
            o = unpack_site(out.cpu().numpy(), case["psi"].shape, case["qL"], case["dL"], case["qR"], case["dR"],
                            case["phys"])
            if prec == "f32":
                assert rel_err(o, ref) < 3e-5
            else:
                assert np.all(np.abs(o - ref) <= bf16_bound(Lr, Wf, Rr, pr))
        plan.close()
    finally:
        c.close()


def test_bind_replaces_the_operator(ctx):
    """A second bind replaces the first (2 L gives twice the product)."""
    case = packed_case(96, 80, 25)
    plan = make_plan(ctx, case, abi.LAYOUT_PACKED)
    psi = dev(case["psip"])
    outs = []
    for scale in (1.0, 2.0):
        plan.bind(dev(scale * case["Lp"]), dev(case["W"]), dev(case["Rp"]), abi.F32)
        out = torch.empty((plan.npsi,), dtype=torch.float64, device=DEV)
        plan.apply_bound(psi, out)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    assert rel_err(outs[1], 2.0 * outs[0]) < 1e-6
    plan.close()


def test_bind_and_layout_errors(ctx):
    """EINVAL: binding for FP64, the bound product with nothing bound, and the
    expansion on a packed-layout plan; nothing is launched."""
    case = packed_case(40, 52, 26)
    plan = make_plan(ctx, case, abi.LAYOUT_PACKED)
    L, W, R, psi = dev(case["Lp"]), dev(case["W"]), dev(case["Rp"]), dev(case["psip"])
    out = torch.empty((plan.npsi,), dtype=torch.float64, device=DEV)
    with pytest.raises(abi.D3SError) as e:
        plan.apply_bound(psi, out)
    assert e.value.status == abi.EINVAL
    with pytest.raises(abi.D3SError) as e:
        plan.bind(L, W, R, abi.F64)
    assert e.value.status == abi.EINVAL
    Mt = torch.empty(plan.npsi * 8, dtype=torch.float64, device=DEV)
    st = abi._expand_blocks(ctx.h, plan.h, abi.L2R, abi._ptr(L), abi._ptr(W), abi._ptr(psi), 1e-3, abi._ptr(Mt))
    assert st == abi.EINVAL and b"dense layout" in abi._last_error(ctx.h)
    plan.close()
