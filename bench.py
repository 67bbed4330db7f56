"""H_eff * psi microbenchmark of the DMRG3S hot path on one MI355X.

Workload (the isolated H_eff microbenchmark): Fermi-Hubbard chain MPO
(t = 1, U = 8, d = 4, w = 6, Jordan-Wigner strings); environments L and R
built on the GPU by contracting a seeded Gaussian MPS of ceil(log_4 m) sites,
left- (right-) canonicalised through the library's truncation, with the MPO
from the chain ends; psi[m, 4, m] Gaussian and normalised.  One step = one
application of H_eff (GEMM over the left MPS bond, W-map, GEMM over the right
MPO and MPS bonds).  Inputs are resident in HBM when timing starts.

Prints one JSON line.  `value` is FP64 GFLOP/s at the default m = 2048 with
the flop count F = 2 wl d ml^2 mr + 2 d^2 wl wr ml mr + 2 wr d ml mr^2.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2516.6e12}
HBM_PEAK = 8.0e12

# HBM bytes per launch of the FP64 H_eff GEMMs at m = 2048 from the rocprofv3
# FETCH_SIZE / WRITE_SIZE passes (scaled by a 1 GiB copy reference), valid
# only for the sources they were taken on (first 16 hex digits of the
# SHA-256 of the GEMM kernels and their host set-up); any other source
# reports null.
TRAFFIC = {"src_sha": "50b046a66d731906", "m": 2048,
           "gemm1": 4.163e9 + 0.940e9, "gemm2": 4.617e9 + 0.134e9}


def gemm_source_sha():
    """SHA-256 (first 16 hex digits) of the sources that decide the measured
    H_eff launches: the GEMM kernels and the host code that sets them up."""
    import hashlib
    h = hashlib.sha256()
    for name in ("gemm.hip", "mfma_tile.h", "ops.hip"):
        with open(os.path.join(ROOT, "paper_1501_05504_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def heff_flops(ml, d, mr, wl, wr):
    return 2.0 * wl * d * ml * ml * mr + 2.0 * d * d * wl * wr * ml * mr + 2.0 * wr * d * ml * mr * mr


def gemm_flops(ml, d, mr, wl, wr):
    return {"gemm1": 2.0 * (ml * wl) * (d * mr) * ml, "wmap": 2.0 * d * d * wl * wr * ml * mr,
            "gemm2": 2.0 * (ml * d) * mr * (wr * mr)}


def build_inputs(ctx, abi, synth, torch, m, dev):
    """L, W, R (FP64, device) of the microbenchmark, built by the library."""
    d = 4
    ns = synth.env_sites_for(m, d)
    mpo = abi.hubbard_chain_mpo(2 * ns + 1, t=1.0, U=8.0)
    W = torch.tensor(mpo[ns], dtype=torch.float64, device=dev)

    def canonical(tensors, direction):
        out = []
        for t in tensors:
            x = torch.tensor(t, dtype=torch.float64, device=dev)
            ml_, d_, mr_ = x.shape
            if direction == abi.L2R:
                k = mr_
                site = torch.empty(ml_ * d_ * k, dtype=torch.float64, device=dev)
                dummy = torch.zeros(mr_, dtype=torch.float64, device=dev)
                nb = torch.empty(k, dtype=torch.float64, device=dev)
                kk, _, _ = ctx.truncate(abi.L2R, x.reshape(ml_ * d_, mr_), x, k, 0.0, dummy, site, nb,
                                        renormalize=False)
                if kk != min(ml_ * d_, mr_):
                    raise RuntimeError("left-canonicalisation lost rank: %d of %d" % (kk, min(ml_ * d_, mr_)))
                out.append(site[: ml_ * d_ * kk].reshape(ml_, d_, kk))
            else:
                k = ml_
                site = torch.empty(k * d_ * mr_, dtype=torch.float64, device=dev)
                dummy = torch.zeros(ml_, dtype=torch.float64, device=dev)
                nb = torch.empty(k, dtype=torch.float64, device=dev)
                kk, _, _ = ctx.truncate(abi.R2L, x.reshape(ml_, d_ * mr_), x, k, 0.0, dummy, site, nb,
                                        renormalize=False)
                if kk != min(ml_, d_ * mr_):
                    raise RuntimeError("right-canonicalisation lost rank: %d of %d" % (kk, min(ml_, d_ * mr_)))
                out.append(site[: kk * d_ * mr_].reshape(kk, d_, mr_))
        return out

    left = canonical(synth.growing_mps(ns, d, m, synth.SEED_LEFT), abi.L2R)
    L = torch.ones(1, dtype=torch.float64, device=dev).reshape(1, 1, 1)
    for i, A in enumerate(left):
        wl, wr = mpo[i].shape[0], mpo[i].shape[1]
        out = torch.empty((A.shape[2], wr, A.shape[2]), dtype=torch.float64, device=dev)
        ctx.update_env(abi.L2R, L, torch.tensor(mpo[i], dtype=torch.float64, device=dev), A, out)
        L = out
    # right environment: mirror image of a growing MPS, attached to the right end
    right_src = [t.transpose(2, 1, 0).copy() for t in reversed(synth.growing_mps(ns, d, m, synth.SEED_RIGHT))]
    right = canonical(right_src, abi.R2L)
    R = torch.ones(1, dtype=torch.float64, device=dev).reshape(1, 1, 1)
    for j in range(ns - 1, -1, -1):
        site_idx = ns + 1 + j
        B = right[j]
        wl = mpo[site_idx].shape[0]
        out = torch.empty((B.shape[0], wl, B.shape[0]), dtype=torch.float64, device=dev)
        ctx.update_env(abi.R2L, R, torch.tensor(mpo[site_idx], dtype=torch.float64, device=dev), B, out)
        R = out
    torch.cuda.synchronize()
    return L.contiguous(), W.contiguous(), R.contiguous()


def time_heff(ctx, torch, L, W, R, psi, out, steps, warmup):
    for _ in range(warmup):
        ctx.apply_heff(L, W, R, psi, out)
    torch.cuda.synchronize()
    ctx.profile_begin(steps)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        ctx.apply_heff(L, W, R, psi, out)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, n = ctx.profile_end()
    ms = start.elapsed_time(stop) / steps
    return ms, wall, [k / max(n, 1) for k in kern_ms]


def block_heff_bench(ctx, abi, synth, torch, np, m, dev, steps):
    """Block-sparse H_eff (U(1)xU(1) Hubbard MPO): sectors with dimensions
    ~ exp(-(N-N0)^2/18 - (2Sz)^2/18) normalised to m on both bonds (uneven
    blocks, 100+ sectors), charge-conserving Gaussian L, R, psi; graph replay."""
    qL, dL = synth.gaussian_sectors((32, 0), (3.0, 3.0), m, (10, 10))
    qR, dR = synth.gaussian_sectors((33, 1), (3.0, 3.0), m, (10, 10))
    W = abi.hubbard_chain_mpo(3, t=1.0, U=8.0)[1]
    wq = abi.mpo_fermion_charges(1)
    phys = np.array(abi.HUBBARD_CHARGES)
    sl, sr = synth.expand_charges(qL, dL), synth.expand_charges(qR, dR)
    L = torch.tensor(synth.gaussian((m, 6, m), synth.SEED_LEFT) * synth.mask_env(sl, wq) / m, device=dev)
    R = torch.tensor(synth.gaussian((m, 6, m), synth.SEED_RIGHT) * synth.mask_env(sr, wq) / m, device=dev)
    psi = torch.tensor(synth.gaussian((m, 4, m), synth.SEED_PSI) * synth.mask_site(sl, phys, sr), device=dev)
    Wd = torch.tensor(W, device=dev)
    out = torch.empty_like(psi)
    plan = abi.BlockPlan(ctx, 2, 4, 6, 6, qL, dL, qR, dR, phys, wq, wq)
    res = {}
    for graph in (True, False):
        for _ in range(3):
            plan.apply(L, Wd, R, psi, out, use_graph=graph)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            plan.apply(L, Wd, R, psi, out, use_graph=graph)
        b.record()
        torch.cuda.synchronize()
        res["graph" if graph else "eager"] = a.elapsed_time(b) / steps
    dense = torch.empty_like(psi)
    ctx.apply_heff(L, Wd, R, psi, dense)
    torch.cuda.synchronize()
    err = float((dense - out).abs().max() / dense.abs().max())
    ms = res["graph"]
    info = {"m": m, "sectors_left": len(dL), "sectors_right": len(dR), "tasks": plan.ntasks,
            "block_gflop": round(plan.flops / 1e9, 2), "ms_graph": round(ms, 4), "ms_eager": round(res["eager"], 4),
            "gflops": round(plan.flops / ms * 1e-6, 1),
            "dense_flop_ratio": round(heff_flops(m, 4, m, 6, 6) / plan.flops, 1),
            "max_rel_diff_vs_dense": err}
    plan.close()
    return info


def cylinder_site_bench(ctx, abi, synth, torch, np, m, dev, steps):
    """Block-sparse H_eff of a middle site of the 4-leg Hubbard cylinder MPO
    (w = 18, d = 4) at bond dimension m, U(1)xU(1) sectors of Gaussian
    weight exp(-(N-N0)^2/(2 1.5^2) - (2Sz)^2/(2 1.5^2)) normalised to m on
    both bonds (45 sectors at m = 4096, as at the middle bond of the
    cylinder sweeps), tensors in the packed layout the sweeps use (Gaussian
    entries).  FP64: the plan's product; FP32 / BF16: the eigensolver's
    product (operator bound once, FP64 vector in and out, conversions
    included).  Graph replay, events around `steps` products.  Reports the
    rate against each precision's dense MFMA peak and the time against the
    HBM floor of this three-kernel scheme (operands read once, output
    written once, the T1 and T2 intermediates each written and read once)."""
    qL, dL = synth.gaussian_sectors((28, 0), (1.5, 1.5), m, (8, 8))
    qR, dR = synth.gaussian_sectors((29, 1), (1.5, 1.5), m, (8, 8))
    mpo = abi.hubbard_cylinder_mpo(4, 16, t=1.0, U=4.0)
    W = mpo[len(mpo) // 2]
    w = int(W.shape[0])
    wq = abi.mpo_fermion_charges(4)
    phys = np.array(abi.HUBBARD_CHARGES)
    plan = abi.BlockPlan(ctx, 2, 4, w, w, qL, dL, qR, dR, phys, wq, wq, layout=abi.LAYOUT_PACKED)
    L = torch.tensor(synth.gaussian((plan.nl,), synth.SEED_LEFT) / m, device=dev)
    R = torch.tensor(synth.gaussian((plan.nr,), synth.SEED_RIGHT) / m, device=dev)
    psi = torch.tensor(synth.gaussian((plan.npsi,), synth.SEED_PSI), device=dev)
    Wd = torch.tensor(W, device=dev)
    # allowed elements of the intermediates T1[a,w,t,y] and T2[a,s,v,y]
    key = {tuple(q): k for k, q in enumerate(np.asarray(qL).tolist())}
    keyr = {tuple(q): k for k, q in enumerate(np.asarray(qR).tolist())}
    nt1 = nt2 = 0
    for i, q in enumerate(np.asarray(qL).tolist()):
        for c in np.asarray(wq).tolist():
            ip = key.get((q[0] - c[0], q[1] - c[1]))
            if ip is None:
                continue
            qp = np.asarray(qL)[ip]
            for t in phys.tolist():
                jp = keyr.get((int(qp[0]) + t[0], int(qp[1]) + t[1]))
                if jp is not None:
                    nt1 += int(dL[i]) * int(dR[jp])
        for sg in phys.tolist():
            j = keyr.get((q[0] + sg[0], q[1] + sg[1]))
            if j is None:
                continue
            for c in np.asarray(wq).tolist():
                jpp = keyr.get((int(qR[j][0]) - c[0], int(qR[j][1]) - c[1]))
                if jpp is not None:
                    nt2 += int(dL[i]) * int(dR[jpp])
    out = {"workload": "block_heff_hubbard_cylinder_site", "m": m, "d": 4, "w": w, "sectors_left": len(dL),
           "sectors_right": len(dR), "tasks": plan.ntasks, "gflop": round(plan.flops / 1e9, 2),
           "layout": "packed", "steps": steps}
    ref = torch.empty((plan.npsi,), dtype=torch.float64, device=dev)
    for name in ("f64", "f32", "bf16"):
        y = torch.empty_like(ref)
        if name == "f64":
            run = lambda: plan.apply(L, Wd, R, psi, y, use_graph=True)
            esz, tsz = 8, 8
        else:
            plan.bind(L, Wd, R, abi.F32 if name == "f32" else abi.BF16)
            run = lambda: plan.apply_bound(psi, y, use_graph=True)
            esz, tsz = (4, 4) if name == "f32" else (2, 4)
        for _ in range(3):
            run()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            run()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        if name == "f64":
            ref.copy_(y)
        # operands once (the low-precision ones in their type, psi and out in
        # FP64 around the conversions), T1 (FP32 or FP64) and T2 (the operand
        # type) written and read once
        byt = esz * (plan.nl + plan.nr) + 8 * 2 * plan.npsi + 2 * tsz * nt1 + 2 * esz * nt2
        floor_ms = byt / HBM_PEAK * 1e3
        tf = plan.flops / ms * 1e-9
        out[name] = {"ms": round(ms, 4), "tflops": round(tf, 2),
                     "pct_mfma_peak": round(100.0 * tf * 1e12 / PEAK[name], 2),
                     "hbm_floor_ms": round(floor_ms, 4), "frac_of_hbm_floor": round(floor_ms / ms, 3),
                     "max_rel_diff_vs_f64": float((y - ref).abs().max() / ref.abs().max())}
        print("bench: cylinder site %s %.4f ms %.1f TFLOP/s (%.1f%% of peak; HBM floor %.4f ms)"
              % (name, ms, tf, out[name]["pct_mfma_peak"], floor_ms), file=sys.stderr, flush=True)
    plan.close()
    return out


def hubbard_sweep_bench(ctx, abi, synth, torch, dev, l, sched, U, tol, lanczos_tol, max_final, growth_tol,
                        mixed_min_gflop):
    """DMRG3S block sweeps on the Hubbard chain (t = 1, half filling, 2Sz = 0)
    from one seeded symmetric state with a growing bond limit: two sweeps at
    each m of the schedule, then sweeps at the last m until the normalised
    sweep energy change is below `tol`.  Once the bonds stay below the
    current limit (the truncation, not the limit, sets them) larger limits
    change nothing and the run moves to the final stage.  The growth sweeps
    solve the local problems to `growth_tol`, the final ones to
    `lanczos_tol`.  Plain FP64 products against FP32 products with FP64
    refinement of every Ritz vector to the same residual tolerance (at every
    site whose product costs at least `mixed_min_gflop`; 0 = all sites); wall
    time from the first environment build on."""
    out = {"workload": "hubbard_chain_blocks", "l": l, "U": U, "filling": "half, 2Sz=0", "m_schedule": sched,
           "tol": tol, "lanczos_tol": lanczos_tol, "growth_lanczos_tol": growth_tol}
    phys = abi.HUBBARD_CHARGES
    mpo = abi.hubbard_chain_mpo(l, t=1.0, U=U)
    for name, prec in (("f64", abi.F64), ("mixed_f32", abi.F32)):
        tensors, secs = synth.random_symmetric_mps(l, phys, [l, 0], sched[0], seed=synth.SEED_MPS)
        st = abi.State(mpo, tensors, max(sched), device=dev)
        sym = abi.Symmetry(phys, abi.mpo_bond_charges(mpo, abi.mpo_fermion_charges(1)), secs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0 = ctx.prepare_blocks(st, sym)
        params = abi.sweep_params(alpha=1e-3, e_before=e0, prec=prec, tol=lanczos_tol)
        if prec != abi.F64:
            params.mixed_min_gflop = mixed_min_gflop
        energies, t_conv, prev, nsweeps, mv, mv64 = [], None, None, 0, 0, 0
        plan = [(m, 2) for m in sched[:-1]] + [(sched[-1], max_final)]
        saturated = False
        for m, count in plan:
            final = m == sched[-1]
            if saturated and not final:
                continue
            params.m_limit = m
            params.lanczos_tol = lanczos_tol if final else growth_tol
            for _ in range(count):
                _, stats, recs = ctx.sweep_blocks(st, sym, params, use_graph=True)
                nsweeps += 1
                mv += sum(r.matvecs for r in recs)
                mv64 += sum(r.f64_matvecs for r in recs)
                energies.append(stats.energy)
                done = (final and prev is not None and abs(stats.energy - prev) / abs(stats.energy) < tol)
                prev = stats.energy
                if done:
                    t_conv = time.perf_counter() - t0
                    break
            if not final and max(st.m) < m:
                saturated = True
        wall = time.perf_counter() - t0
        split = {k: round(sum(getattr(r, k) for r in recs), 3)
                 for k in ("t_eig", "t_expand", "t_trunc", "t_trunc_eig", "t_env", "t_energy")}
        split["trunc_passes_mean"] = round(sum(r.trunc_passes for r in recs) / len(recs), 2)
        out[name] = {"seconds_to_tol": None if t_conv is None else round(t_conv, 3), "seconds": round(wall, 3),
                     "sweeps": nsweeps, "energy": energies[-1], "matvecs": mv, "f64_matvecs": mv64,
                     "low_precision_share": round(1.0 - mv64 / max(mv, 1), 4),
                     "last_sweep_split_s": split, "max_bond": max(st.m),
                     "sectors_mid_bond": int(sym._nsec[l // 2])}
        print("bench: hubbard sweeps %s: %d sweeps %.2f s  E=%.12f  max bond %d" % (
            name, nsweeps, wall, energies[-1], max(st.m)), file=sys.stderr, flush=True)
        del st
        torch.cuda.empty_cache()
    out["energy_diff"] = abs(out["f64"]["energy"] - out["mixed_f32"]["energy"])
    out["mixed_min_gflop"] = mixed_min_gflop
    return out


def cylinder_bench(ctx, abi, synth, torch, dev, sched, sweeps_last, lanczos_tol, precs, tol):
    """4 x 16 Hubbard cylinder (t = 1, U = 4, N = 56, 2Sz = 0, w = 18, every
    column traversed in the same direction), U(1)xU(1) blocks.  The bond
    grows with FP64 products, one sweep at each limit of the schedule but
    the last; that state is saved (site tensors and sectors), and for every
    precision of the eigensolver's products (FP64; FP32 / BF16 with FP64
    refinement to the same residual) a fresh state is rebuilt from it
    (environments by d3s_prepare_blocks) and swept at the last limit until
    the normalised sweep energy change is below `tol`, at most `sweeps_last`
    sweeps.  Reports per-sweep energies, times and energy changes, the time
    to `tol` (null if not reached), and each mixed run's energy difference
    against the FP64 run, sweep by sweep."""
    width, length = 4, 16
    l = width * length
    mpo = abi.hubbard_cylinder_mpo(width, length, t=1.0, U=4.0)
    phys = abi.HUBBARD_CHARGES
    chan = abi.mpo_bond_charges(mpo, abi.mpo_fermion_charges(width))
    wmax = max(int(b.shape[1]) for b in mpo)
    mmax = max(sched)
    cap = mmax * mmax * wmax // 4
    out = {"workload": "hubbard_cylinder_blocks", "width": width, "length": length, "U": 4.0, "N": 56, "w": wmax,
           "m_schedule": sched, "max_sweeps_at_last_m": sweeps_last, "lanczos_tol": lanczos_tol, "tol": tol}
    tensors, secs = synth.random_symmetric_mps(l, phys, [56, 0], sched[0], seed=synth.SEED_MPS)
    st = abi.State(mpo, tensors, mmax, device=dev, env_cap=cap)
    sym = abi.Symmetry(phys, chan, secs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = ctx.prepare_blocks(st, sym)
    params = abi.sweep_params(alpha=1e-3, e_before=e0, prec=abi.F64, tol=lanczos_tol)
    growth = []
    for m in sched[:-1]:
        params.m_limit = m
        t = time.perf_counter()
        _, stats, recs = ctx.sweep_blocks(st, sym, params, use_graph=True)
        growth.append({"m": m, "seconds": round(time.perf_counter() - t, 3), "energy": stats.energy,
                       "t_eig": round(sum(r.t_eig for r in recs), 3), "t_trunc": round(sum(r.t_trunc for r in recs), 3),
                       "max_bond": max(st.m), "sectors_mid_bond": int(sym._nsec[l // 2])})
        print("bench: cylinder growth m=%d %.2f s E=%.10f" % (m, growth[-1]["seconds"], stats.energy),
              file=sys.stderr, flush=True)
    out["growth_f64"] = {"sweeps": growth, "seconds": round(time.perf_counter() - t0, 3)}
    saved = [t.cpu() for t in st.tensors()]
    saved_secs = [sym.sectors(b) for b in range(l + 1)]
    alpha = params.alpha
    del st
    torch.cuda.empty_cache()
    for name in precs:
        prec = {"f64": abi.F64, "mixed_f32": abi.F32, "mixed_bf16": abi.BF16}[name]
        st = abi.State(mpo, saved, mmax, device=dev, env_cap=cap)
        sym = abi.Symmetry(phys, chan, saved_secs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0 = ctx.prepare_blocks(st, sym)
        params = abi.sweep_params(alpha=alpha, e_before=e0, prec=prec, tol=lanczos_tol)
        params.m_limit = sched[-1]
        rows, prev, t_conv = [], None, None
        for _ in range(sweeps_last):
            t = time.perf_counter()
            _, stats, recs = ctx.sweep_blocks(st, sym, params, use_graph=True)
            dE = None if prev is None else abs(stats.energy - prev) / abs(stats.energy)
            rows.append({"m": sched[-1], "seconds": round(time.perf_counter() - t, 3), "energy": stats.energy,
                         "rel_energy_change": dE, "t_eig": round(sum(r.t_eig for r in recs), 3),
                         "t_trunc": round(sum(r.t_trunc for r in recs), 3),
                         "t_trunc_eig": round(sum(r.t_trunc_eig for r in recs), 3),
                         "trunc_passes_max": max(r.trunc_passes for r in recs),
                         "trunc_passes_mean": round(sum(r.trunc_passes for r in recs) / len(recs), 2),
                         "matvecs": sum(r.matvecs for r in recs), "f64_matvecs": sum(r.f64_matvecs for r in recs),
                         "max_bond": max(st.m), "sectors_mid_bond": int(sym._nsec[l // 2])})
            print("bench: cylinder %s m=%d %.2f s E=%.10f dE=%s" % (name, sched[-1], rows[-1]["seconds"],
                                                                    stats.energy, dE), file=sys.stderr, flush=True)
            prev = stats.energy
            if dE is not None and dE < tol:
                t_conv = time.perf_counter() - t0
                break
        out[name] = {"sweeps": rows, "seconds": round(time.perf_counter() - t0, 3),
                     "seconds_to_tol": None if t_conv is None else round(t_conv, 3)}
        del st
        torch.cuda.empty_cache()
    if "f64" in out:
        for name in precs:
            if name != "f64":
                out[name]["energy_diff_vs_f64"] = [abs(a["energy"] - b["energy"])
                                                   for a, b in zip(out[name]["sweeps"], out["f64"]["sweeps"])]
    return out


def gradient_bench(ctx, abi, synth, torch, dev, l, m_sched, J2, dJ, tol):
    """J1-J2 chain (J1 = 1, open): converge DMRG3S (block sweeps, growing
    bond limit, then to a normalised energy change below `tol`), then dE/dJ2
    through the hand-written adjoint (torch.autograd on the MPO energy),
    against the Hellmann-Feynman value <Psi|sum_i S_i.S_{i+2}|Psi> (the
    energy of the same state under the next-nearest-neighbour MPO) and the
    central finite difference of two further converged runs at J2 -+ dJ,
    warm-started from the converged state.  The convergence runs with FP64
    products and with FP32 products plus FP64 refinement."""
    from paper_1501_05504_amd.autograd import mpo_energy
    phys = abi.SPIN_HALF_CHARGES
    chan = abi.mpo_spin_charges(2)
    mmax = max(m_sched)
    out = {"workload": "j1j2_chain", "l": l, "J1": 1.0, "J2": J2, "m_schedule": m_sched, "dJ": dJ, "tol": tol}

    def converge(mpo, tensors, secs, prec, sched):
        st = abi.State(mpo, tensors, mmax, device=dev)
        sym = abi.Symmetry(phys, abi.mpo_bond_charges(mpo, chan), secs)
        e0 = ctx.prepare_blocks(st, sym)
        params = abi.sweep_params(alpha=1e-3, e_before=e0, prec=prec, tol=1e-12, mixed_min_gflop=0.0)
        prev, n = None, 0
        plan = [(mm, 2) for mm in sched[:-1]] + [(sched[-1], 12)]
        for mm, count in plan:
            params.m_limit = mm
            for _ in range(count):
                _, stats, _ = ctx.sweep_blocks(st, sym, params)
                n += 1
                done = mm == sched[-1] and prev is not None and abs(stats.energy - prev) / abs(stats.energy) < tol
                prev = stats.energy
                if done:
                    break
        return st, sym, stats.energy, n

    for name, prec in (("f64", abi.F64), ("mixed_f32", abi.F32)):
        t0 = time.perf_counter()
        tensors, secs = synth.random_symmetric_mps(l, phys, [0], m_sched[0], seed=synth.SEED_MPS)
        st, sym, E, nsw = converge(abi.j1j2_mpo(l, 1.0, J2), tensors, secs, prec, m_sched)
        t_conv = time.perf_counter() - t0
        conv_tensors = [t.cpu().numpy() for t in st.tensors()]
        conv_secs = [sym.sectors(b) for b in range(l + 1)]
        # adjoint through autograd (dense environments rebuilt by d3s_prepare)
        W0 = [torch.tensor(w, dtype=torch.float64, device=dev) for w in abi.j1j2_mpo(l, 1.0, 0.0)]
        W1 = [torch.tensor(w, dtype=torch.float64, device=dev) for w in abi.j1j2_mpo(l, 1.0, 1.0)]
        j = torch.tensor(J2, dtype=torch.float64, device=dev, requires_grad=True)
        t1 = time.perf_counter()
        Ewf = mpo_energy(ctx, st, [a + j * (b - a) for a, b in zip(W0, W1)])
        Ewf.backward()
        t_grad = time.perf_counter() - t1
        adj = float(j.grad)
        del st
        # Hellmann-Feynman: the same state under the next-nearest-neighbour MPO
        st2 = abi.State(abi.j1j2_mpo(l, 0.0, 1.0), conv_tensors, mmax, device=dev)
        hf = ctx.prepare(st2)
        del st2
        res = {"energy": E, "sweeps": nsw, "seconds_to_converge": round(t_conv, 2), "dE_dJ2_adjoint": adj,
               "hellmann_feynman": hf, "adjoint_minus_hf": abs(adj - hf), "gradient_seconds": round(t_grad, 3)}
        if name == "f64":
            eps = []
            for sgn in (+1, -1):
                _, _, Es, _ = converge(abi.j1j2_mpo(l, 1.0, J2 + sgn * dJ), conv_tensors, conv_secs, abi.F64,
                                       [m_sched[-1]])
                eps.append(Es)
            fd = (eps[0] - eps[1]) / (2 * dJ)
            res.update({"finite_difference": fd, "adjoint_minus_fd": abs(adj - fd)})
        out[name] = res
        print("bench: gradient %s E=%.12f adjoint %.10f HF %.10f %s" % (
            name, E, adj, hf, ("FD %.10f" % res["finite_difference"]) if "finite_difference" in res else ""),
            file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    return out


def dense_vs_blocks_bench(ctx, abi, synth, torch, dev, l, m, U):
    """One FP64 sweep of the dense path and one of the block-sparse path from
    the same seeded symmetric state of the Hubbard chain at bond limit m.  The
    chemical potential mu = U/2 makes half filling the ground-state sector, so
    the dense path (which does not fix N) and the block path (N = l) solve the
    same problem."""
    phys = abi.HUBBARD_CHARGES
    mpo = abi.hubbard_chain_mpo(l, t=1.0, U=U, mu=[U / 2] * l)
    out = {"workload": "hubbard_chain", "l": l, "m": m, "U": U, "mu": U / 2}
    for name in ("dense", "blocks"):
        tensors, secs = synth.random_symmetric_mps(l, phys, [l, 0], m, seed=synth.SEED_MPS)
        st = abi.State(mpo, tensors, m, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if name == "dense":
            e0 = ctx.prepare(st)
            params = abi.sweep_params(alpha=1e-3, e_before=e0, tol=1e-10)
            _, stats, _ = ctx.sweep(st, params)
        else:
            sym = abi.Symmetry(phys, abi.mpo_bond_charges(mpo, abi.mpo_fermion_charges(1)), secs)
            e0 = ctx.prepare_blocks(st, sym)
            params = abi.sweep_params(alpha=1e-3, e_before=e0, tol=1e-10)
            _, stats, _ = ctx.sweep_blocks(st, sym, params, use_graph=True)
        out[name] = {"seconds": round(time.perf_counter() - t0, 3), "energy": stats.energy}
        print("bench: one sweep %s m=%d: %.2f s  E=%.10f" % (name, m, out[name]["seconds"], stats.energy),
              file=sys.stderr, flush=True)
        del st
        torch.cuda.empty_cache()
    out["speedup_blocks"] = round(out["dense"]["seconds"] / out["blocks"]["seconds"], 2)
    return out


def comparison_bench(ctx, abi, synth, torch, dev, ms_list, steps, warmup=3):
    """FP64 H application of the three local problems on the Hubbard MPO
    shape (d = 4, w = 6), same GEMM machinery: the single-site product, the
    centre-matrix (CWF) form with its enlarged environment, and the two-site
    product.  Timed with events on the context's stream; flop counts are the
    algorithmic ones of each contraction order."""
    d, w = 4, 6
    W = torch.tensor(abi.hubbard_chain_mpo(3, t=1.0, U=8.0)[1], dtype=torch.float64, device=dev)
    out = {"workload": "local_problem_comparison_hubbard", "d": d, "w": w}

    def timed(fn, n):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    for m in ms_list:
        L = torch.tensor(synth.gaussian((m, w, m), synth.SEED_LEFT), dtype=torch.float64, device=dev) / m
        R = torch.tensor(synth.gaussian((m, w, m), synth.SEED_RIGHT), dtype=torch.float64, device=dev) / m
        psi = torch.tensor(synth.gaussian((m, d, m), synth.SEED_PSI), dtype=torch.float64, device=dev)
        y = torch.empty_like(psi)
        f1 = heff_flops(m, d, m, w, w)
        t1 = timed(lambda: ctx.apply_heff(L, W, R, psi, y), steps)
        Lt = torch.empty((m * d, w, m * d), dtype=torch.float64, device=dev)
        t_env = timed(lambda: ctx.cwf_environment(L, W, Lt), max(3, steps // 4))
        yc = torch.empty((m * d, m), dtype=torch.float64, device=dev)
        pc = psi.view(m * d, m)
        fc = 2.0 * w * d * d * m ** 3 + 2.0 * w * d * m ** 3
        tc = timed(lambda: ctx.apply_cwf(Lt, R, pc, yc), steps)
        del Lt, yc
        torch.cuda.empty_cache()
        p2 = torch.tensor(synth.gaussian((m, d, d, m), synth.SEED_PSI + 1), dtype=torch.float64, device=dev)
        y2 = torch.empty_like(p2)
        f2 = (2.0 * w * d * d * m ** 3 + 2.0 * d ** 3 * w * w * m * m * 2 + 2.0 * w * d * d * m ** 3)
        t2 = timed(lambda: ctx.apply_heff_two_site(L, W, W, R, p2, y2), max(5, steps // 2))
        del p2, y2, L, R, psi, y
        torch.cuda.empty_cache()
        e = {"single_site": {"ms": round(t1, 4), "gflop": round(f1 * 1e-9, 2), "tflops": round(f1 / t1 * 1e-9, 2)},
             "cwf": {"ms": round(tc, 4), "gflop": round(fc * 1e-9, 2), "tflops": round(fc / tc * 1e-9, 2),
                     "env_build_ms": round(t_env, 4)},
             "two_site": {"ms": round(t2, 4), "gflop": round(f2 * 1e-9, 2), "tflops": round(f2 / t2 * 1e-9, 2)},
             "time_ratio_cwf": round(tc / t1, 3), "flop_ratio_cwf": round(fc / f1, 3),
             "time_ratio_two_site": round(t2 / t1, 3), "flop_ratio_two_site": round(f2 / f1, 3)}
        out[str(m)] = e
        print("bench: local problems m=%d: single-site %.3f ms, CWF %.3f ms (x%.2f, flops x%.2f), "
              "two-site %.3f ms (x%.2f, flops x%.2f)" % (m, t1, tc, tc / t1, fc / f1, t2, t2 / t1, f2 / f1),
              file=sys.stderr, flush=True)
    return out


def residual_bench(ctx, abi, synth, torch, dev, l, m, U, max_sweeps, tol):
    """Convergence per sweep of the two expansion terms, FP64 dense sweeps
    from the same seeded state: the cheap term of eq. subexp-ourt and the
    exact residual H Psi - E Psi.  Heisenberg l = 12, m = 16, and the Hubbard
    chain (mu = U/2, so half filling is the ground-state sector) at bond
    limit m, where the exact residual is still affordable."""
    out = {"workload": "expansion_term_comparison"}
    cases = [("heisenberg_l12_m16", abi.heisenberg_mpo(12), synth.random_mps(12, 2, 16), 16),
             ("hubbard_l%d_m%d" % (l, m), abi.hubbard_chain_mpo(l, t=1.0, U=U, mu=[U / 2] * l),
              synth.random_mps(l, 4, m, seed=synth.SEED_MPS), m)]
    for name, mpo, tensors, mm in cases:
        entry = {}
        for kind in ("heuristic", "residual"):
            st = abi.State(mpo, tensors, mm, device=dev)
            e0 = ctx.prepare(st)
            params = abi.sweep_params(alpha=1e-3, e_before=e0, tol=1e-10, expansion=kind)
            energies, secs, t_exp = [], [], 0.0
            prev = None
            for _ in range(max_sweeps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, stats, recs = ctx.sweep(st, params)
                torch.cuda.synchronize()
                secs.append(round(time.perf_counter() - t0, 3))
                t_exp += sum(r.t_expand + r.t_trunc for r in recs)
                energies.append(stats.energy)
                if prev is not None and abs(stats.energy - prev) / abs(stats.energy) < tol:
                    break
                prev = stats.energy
            entry[kind] = {"energies": energies, "sweep_seconds": secs,
                           "expand_plus_truncate_seconds": round(t_exp, 3), "max_bond": max(st.m)}
            print("bench: expansion %s %s: %d sweeps, E=%.12f, %.2f s (expansion+truncation %.2f s)"
                  % (name, kind, len(energies), energies[-1], sum(secs), t_exp), file=sys.stderr, flush=True)
            del st
            torch.cuda.empty_cache()
        entry["final_energy_diff"] = entry["residual"]["energies"][-1] - entry["heuristic"]["energies"][-1]
        out[name] = entry
    return out


def cpu_baseline(L, W, R, psi, budget_s):
    """The oracle's H_eff (NumPy FP64, tensordot in the paper's order) on the
    same arrays, repeated until `budget_s` seconds are used (at least once)."""
    import numpy as np
    from oracle import contract as C
    try:
        import threadpoolctl
        threads = max([p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    Ln, Wn, Rn, pn = [np.ascontiguousarray(x) for x in (L, W, R, psi)]
    reps = 0
    t0 = time.perf_counter()
    while True:
        C.apply_heff(Ln, Wn, Rn, pn)
        reps += 1
        if time.perf_counter() - t0 >= budget_s or reps >= 100:
            break
    dt = (time.perf_counter() - t0) / reps
    return dt, reps, threads


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--m", type=int, default=2048)
    ap.add_argument("--extra-m", type=str, default="256,1024,4096",
                    help="other bond dimensions reported beside the headline (comma list, '' = none)")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=int, default=-1, help="GEMM tile configuration (-1 = library heuristic)")
    ap.add_argument("--gaussian-env", action="store_true",
                    help="Gaussian L and R instead of MPS-built environments (same kernels and shapes; "
                         "no eigensolver calls, for counter runs)")
    ap.add_argument("--no-blocks", action="store_true", help="skip the block-sparse H_eff, sweep and cylinder measurements")
    ap.add_argument("--sweep-l", type=int, default=64, help="Hubbard chain length of the block sweeps (0 = skip)")
    ap.add_argument("--sweep-sched", type=str, default="128,256,512,1024,2048",
                    help="bond limits of the block sweep run (two sweeps each, then to convergence at the last)")
    ap.add_argument("--sweep-max", type=int, default=8, help="sweeps at the last bond limit")
    ap.add_argument("--growth-tol", type=float, default=1e-6,
                    help="eigensolver residual tolerance of the bond-growth sweeps of the Hubbard chain run")
    ap.add_argument("--mixed-min-gflop", type=float, default=0.0,
                    help="mixed-precision leg of the Hubbard chain run: sites whose product costs fewer GFLOP use "
                         "FP64 products (0 = every site mixed)")
    ap.add_argument("--dense-m", type=int, default=256, help="bond limit of the dense-vs-block one-sweep comparison")
    ap.add_argument("--cylinder", type=str, default="256,512,1024,2048,4096",
                    help="bond limits of the 4x16 cylinder run ('' = skip)")
    ap.add_argument("--site-m", type=int, default=4096,
                    help="bond dimension of the cylinder-site block H_eff microbenchmark (0 = skip)")
    ap.add_argument("--cylinder-last", type=int, default=3,
                    help="at most this many sweeps at the last cylinder bond limit (until dE < 1e-8)")
    ap.add_argument("--cylinder-precs", type=str, default="f64,mixed_bf16",
                    help="eigensolver product precisions compared (f64, mixed_f32, mixed_bf16)")
    ap.add_argument("--gradient", type=str, default="64,128,256,512",
                    help="bond limits of the J1-J2 dE/dJ2 run (l=48, J2=0.24; '' = skip)")

    ap.add_argument("--residual-m", type=int, default=128,
                    help="bond limit of the Hubbard chain in the expansion-term comparison (0 = skip)")
    ap.add_argument("--compare", type=str, default="1024,2048",
                    help="bond dimensions of the single-site / CWF / two-site H application comparison ('' = skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 1 GiB read + 1 GiB write elementwise kernel (torch.neg) first, "
                         "as the reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the H_eff hot path of one GPU's share); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1501_05504_amd import abi, synth

    dev = torch.device("cuda:0")
    ctx = abi.Context(0)
    if args.copy_probe:
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y
        print("bench: copy probe done (1 GiB read, 1 GiB written)", file=sys.stderr, flush=True)
    d, w = 4, 6
    results = {}
    heads = None
    for m in [args.m] + [int(x) for x in args.extra_m.split(",") if x.strip()]:
        print("bench: building inputs m=%d" % m, file=sys.stderr, flush=True)
        if args.gaussian_env:
            mpo = abi.hubbard_chain_mpo(3, t=1.0, U=8.0)
            W = torch.tensor(mpo[1], dtype=torch.float64, device=dev)
            L = torch.tensor(synth.gaussian((m, w, m), synth.SEED_LEFT), dtype=torch.float64, device=dev) / m
            R = torch.tensor(synth.gaussian((m, w, m), synth.SEED_RIGHT), dtype=torch.float64, device=dev) / m
        else:
            L, W, R = build_inputs(ctx, abi, synth, torch, m, dev)
        ctx.set_tile_config(args.tile)
        psi = torch.tensor(synth.gaussian((m, d, m), synth.SEED_PSI), dtype=torch.float64, device=dev)
        psi /= torch.linalg.vector_norm(psi)
        out = torch.empty_like(psi)
        F = heff_flops(m, d, m, w, w)
        steps = args.steps if m == args.m else max(10, args.steps // 2)
        ms, wall, kern = time_heff(ctx, torch, L, W, R, psi, out, steps, args.warmup)
        entry = {"ms": ms, "gflops": F / ms * 1e-6, "kernel_ms": dict(zip(["gemm1", "wmap", "gemm2"], kern)),
                 "steps": steps, "wall_s": wall}
        print("bench: m=%d f64 %.3f ms  %.1f GFLOP/s  kernels %s" % (m, ms, F / ms * 1e-6, kern),
              file=sys.stderr, flush=True)
        if not args.no_f32:
            Lf, Wf, Rf, pf = L.float(), W.float(), R.float(), psi.float()
            of = torch.empty_like(pf)
            ms32, _, kern32 = time_heff(ctx, torch, Lf, Wf, Rf, pf, of, steps, args.warmup)
            entry["f32"] = {"ms": ms32, "gflops": F / ms32 * 1e-6,
                            "kernel_ms": dict(zip(["gemm1", "wmap", "gemm2"], kern32))}
            print("bench: m=%d f32 %.3f ms  %.1f GFLOP/s" % (m, ms32, F / ms32 * 1e-6), file=sys.stderr, flush=True)
            # BF16 operands (L, R, psi; W in FP32), FP32 accumulation and output
            Lb, Rb, pb = L.to(torch.bfloat16), R.to(torch.bfloat16), psi.to(torch.bfloat16)
            msb, _, kernb = time_heff(ctx, torch, Lb, Wf, Rb, pb, of, steps, args.warmup)
            entry["bf16"] = {"ms": msb, "gflops": F / msb * 1e-6,
                             "kernel_ms": dict(zip(["gemm1", "wmap", "gemm2"], kernb))}
            print("bench: m=%d bf16 %.3f ms  %.1f GFLOP/s  kernels %s" % (m, msb, F / msb * 1e-6, kernb),
                  file=sys.stderr, flush=True)
            del Lb, Rb, pb
        results[m] = entry
        if m == args.m:
            heads = (L, W, R, psi, out, ms, kern, steps)
        else:
            del L, R, psi, out
            torch.cuda.empty_cache()

    L, W, R, psi, out, ms, kern, steps = heads
    m = args.m
    F = heff_flops(m, d, m, w, w)
    gf = gemm_flops(m, d, m, w, w)
    names = ["gemm1", "wmap", "gemm2"]
    dom = max([0, 2], key=lambda i: kern[i])           # dominant MFMA kernel
    achieved = gf[names[dom]] / (kern[dom] * 1e-3)
    line = {
        "metric": "H_eff*psi GFLOP/s (FP64, Hubbard MPO d=4 w=6, m=%d)" % m,
        "value": round(F / ms * 1e-6, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian MPS environments, Gaussian psi)",
        "config": {"workload": "heff_microbench_hubbard", "m": m, "d": d, "w": w, "tile": args.tile,
                   "environments": "gaussian" if args.gaussian_env else "mps",
                   "flop_per_step": F, "seeds": {"left": synth.SEED_LEFT, "right": synth.SEED_RIGHT,
                                                 "psi": synth.SEED_PSI}},
        "pct_fp64_mfma_peak": round(100 * F / (ms * 1e-3) / PEAK["f64"], 2),
        "roofline": {"bound": "mfma", "kernel": names[dom], "achieved": round(achieved / 1e12, 3),
                     "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK["f64"], 4),
                     "traffic": (TRAFFIC[names[dom]] if (gemm_source_sha() == TRAFFIC["src_sha"]
                                                         and m == TRAFFIC["m"]) else None)},
        "per_m": {str(k): {"f64_gflops": round(v["gflops"], 1),
                           "f64_pct_peak": round(100 * v["gflops"] * 1e9 / PEAK["f64"], 2),
                           "f32_gflops": round(v["f32"]["gflops"], 1) if "f32" in v else None,
                           "f32_pct_peak": round(100 * v["f32"]["gflops"] * 1e9 / PEAK["f32"], 2) if "f32" in v else None,
                           "bf16_gflops": round(v["bf16"]["gflops"], 1) if "bf16" in v else None,
                           "bf16_kernel_ms": ({a: round(b, 4) for a, b in v["bf16"]["kernel_ms"].items()}
                                              if "bf16" in v else None),
                           "kernel_ms_f64": {a: round(b, 4) for a, b in v["kernel_ms"].items()}}
                  for k, v in results.items()},
    }
    if not args.no_blocks:
        print("bench: block-sparse H_eff ...", file=sys.stderr, flush=True)
        line["blocks"] = block_heff_bench(ctx, abi, synth, torch, np, m, dev, max(10, steps // 2))
        print("bench: blocks %s" % line["blocks"], file=sys.stderr, flush=True)
        if args.site_m > 0:
            line["cylinder_site"] = cylinder_site_bench(ctx, abi, synth, torch, np, args.site_m, dev, 20)
        sched = [int(x) for x in args.sweep_sched.split(",")]
        if args.sweep_l > 0:
            line["sweep"] = hubbard_sweep_bench(ctx, abi, synth, torch, dev, args.sweep_l, sched, 8.0, 1e-8, 1e-10,
                                                args.sweep_max, args.growth_tol, args.mixed_min_gflop)
        if args.dense_m > 0:
            line["dense_vs_blocks"] = dense_vs_blocks_bench(ctx, abi, synth, torch, dev, args.sweep_l, args.dense_m,
                                                            8.0)
    if args.gradient:
        line["gradient"] = gradient_bench(ctx, abi, synth, torch, dev, 48, [int(x) for x in args.gradient.split(",")],
                                          0.24, 1e-4, 1e-11)
    if args.residual_m > 0:
        line["expansion_terms"] = residual_bench(ctx, abi, synth, torch, dev, args.sweep_l, args.residual_m, 8.0,
                                                 10, 1e-10)
    if args.compare:
        line["local_problems"] = comparison_bench(ctx, abi, synth, torch, dev,
                                                  [int(x) for x in args.compare.split(",")], 20)
    if args.cylinder and not args.no_blocks:
        line["cylinder"] = cylinder_bench(ctx, abi, synth, torch, dev, [int(x) for x in args.cylinder.split(",")],
                                          args.cylinder_last, 1e-10, args.cylinder_precs.split(","), 1e-8)
    if not args.no_cpu:
        print("bench: cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        Ln, Wn, Rn, pn = [x.cpu().numpy() for x in (L, W, R, psi)]
        dt, reps, threads = cpu_baseline(Ln, Wn, Rn, pn, args.cpu_budget)
        line["cpu_baseline"] = {"value": round(F / dt * 1e-9, 2), "unit": "GFLOP/s", "cores": threads,
                                "kind": "oracle",
                                "sample": "%d H_eff application(s) at m=%d (same arrays), %.2f s each" % (reps, m, dt)}
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
