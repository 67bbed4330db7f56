"""Seeded synthetic inputs.

This module only draws random numbers and picks sizes; it contains none of the
method's arithmetic (no contraction, no canonicalisation, no MPO).  Both the
GPU path and the CPU oracle consume the arrays it returns.

Default seeds: 1501 for the initial MPS, 5504 for psi, 1 / 2 for the MPS that
generate the left / right environments of the H_eff microbenchmark.
"""
import numpy as np

SEED_MPS = 1501
SEED_PSI = 5504
SEED_LEFT = 1
SEED_RIGHT = 2


def gaussian(shape, seed):
    """Standard-normal float64 array."""
    return np.random.default_rng(seed).standard_normal(shape)


def bond_dims(l, d, mmax):
    """Open-chain bond dimensions min(mmax, d^b, d^(l-b)) for bonds 0..l."""
    return [int(min(mmax, d ** b, d ** (l - b))) for b in range(l + 1)]


def random_mps(l, d, mmax, seed=SEED_MPS):
    """Gaussian site tensors M_i[a, s, b] of shape (m_{i-1}, d, m_i)."""
    m = bond_dims(l, d, mmax)
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((m[i], d, m[i + 1])) for i in range(l)]


def growing_mps(nsites, d, m, seed):
    """Gaussian tensors of `nsites` sites whose bonds grow as min(d^k, m) from
    a dimension-1 left edge: the generator of a left (or, mirrored, right)
    environment of bond m for the H_eff microbenchmark."""
    rng = np.random.default_rng(seed)
    dims = [min(d ** k, m) for k in range(nsites + 1)]
    return [rng.standard_normal((dims[k], d, dims[k + 1])) for k in range(nsites)]


def env_sites_for(m, d):
    """Smallest number of sites whose grown bond reaches m: ceil(log_d m)."""
    k = 0
    while d ** k < m:
        k += 1
    return k


# --- block structure of symmetric workloads ---------------------------------
# Index bookkeeping only: which entries a charge-conserving tensor may hold.

def gaussian_sectors(center, sigma, m, span, parity=True):
    """(N, 2Sz) sectors around `center` with dimensions proportional to
    exp(-(N-N0)^2 / 2 sN^2 - (2Sz-S0)^2 / 2 sS^2), normalised to m (largest
    remainder rounding, empty sectors dropped).  parity: 2Sz = N mod 2."""
    N0, S0 = center
    sN, sS = sigma
    qs, ws = [], []
    for N in range(N0 - span[0], N0 + span[0] + 1):
        for S in range(S0 - span[1], S0 + span[1] + 1):
            if parity and (N - S) % 2:
                continue
            qs.append((N, S))
            ws.append(np.exp(-(N - N0) ** 2 / (2 * sN ** 2) - (S - S0) ** 2 / (2 * sS ** 2)))
    ws = np.array(ws) / np.sum(ws) * m
    dims = np.floor(ws).astype(int)
    rem = m - dims.sum()
    for i in np.argsort(-(ws - dims))[:rem]:
        dims[i] += 1
    keep = dims > 0
    return np.array(qs)[keep], dims[keep]


def expand_charges(q, dims):
    """Charge of every basis state of a bond (states ordered by sector)."""
    return np.repeat(np.asarray(q), np.asarray(dims), axis=0)


def mask_site(ql, qphys, qr):
    """psi[a,s,b] may be nonzero iff q_a + q_s = q_b."""
    ql, qphys, qr = (np.asarray(x) for x in (ql, qphys, qr))
    return np.all(ql[:, None, None, :] + qphys[None, :, None, :] == qr[None, None, :, :], axis=-1)


def mask_env(q, wq):
    """L[a,w,x] may be nonzero iff q_a - q_x = Delta_w."""
    q, wq = np.asarray(q), np.asarray(wq)
    return np.all(q[:, None, None, :] - q[None, None, :, :] == wq[None, :, None, :], axis=-1)


def initial_sectors(l, phys_q, target, mmax):
    """Sectors of the initial symmetric MPS: on bond b every charge Q that can
    be reached from the left edge with b sites and completed to `target` with
    the remaining l - b sites, with dimension min(#left states of charge Q,
    #right states completing it); when these exceed the bond budget
    min(mmax, d^b, d^(l-b)) the budget is shared in proportion (largest
    remainder, at least one state for the heaviest sectors).  Sectors are
    ordered by charge (lexicographically).  Returns a list of (q, dims)."""
    phys = [tuple(int(x) for x in np.atleast_1d(q)) for q in phys_q]
    nq = len(phys[0])
    d = len(phys)
    zero = tuple([0] * nq)
    tgt = tuple(int(x) for x in np.atleast_1d(target))

    def add(a, b, sign=1):
        return tuple(x + sign * y for x, y in zip(a, b))
    cap = 10 ** 15
    left = [{zero: 1}]
    for _ in range(l):
        nxt = {}
        for q, n in left[-1].items():
            for ps in phys:
                k = add(q, ps)
                nxt[k] = min(cap, nxt.get(k, 0) + n)
        left.append(nxt)
    right = [None] * (l + 1)
    right[l] = {tgt: 1}
    for b in range(l - 1, -1, -1):
        nxt = {}
        for q, n in right[b + 1].items():
            for ps in phys:
                k = add(q, ps, -1)
                nxt[k] = min(cap, nxt.get(k, 0) + n)
        right[b] = nxt
    out = []
    for b in range(l + 1):
        qs = sorted(q for q in left[b] if q in right[b])
        w = np.array([min(left[b][q], right[b][q]) for q in qs], dtype=float)
        budget = int(min(mmax, d ** b, d ** (l - b)))
        if w.sum() <= budget:
            dims = w.astype(int)
        else:
            share = w / w.sum() * budget
            dims = np.floor(share).astype(int)
            if dims.sum() == 0:
                dims[np.argsort(-w)[:budget]] = 1
            rem = budget - dims.sum()
            for i in np.argsort(-(share - dims))[:max(rem, 0)]:
                dims[i] += 1
            dims = np.minimum(dims, w.astype(int))
        keep = dims > 0
        out.append((np.array(qs, dtype=int).reshape(-1, nq)[keep], dims[keep]))
    return out


def random_symmetric_mps(l, phys_q, target, mmax, seed=SEED_MPS):
    """Gaussian site tensors on the initial sectors, zero outside the
    symmetry-allowed blocks.  Returns (tensors, sectors)."""
    secs = initial_sectors(l, phys_q, target, mmax)
    rng = np.random.default_rng(seed)
    d = len(phys_q)
    tensors = []
    for i in range(l):
        ql = expand_charges(*secs[i])
        qr = expand_charges(*secs[i + 1])
        t = rng.standard_normal((len(ql), d, len(qr)))
        tensors.append(t * mask_site(ql, np.asarray(phys_q).reshape(d, -1), qr))
    return tensors, secs
