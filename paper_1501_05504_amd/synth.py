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
