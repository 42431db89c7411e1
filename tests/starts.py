"""Seeded starting configurations shared by the tests (oracle Metropolis
burn-in of the seeded uniform positions; no product code)."""
import numpy as np

import oracle
from paper_1708_00744_amd import inputs


def uniform(n, L, walkers, spins, seed):
    """Seeded uniform positions in [0, L)^3, shape (walkers, spins, n, 3)."""
    return np.stack([inputs.positions(seed, w, spins * n, L).reshape(spins, n, 3) for w in range(walkers)])


def burned_in(n, L, walkers, spins, seed, sweeps=3, sigma_frac=0.1):
    """Seeded uniform positions after `sweeps` oracle Metropolis sweeps with
    sigma = sigma_frac * L (acceptance about 0.4 at 0.1 L).  Uniform-random
    starts put some electrons close together and are poorly conditioned
    (cond(A) 1e3-1e5 at N = 256-512); equilibrated ones avoid that (cond(A)
    1e2-1e3)."""
    p0 = uniform(n, L, walkers, spins, seed)
    out = np.zeros_like(p0)
    for w in range(walkers):
        for s in range(spins):
            out[w, s] = oracle.walker_run(n, L, seed + 7919, w, s, sigma_frac * L, p0[w, s], sweeps, residual=False,
                                          fresh=False).pos
    return out
