"""Fixed-step leapfrog HMC with Metropolis-Hastings accept (App. A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

H(x, p) = -log p(x) + 1/2 p^T M^-1 p with a diagonal inverse mass
(Eqs. Hamiltonian and Gaussian_momentum); momenta p ~ N(0, M), and a
coordinate whose inverse mass is 0 is frozen (zero momentum); a trajectory
is a half kick, L drift/kick steps (the last kick a half kick) and the
accept test ln u < H0 - H1 (Eq. HMC_acceptance).  Random numbers come from
Philox4x32-10 (oracle.philox) so that a GPU sampler following the same
conventions makes the same draws.
"""
from __future__ import annotations

import numpy as np

from . import philox


def run(logp_grad, x0, *, n_traj, n_leapfrog, eps, seed, traj0=0, inv_mass=None,
        keep_samples=False):
    """``logp_grad(X) -> (logp (C,), grad (C, d))`` for a batch of chains.

    Returns final x, logp, grad, accept counts and optionally the samples
    after every trajectory (n_traj, C, d)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    C, d = x.shape
    im = np.ones(d) if inv_mass is None else np.asarray(inv_mass, np.float64)
    lp, gr = logp_grad(x)
    nacc = np.zeros(C, dtype=np.int64)
    samples = [] if keep_samples else None
    for j in range(traj0, traj0 + n_traj):
        nrm = np.stack([philox.momentum_normals(seed, c, j, d) for c in range(C)])
        # coordinates with inverse mass 0 are frozen: zero momentum
        p = np.where(im > 0, nrm / np.sqrt(np.where(im > 0, im, 1.0)), 0.0)
        H0 = -lp + 0.5 * np.sum(im * p * p, axis=1)
        xn, pn = x.copy(), p + 0.5 * eps * gr
        for step in range(n_leapfrog):
            xn = xn + eps * im * pn
            lpn, grn = logp_grad(xn)
            pn = pn + (eps if step + 1 < n_leapfrog else 0.5 * eps) * grn
        H1 = -lpn + 0.5 * np.sum(im * pn * pn, axis=1)
        for c in range(C):
            u = philox.accept_uniform(seed, c, j)
            if np.isfinite(H1[c]) and np.log(u) < H0[c] - H1[c]:
                x[c], lp[c], gr[c] = xn[c], lpn[c], grn[c]
                nacc[c] += 1
        if keep_samples:
            samples.append(x.copy())
    return x, lp, gr, nacc, (np.stack(samples) if keep_samples else None)
