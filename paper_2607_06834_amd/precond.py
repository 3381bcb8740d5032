"""Diagonal mass-matrix estimate for HMC (App. A: M^-1 = cov(x)).

The inverse mass is taken from the diagonal of the local precision
-d^2 log p / dx^2 at a reference point, estimated without forming the
Hessian: for random sign vectors v, E[v * (H v)] = diag(H), with H v from a
central difference of two batched gradient evaluations (Hutchinson's
estimator).  Each batch of probes is one call of the batched gradient.
"""
from __future__ import annotations

import torch


def precision_diag(ds, x_ref, n_batches=8, batch=64, h=1e-4, seed=0):
    """Estimate diag(-Hessian of log p) at ``x_ref`` (float64 CUDA, [d])."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    d = x_ref.numel()
    acc = torch.zeros(d, dtype=torch.float64, device=x_ref.device)
    for _ in range(n_batches):
        v = (torch.randint(0, 2, (batch, d), generator=gen, dtype=torch.int8) * 2 - 1).to(
            device=x_ref.device, dtype=torch.float64)
        xp = x_ref[None, :] + h * v
        xm = x_ref[None, :] - h * v
        _, gp, sp = ds.ptafs_logp_grad(xp)
        _, gm, sm = ds.ptafs_logp_grad(xm)
        if int((sp != 0).sum()) or int((sm != 0).sum()):
            raise RuntimeError("probe points left the support; choose a smaller h")
        acc += (-(gp - gm) / (2.0 * h) * v).sum(0)
    return acc / (n_batches * batch)


def inverse_mass(ds, x_ref, theta_step=0.05, **kw):
    """Inverse mass = 1 / (estimated precision), floored per block:
    the whitened coordinates (u, z, z_dm) have prior precision 1, so their
    posterior precision is at least 1; a hyper-parameter's precision is
    floored at 1/(theta_step * prior width)^2 so that a unit-momentum step
    never spans more than a small fraction of its box."""
    p = precision_diag(ds, x_ref, **kw)
    lay = ds.layout
    nt = int(lay.n_theta)
    floor = torch.ones_like(p)
    if nt:
        lo = torch.as_tensor(ds.prior_lo, dtype=torch.float64, device=p.device)
        hi = torch.as_tensor(ds.prior_hi, dtype=torch.float64, device=p.device)
        floor[:nt] = 1.0 / (theta_step * (hi - lo)) ** 2
    return 1.0 / torch.maximum(p, floor)


def ascend_coefficients(ds, x, inv_mass, n_steps=40, rate=0.5):
    """Move the whitened coefficients (u, z, z_dm) of every chain towards
    their conditional mode at fixed hyper-parameters with preconditioned
    gradient ascent, x_w += rate_c * M^-1 grad_w, halving a chain's rate
    whenever a step would lower its log density (a start inside the typical
    set for HMC).  Hyper-parameters are left unchanged."""
    nt = int(ds.layout.n_theta)
    im = inv_mass.clone()
    im[:nt] = 0.0
    x = x.clone()
    lp, g, st = ds.ptafs_logp_grad(x)
    r = torch.full((x.shape[0], 1), rate, dtype=torch.float64, device=x.device)
    for _ in range(n_steps):
        xn = x + r * im[None, :] * g
        lpn, gn, stn = ds.ptafs_logp_grad(xn)
        ok = (stn == 0) & (lpn >= lp)
        x = torch.where(ok[:, None], xn, x)
        g = torch.where(ok[:, None], gn, g)
        lp = torch.where(ok, lpn, lp)
        r = torch.where(ok[:, None], r, 0.5 * r)
    return x


def find_step(ds, x, logp, grad, inv_mass, *, n_leapfrog, eps0=0.2, seed=1, max_halvings=14,
              stream=None):
    """Largest step eps0 / 2^m whose trial trajectory keeps every leapfrog
    evaluation of every chain valid and accepts at least one chain."""
    C = x.shape[0]
    eps = eps0
    for _ in range(max_halvings):
        xx, lp, gr = x.clone(), logp.clone(), grad.clone()
        acc = torch.zeros(C, dtype=torch.int64, device=x.device)
        bad = torch.zeros(C, dtype=torch.int64, device=x.device)
        ds.ptafs_hmc_run(xx, lp, gr, acc, n_traj=1, n_leapfrog=n_leapfrog, eps=eps, seed=seed,
                         traj0=1 << 30, inv_mass=inv_mass, n_invalid=bad, use_graph=False,
                         stream=stream)
        torch.cuda.synchronize()
        if int(bad.sum()) == 0 and int(acc.sum()) > 0:
            return eps
        eps *= 0.5
    return eps
