"""Residuals drawn from the model itself (Sec. III decomposition).

TEST INFRASTRUCTURE ONLY (see the package docstring).

dt = M b + F a + w F a_dm + h + n with (u, z, z_dm) standard normal, mapped
through the injected hyper-parameters, and n ~ N(0, N).
"""
from __future__ import annotations

import numpy as np

from . import cw as cwmod
from .model import Prepared


def model_residuals(ds, theta, draws):
    """Return a copy of ``ds`` whose ``dt`` is drawn from the model at
    ``theta`` using the standard normals in ``draws``."""
    prep = Prepared(ds)
    lay = prep.lay
    x = np.concatenate([theta, draws["u"], draws["z"], draws["zdm"]])
    gw, rn, dm, cwp, u, z, zdm = prep.split(x[None, :])
    rho, kap, kdm = prep.spectra(gw, rn, dm, 1)
    n, K = prep.n_psr, prep.K
    a = np.zeros((n, 2 * K))
    for k in range(K):
        Lk = np.linalg.cholesky(rho[0, k] * prep.Gamma + np.diag(kap[0, :, k]))
        a[:, 2 * k] = Lk @ z[0, :, 2 * k]
        a[:, 2 * k + 1] = Lk @ z[0, :, 2 * k + 1]
    adm = np.repeat(np.sqrt(kdm[0]), 2, axis=1) * zdm[0]
    b = prep.sigma_b * u[0]
    out = dict(ds)
    dt = np.empty_like(np.asarray(ds["dt"], np.float64))
    off = ds["toa_offsets"]
    for I, p in enumerate(prep.psr):
        s, e = int(off[I]), int(off[I + 1])
        sig = p["M"] @ b[I] + p["F"] @ a[I] + p["w"] * (p["Fdm"] @ adm[I])
        if prep.has_cw:
            sig = sig + cwmod.delay(p["t"], p["pos"], cwp[0], want_grad=False)[0]
        dt[s:e] = sig + np.sqrt(p["N"]) * draws["white"][s:e]
    out["dt"] = dt
    return out
