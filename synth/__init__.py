"""Seeded synthetic PTA inputs shared by the oracle tests and the GPU path.

This module only draws random inputs: TOA times, uncertainties, radio
frequencies, backend labels, sky positions, hyper-parameter points and
standard-normal vectors.  It holds none of the likelihood, prior, basis,
correlation or transform arithmetic of the method; those live separately in
the oracle and in the HIP library.

The data sets stand in for the NANOGrav 15-year release and the simulated
arrays of the paper's Sec. VI (67 pulsars over ~16 yr, 100 pulsars over 15 yr),
which are not available here.  Shapes, sizes and value distributions follow
the workload descriptions:

* sky positions uniform on the sphere;
* TOAs uniform over the span with random 30-day gaps (small arrays) or
  uniform (large arrays), counts per pulsar lognormal;
* log10 sigma ~ N(-6, 0.7) clipped at 3 s.d.; EFAC 1.1; EQUAD 10^-6.5 s
  (white-noise model of Sec. III.B);
* radio frequencies uniform in 0.4-2.0 GHz;
* 1-4 backends per pulsar.

Residuals ``dt`` are drawn without the method's model: white noise at the
quoted TOA uncertainty plus a Brownian (random-walk) red process of ~1 us
amplitude.  The values of ``dt`` do not change the work any evaluation does;
model-drawn residuals, where a test needs them, are produced by the oracle
from the standard-normal draws returned under ``"draws"``.
"""
from __future__ import annotations

import numpy as np

YEAR_S = 365.25 * 86400.0          # Julian year in seconds
DAY_S = 86400.0

# Hyper-prior boxes (Sec. IV.A: log10 A ~ U(-20, -10), gamma ~ U(0, 7); the
# same box is used for intrinsic red noise and DM noise).
LOG10A_BOX = (-20.0, -10.0)
GAMMA_BOX = (0.0, 7.0)
# Continuous-wave parameter box, in the order
# (cos theta, phi, log10 Mc, log10 f_gw, Phi0, cos iota, psi, log10 h).
CW_BOX = (
    (-1.0, 1.0),
    (0.0, 2.0 * np.pi),
    (8.5, 9.5),
    (-8.5, -7.5),
    (0.0, 2.0 * np.pi),
    (-1.0, 1.0),
    (0.0, np.pi),
    (-18.0, -11.0),
)


def _sky(rng, n):
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)


def _toas_with_gaps(rng, n, span, n_gaps, gap_len):
    starts = rng.uniform(0.0, span - gap_len, n_gaps)
    out = np.empty(0)
    while out.size < n:
        cand = rng.uniform(0.0, span, 2 * n)
        keep = np.ones(cand.size, bool)
        for s in starts:
            keep &= ~((cand >= s) & (cand < s + gap_len))
        out = np.concatenate([out, cand[keep]])
    return np.sort(out[:n])


def _sigmas(rng, n):
    z = np.clip(rng.standard_normal(n), -3.0, 3.0)
    return 10.0 ** (-6.0 + 0.7 * z)


def theta_box(n_psr, nf_rn, nf_gw, nf_dm, has_cw):
    """Prior box (lo, hi) per hyper-parameter entry, in boundary order
    [gw (log10A, gamma) | rn per pulsar | dm per pulsar | cw (8)]."""
    lo, hi = [], []
    pl = [LOG10A_BOX, GAMMA_BOX]
    if nf_gw > 0:
        for b in pl:
            lo.append(b[0]); hi.append(b[1])
    if nf_rn > 0:
        for _ in range(n_psr):
            for b in pl:
                lo.append(b[0]); hi.append(b[1])
    if nf_dm > 0:
        for _ in range(n_psr):
            for b in pl:
                lo.append(b[0]); hi.append(b[1])
    if has_cw:
        for b in CW_BOX:
            lo.append(b[0]); hi.append(b[1])
    return np.array(lo, dtype=np.float64), np.array(hi, dtype=np.float64)


def block_widths(ds):
    """Widths of the blocks of a flat parameter vector, in boundary order."""
    n = ds["n_psr"]
    ka = max(ds["nf_rn"], ds["nf_gw"])
    return dict(
        theta=ds["prior_lo"].size,
        u=3 * n,
        z=n * 2 * ka,
        zdm=n * 2 * ds["nf_dm"],
    )


def _finish(rng, ds, red_amp=1e-6):
    """Attach residuals (white + Brownian red, model-free) and the
    standard-normal draws a model injection would need."""
    off = ds["toa_offsets"]
    n = ds["n_psr"]
    t = ds["t"]
    white = rng.standard_normal(t.size)
    eff = ds["efac"][ds["backend"]] * ds["sigma"]
    dt = eff * white
    for p in range(n):
        s, e = off[p], off[p + 1]
        tt = t[s:e]
        inc = np.diff(np.concatenate([[0.0], tt])) / ds["tspan"]
        walk = np.cumsum(np.sqrt(np.maximum(inc, 0.0)) * rng.standard_normal(e - s))
        dt[s:e] += red_amp * (walk - walk.mean())
    ds["dt"] = dt
    w = block_widths(ds)
    ds["draws"] = dict(
        white=rng.standard_normal(t.size),
        u=rng.standard_normal(w["u"]),
        z=rng.standard_normal(w["z"]),
        zdm=rng.standard_normal(w["zdm"]),
    )
    return ds


def make_array(seed, n_psr, counts, span, *, backends_per_psr, nu_range=None,
               nf_rn, nf_gw, nf_dm, has_cw=False, gaps=None,
               efac=1.1, log10_equad=-6.5, sigma_b=1e-5, dm_ref_hz=1.4e9):
    """Generic generator: ``counts`` TOAs per pulsar over ``span`` seconds."""
    rng = np.random.default_rng(seed)
    pos = _sky(rng, n_psr)
    ts, sig, nus, be = [], [], [], []
    nb_total = 0
    for p in range(n_psr):
        c = int(counts[p])
        if gaps is not None:
            tt = _toas_with_gaps(rng, c, span, gaps[0], gaps[1])
        else:
            tt = np.sort(rng.uniform(0.0, span, c))
        ts.append(tt)
        sig.append(_sigmas(rng, c))
        if nu_range is None:
            nus.append(np.full(c, 1.4e9))
        else:
            nus.append(rng.uniform(nu_range[0], nu_range[1], c))
        nb = int(backends_per_psr[p])
        be.append(nb_total + rng.integers(0, nb, c))
        nb_total += nb
    offs = np.zeros(n_psr + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(x) for x in ts])
    lo, hi = theta_box(n_psr, nf_rn, nf_gw, nf_dm, has_cw)
    ds = dict(
        n_psr=n_psr,
        toa_offsets=offs,
        t=np.concatenate(ts),
        sigma=np.concatenate(sig),
        nu=np.concatenate(nus),
        backend=np.concatenate(be).astype(np.int32),
        n_backend=nb_total,
        efac=np.full(nb_total, efac),
        equad=np.full(nb_total, 10.0 ** log10_equad),
        psr_pos=pos,
        tspan=float(span),
        nf_rn=int(nf_rn), nf_gw=int(nf_gw), nf_dm=int(nf_dm),
        dm_scale=float(dm_ref_hz) ** 2,
        sigma_b=float(sigma_b),
        has_cw=int(bool(has_cw)),
        prior_lo=lo, prior_hi=hi,
    )
    return _finish(rng, ds)


def injected_theta(ds, seed, *, gw=(-14.5, 13.0 / 3.0), rn=None, dm=None, cw=None):
    """Hyper-parameter vector of an injection, in boundary order.

    ``rn``/``dm`` None draws per-pulsar log10A ~ U(-18,-13), gamma ~ U(2,5)
    (the simulated-array distributions of Sec. VI); a 2-tuple fixes them.
    ``cw`` None draws the CW parameters from their prior box.
    """
    rng = np.random.default_rng(seed)
    n = ds["n_psr"]
    th = []
    if ds["nf_gw"] > 0:
        th += list(gw)
    for on, fix in ((ds["nf_rn"] > 0, rn), (ds["nf_dm"] > 0, dm)):
        if not on:
            continue
        for _ in range(n):
            if fix is None:
                th += [rng.uniform(-18.0, -13.0), rng.uniform(2.0, 5.0)]
            else:
                th += list(fix)
    if ds["has_cw"]:
        if cw is None:
            th += [rng.uniform(b[0], b[1]) for b in CW_BOX]
        else:
            th += list(cw)
    return np.array(th, dtype=np.float64)


def random_points(ds, n, seed, *, theta=None, theta_jitter=None, in_box=True):
    """``n`` flat parameter vectors: hyper-parameters uniform in the prior box
    (or ``theta`` plus uniform jitter), u, z, z_dm standard normal."""
    rng = np.random.default_rng(seed)
    w = block_widths(ds)
    lo, hi = ds["prior_lo"], ds["prior_hi"]
    if theta is None:
        th = rng.uniform(lo, hi, size=(n, lo.size))
    else:
        th = np.tile(np.asarray(theta, np.float64), (n, 1))
        if theta_jitter:
            th += rng.uniform(-theta_jitter, theta_jitter, size=th.shape)
        if in_box:
            th = np.clip(th, lo, hi)
    rest = rng.standard_normal((n, w["u"] + w["z"] + w["zdm"]))
    return np.concatenate([th, rest], axis=1)


# ---------------------------------------------------------------- configs --

def cfg1(seed=101):
    """3 pulsars x 500 TOAs over 10 yr with five 30-day gaps each, 2 backends
    per pulsar, 10 frequencies for intrinsic and common red noise, no DM."""
    return make_array(seed, 3, [500, 500, 500], 10.0 * YEAR_S,
                      backends_per_psr=[2, 2, 2], nf_rn=10, nf_gw=10, nf_dm=0,
                      gaps=(5, 30.0 * DAY_S))


def cfg3(seed=101):
    """The 3-pulsar array of ``cfg1`` plus a continuous-wave signal."""
    return make_array(seed, 3, [500, 500, 500], 10.0 * YEAR_S,
                      backends_per_psr=[2, 2, 2], nf_rn=10, nf_gw=10, nf_dm=0,
                      gaps=(5, 30.0 * DAY_S), has_cw=True)


def lognormal_counts(rng, n_psr, total, lo, hi, mu=3.5, sd=0.3):
    """TOA counts per pulsar: 10^N(mu, sd), clipped to [lo, hi], rescaled so
    they sum to ``total`` exactly (remainder to the largest)."""
    c = np.clip(10.0 ** rng.normal(mu, sd, n_psr), lo, hi)
    c = np.floor(c * total / c.sum()).astype(np.int64)
    c = np.clip(c, lo, hi)
    c[np.argmax(c)] += total - c.sum()
    return c


def cfg2(seed=201, n_psr=67, total=250_000):
    """67 pulsars, ~250k TOAs over 16 yr, 1-4 backends, radio frequencies in
    0.4-2.0 GHz, 30 intrinsic-red-noise and 30 DM frequencies, 14 common."""
    rng = np.random.default_rng(seed + 10_000)
    counts = lognormal_counts(rng, n_psr, total, 1000, 10000)
    nb = rng.integers(1, 5, n_psr)
    return make_array(seed, n_psr, counts, 16.0 * YEAR_S, backends_per_psr=nb,
                      nu_range=(0.4e9, 2.0e9), nf_rn=30, nf_gw=14, nf_dm=30)


def cw_array(seed=301, n_psr=100, n_toa=180):
    """The simulated CW array of the paper's results section, stand-in: 100
    pulsars uniform on the sky, ~monthly TOAs (180 over 15 yr), TOA
    uncertainty 0.5 us, EFAC 1, negligible EQUAD, 30 intrinsic red-noise and
    14 common (HD) frequencies, no DM, and a CW represented in its own basis
    of 60 frequencies on twice the span.  The CW box is widened to hold the
    paper's injected source (log10 Mc = 8.4, log10 f = -8.4)."""
    ds = make_array(seed, n_psr, [n_toa] * n_psr, 15.0 * YEAR_S, backends_per_psr=[1] * n_psr,
                    nf_rn=30, nf_gw=14, nf_dm=0, has_cw=True, efac=1.0, log10_equad=-12.0)
    rng = np.random.default_rng(seed + 1)
    ds["sigma"] = np.full(ds["t"].size, 0.5e-6)
    ds["dt"] = 0.5e-6 * rng.standard_normal(ds["t"].size)
    ds["cw_nf"] = 60
    ds["cw_tspan"] = 2.0 * ds["tspan"]
    lo, hi = ds["prior_lo"].copy(), ds["prior_hi"].copy()
    c0 = lo.size - 8
    lo[c0 + 2], hi[c0 + 2] = 7.0, 10.0
    lo[c0 + 3], hi[c0 + 3] = -9.0, -7.5
    ds["prior_lo"], ds["prior_hi"] = lo, hi
    return ds


# the paper's injected CW: cos(theta), phi, log10 Mc, log10 f, Phi0, cos(iota), psi, log10 h
CW_PAPER = (np.sqrt(2.0) / 2.0, np.pi / 4.0, 8.4, -8.4, np.pi / 4.0, np.sqrt(2.0) / 2.0, np.pi / 3.0, -14.4)


def serving_request(seed):
    """One independent data set of the request stream: 20-120 pulsars,
    200-8000 TOAs each (lognormal), 10-30 frequencies shared by intrinsic,
    common and DM noise, a CW signal with probability 1/2."""
    rng = np.random.default_rng(seed)
    n_psr = int(rng.integers(20, 121))
    counts = np.clip(10.0 ** rng.normal(3.0, 0.35, n_psr), 200, 8000).astype(np.int64)
    k = int(rng.integers(10, 31))
    cw = bool(rng.random() < 0.5)
    nb = rng.integers(1, 5, n_psr)
    span = rng.uniform(10.0, 16.0) * YEAR_S
    return make_array(int(rng.integers(1 << 30)), n_psr, counts, span,
                      backends_per_psr=nb, nu_range=(0.4e9, 2.0e9),
                      nf_rn=k, nf_gw=k, nf_dm=k, has_cw=cw)
