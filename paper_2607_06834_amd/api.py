"""Python binding of libptafs with the same names as the C ABI.

PyTorch provides device memory and streams; every arithmetic step runs in the
HIP library.  Tensors passed in must be float64 on the data set's device.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _make_desc(desc, keep):
    """ptafs_dataset_desc for a mapping of NumPy arrays / scalars; the arrays
    it points into are appended to ``keep`` (prior_lo, prior_hi last)."""
    def arr(name, dtype):
        a = np.ascontiguousarray(np.asarray(desc[name]), dtype=dtype)
        keep.append(a)
        return a

    offs = arr("toa_offsets", np.int64)
    t, dt = arr("t", np.float64), arr("dt", np.float64)
    sig, nu = arr("sigma", np.float64), arr("nu", np.float64)
    be = arr("backend", np.int32)
    efac, equad = arr("efac", np.float64), arr("equad", np.float64)
    pos = arr("psr_pos", np.float64)
    lo, hi = arr("prior_lo", np.float64), arr("prior_hi", np.float64)
    d = _lib.DatasetDesc()
    d.n_psr = int(desc["n_psr"])
    d.toa_offsets = _ptr(offs, C.c_int64)
    d.t, d.dt, d.sigma, d.nu = (_ptr(a, C.c_double) for a in (t, dt, sig, nu))
    d.backend = _ptr(be, C.c_int32)
    d.n_backend = int(efac.size)
    d.efac, d.equad, d.psr_pos = (_ptr(a, C.c_double) for a in (efac, equad, pos))
    d.tspan = float(desc["tspan"])
    d.nf_rn, d.nf_gw, d.nf_dm = int(desc["nf_rn"]), int(desc["nf_gw"]), int(desc["nf_dm"])
    d.dm_scale = float(desc["dm_scale"])
    d.sigma_b = float(desc["sigma_b"])
    d.has_cw = int(desc["has_cw"])
    d.prior_lo, d.prior_hi = _ptr(lo, C.c_double), _ptr(hi, C.c_double)
    return d


def ptafs_estimate(desc, n_chains):
    """Layout and device footprint of a data set before it is created
    (ptafs_estimate: host arithmetic only, no GPU needed)."""
    keep = []
    d = _make_desc(desc, keep)
    out = _lib.LayoutInfo()
    _lib.check(_lib.load().ptafs_estimate(C.byref(d), int(n_chains), C.byref(out)),
               "ptafs_estimate")
    return out


class Dataset:
    """A PTA data set resident on the current GPU (ptafs_dataset_create).

    ``desc`` is a mapping with the fields of ``ptafs_dataset_desc``: n_psr,
    toa_offsets, t, dt, sigma, nu, backend, efac, equad, psr_pos, tspan,
    nf_rn, nf_gw, nf_dm, dm_scale, sigma_b, has_cw, prior_lo, prior_hi
    (NumPy arrays or scalars; n_backend is taken from efac)."""

    def __init__(self, desc, stream=None):
        lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libptafs needs a HIP GPU")
        keep = []
        d = _make_desc(desc, keep)
        lo, hi = keep[-2], keep[-1]
        h = C.c_void_p()
        _lib.check(lib.ptafs_dataset_create(C.byref(d), _stream_handle(stream), C.byref(h)),
                   "ptafs_dataset_create")
        self._h = h
        self.prior_lo, self.prior_hi = lo.copy(), hi.copy()
        self.toa_offsets = np.asarray(desc["toa_offsets"], dtype=np.int64).copy()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.layout = self.ptafs_layout(0)
        self.d = int(self.layout.d)

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.load().ptafs_dataset_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ptafs_layout(self, n_chains):
        out = _lib.LayoutInfo()
        _lib.check(_lib.load().ptafs_layout(self._h, int(n_chains), C.byref(out)), "ptafs_layout")
        return out

    def ptafs_reserve(self, n_chains):
        _lib.check(_lib.load().ptafs_reserve(self._h, int(n_chains)), "ptafs_reserve")

    def ptafs_set_tuning(self, tiles_per_chunk, waves_per_block=1, xcd_map=1):
        _lib.check(_lib.load().ptafs_set_tuning(self._h, int(tiles_per_chunk), int(waves_per_block),
                                                int(xcd_map)), "ptafs_set_tuning")

    def ptafs_get_tuning(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _lib.check(_lib.load().ptafs_get_tuning(self._h, C.byref(a), C.byref(b), C.byref(c)),
                   "ptafs_get_tuning")
        return a.value, b.value, c.value

    def _check_x(self, x, inplace=False):
        """x as the library reads it.  A non-contiguous x is copied for
        read-only calls; calls that update x in place refuse it (the update
        would land in the copy)."""
        if not (isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.is_cuda):
            raise TypeError("x must be a float64 CUDA tensor")
        if x.dim() != 2 or x.shape[1] != self.d:
            raise ValueError(f"x must have shape (n_chains, {self.d})")
        if not x.is_contiguous():
            if inplace:
                raise ValueError("x is updated in place and must be contiguous")
            x = x.contiguous()
        return x

    @staticmethod
    def _check_out(t, dtype, shape, name):
        if not (isinstance(t, torch.Tensor) and t.dtype == dtype and t.is_cuda
                and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape {tuple(shape)}")

    def _call(self, fn, x, out=None, stream=None):
        x = self._check_x(x)
        n = x.shape[0]
        if out is None:
            # outputs (and the copy of a non-contiguous x) belong to the launch
            # stream, so the caching allocator does not hand them out again
            # while that stream still writes them
            if stream is not None:
                x.record_stream(stream)
            with torch.cuda.stream(stream) if stream is not None else _nullctx():
                logp = torch.empty(n, dtype=torch.float64, device=x.device)
                grad = torch.empty_like(x)
                status = torch.empty(n, dtype=torch.int32, device=x.device)
        else:
            logp, grad, status = out
            self._check_out(logp, torch.float64, (n,), "logp")
            self._check_out(grad, torch.float64, (n, self.d), "grad")
            self._check_out(status, torch.int32, (n,), "status")
        _lib.check(fn(self._h, n, C.c_void_p(x.data_ptr()), C.c_void_p(logp.data_ptr()),
                      C.c_void_p(grad.data_ptr()), C.c_void_p(status.data_ptr()),
                      _stream_handle(stream)), fn.__name__)
        return logp, grad, status

    def ptafs_logp_grad(self, x, out=None, stream=None):
        """Batched form: returns (logp [C], grad [C, d], status [C])."""
        return self._call(_lib.load().ptafs_logp_grad, x, out, stream)

    def ptafs_logp_grad_noalloc(self, x, out=None, stream=None):
        """Batched form on the library's static per-device workspace (no
        device allocation in the library call); same outputs."""
        return self._call(_lib.load().ptafs_logp_grad_noalloc, x, out, stream)

    def ptafs_logp_grad_plain(self, x, out=None, stream=None):
        """Plain (launch per pulsar, vector ALU) form; same outputs."""
        return self._call(_lib.load().ptafs_logp_grad_plain, x, out, stream)

    STAGES = ("spec_fwd", "toa", "reduce", "spec_bwd", "finalize")

    def ptafs_profile_stages(self, x, reps=10, plain=False, stream=None):
        """Mean ms per pipeline stage over ``reps`` evaluations (HIP events;
        synchronises the stream, so its temporaries are idle on return)."""
        x = self._check_x(x)
        n = x.shape[0]
        logp = torch.empty(n, dtype=torch.float64, device=x.device)
        grad = torch.empty_like(x)
        status = torch.empty(n, dtype=torch.int32, device=x.device)
        ms = (C.c_double * 5)()
        _lib.check(_lib.load().ptafs_profile_stages(
            self._h, n, C.c_void_p(x.data_ptr()), C.c_void_p(logp.data_ptr()),
            C.c_void_p(grad.data_ptr()), C.c_void_p(status.data_ptr()), int(reps), int(bool(plain)),
            ms, _stream_handle(stream)), "ptafs_profile_stages")
        return dict(zip(self.STAGES, list(ms)))

    def ptafs_hmc_run(self, x, logp, grad, n_accept, *, n_traj, n_leapfrog, eps, seed, traj0=0,
                      inv_mass=None, samples=None, n_invalid=None, use_graph=True, stream=None):
        """Fixed-step HMC in place on (x, logp, grad); n_accept int64 [C];
        n_invalid (int64 [C], optional) counts leapfrog evaluations with a
        nonzero status."""
        x = self._check_x(x, inplace=True)
        n = x.shape[0]
        self._check_out(logp, torch.float64, (n,), "logp")
        self._check_out(grad, torch.float64, (n, self.d), "grad")
        self._check_out(n_accept, torch.int64, (n,), "n_accept")
        if inv_mass is not None:
            self._check_out(inv_mass, torch.float64, (self.d,), "inv_mass")
        if n_invalid is not None:
            self._check_out(n_invalid, torch.int64, (n,), "n_invalid")
        if samples is not None:
            self._check_out(samples, torch.float64, (n_traj, n, self.d), "samples")
        im = C.c_void_p(inv_mass.data_ptr()) if inv_mass is not None else C.c_void_p()
        sm = C.c_void_p(samples.data_ptr()) if samples is not None else C.c_void_p()
        nv = C.c_void_p(n_invalid.data_ptr()) if n_invalid is not None else C.c_void_p()
        _lib.check(_lib.load().ptafs_hmc_run(
            self._h, n, int(n_traj), int(n_leapfrog), float(eps), im, C.c_uint64(seed),
            C.c_uint64(traj0), C.c_void_p(x.data_ptr()), C.c_void_p(logp.data_ptr()),
            C.c_void_p(grad.data_ptr()), C.c_void_p(n_accept.data_ptr()), sm, nv,
            int(bool(use_graph)), _stream_handle(stream)), "ptafs_hmc_run")


def _make_std_desc(desc, keep):
    """ptafs_std_desc for a mapping: the fields of a data set plus optional
    ``tm`` (n_toa x n_tm design matrix), ``spectrum`` ("powerlaw" or "free")
    and, with ``has_cw``, ``cw_nf`` (K_D, default 60) and ``cw_tspan`` (T_D,
    default twice ``tspan``) of the deterministic basis; ``split`` (0 or 1)
    for separate common-process and pulsar-noise coefficient sets."""
    def arr(a, dtype):
        a = np.ascontiguousarray(np.asarray(a), dtype=dtype)
        keep.append(a)
        return a

    d = _lib.StdDesc()
    d.n_psr = int(desc["n_psr"])
    d.toa_offsets = _ptr(arr(desc["toa_offsets"], np.int64), C.c_int64)
    d.t, d.dt, d.sigma, d.nu = (_ptr(arr(desc[k], np.float64), C.c_double) for k in ("t", "dt", "sigma", "nu"))
    d.backend = _ptr(arr(desc["backend"], np.int32), C.c_int32)
    efac = arr(desc["efac"], np.float64)
    d.n_backend = int(efac.size)
    d.efac = _ptr(efac, C.c_double)
    d.equad = _ptr(arr(desc["equad"], np.float64), C.c_double)
    d.psr_pos = _ptr(arr(desc["psr_pos"], np.float64), C.c_double)
    d.tspan = float(desc["tspan"])
    d.nf_rn, d.nf_gw, d.nf_dm = int(desc["nf_rn"]), int(desc["nf_gw"]), int(desc["nf_dm"])
    d.dm_scale = float(desc["dm_scale"])
    tm = desc.get("tm")
    if tm is None:
        d.n_tm, d.tm = 0, C.cast(None, _lib.c_double_p)
    else:
        tm = arr(tm, np.float64)
        d.n_tm, d.tm = int(tm.shape[1]), _ptr(tm, C.c_double)
    d.spectrum = 1 if desc.get("spectrum", "powerlaw") == "free" else 0
    d.prior_lo = _ptr(arr(desc["prior_lo"], np.float64), C.c_double)
    d.prior_hi = _ptr(arr(desc["prior_hi"], np.float64), C.c_double)
    d.has_cw = 1 if desc.get("has_cw", 0) else 0
    d.cw_nf = int(desc.get("cw_nf", 60)) if d.has_cw else 0
    d.cw_tspan = float(desc.get("cw_tspan", 2.0 * float(desc["tspan"]))) if d.has_cw else 0.0
    d.split = 1 if desc.get("split", 0) else 0
    return d


def ptafs_std_precompute_cw(desc, pulsar):
    """Host-only CW products of the standardized form for one pulsar:
    (F~^T N~^-1 F_D [p, 2 K_D], F_D^T N~^-1 dt [2 K_D], F_D^T N~^-1 F_D [2 K_D, 2 K_D])."""
    keep = []
    d = _make_std_desc(desc, keep)
    ka = max(int(desc["nf_rn"]), int(desc["nf_gw"]))
    p = 2 * ka + 2 * int(desc["nf_dm"])
    k2 = 2 * int(d.cw_nf)
    sd, ed, qd = np.zeros((p, k2)), np.zeros(k2), np.zeros((k2, k2))
    _lib.check(_lib.load().ptafs_std_precompute_cw(C.byref(d), int(pulsar), _ptr(sd, C.c_double),
                                                   _ptr(ed, C.c_double), _ptr(qd, C.c_double)),
               "ptafs_std_precompute_cw")
    return sd, ed, qd


def ptafs_std_precompute(desc, pulsar):
    """Host-only per-pulsar Gram quantities of the standardized form:
    (s0 [p, p], dvec [p], dt^T N~^-1 dt, -1/2 ln det(2 pi G^T N G), columns kept)."""
    keep = []
    d = _make_std_desc(desc, keep)
    ka = max(int(desc["nf_rn"]), int(desc["nf_gw"]))
    p = 2 * ka + 2 * int(desc["nf_dm"])
    s0 = np.zeros((p, p))
    dv = np.zeros(p)
    sc = np.zeros(3)
    _lib.check(_lib.load().ptafs_std_precompute(C.byref(d), int(pulsar), _ptr(s0, C.c_double),
                                                _ptr(dv, C.c_double), _ptr(sc, C.c_double)),
               "ptafs_std_precompute")
    return s0, dv, float(sc[0]), float(sc[1]), int(sc[2])


class StdDataset:
    """A data set in the standardized form (ptafs_std_create): timing model
    marginalised, CURN standardizing transform, optional tempering and free
    spectra.  Parameter vector [theta | z] (ptafs_std_layout)."""

    def __init__(self, desc, stream=None):
        lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libptafs needs a HIP GPU")
        keep = []
        d = _make_std_desc(desc, keep)
        h = C.c_void_p()
        _lib.check(lib.ptafs_std_create(C.byref(d), _stream_handle(stream), C.byref(h)), "ptafs_std_create")
        self._h = h
        self.layout = self.ptafs_std_layout(0)
        self.d = int(self.layout.d)

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().ptafs_std_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ptafs_std_layout(self, n_chains):
        out = _lib.StdLayoutInfo()
        _lib.check(_lib.load().ptafs_std_layout(self._h, int(n_chains), C.byref(out)), "ptafs_std_layout")
        return out

    def _x(self, x, inplace=False):
        return Dataset._check_x(self, x, inplace)

    def _beta(self, beta, n):
        if beta is None:
            return C.c_void_p()
        Dataset._check_out(beta, torch.float64, (n,), "beta")
        return C.c_void_p(beta.data_ptr())

    def ptafs_std_logp_grad(self, x, beta=None, out=None, stream=None):
        """(logp [C], grad [C, d], status [C]); beta: float64 [C] or None."""
        x = self._x(x)
        n = x.shape[0]
        if out is None:
            with torch.cuda.stream(stream) if stream is not None else _nullctx():
                logp = torch.empty(n, dtype=torch.float64, device=x.device)
                grad = torch.empty_like(x)
                status = torch.empty(n, dtype=torch.int32, device=x.device)
        else:
            logp, grad, status = out
            Dataset._check_out(logp, torch.float64, (n,), "logp")
            Dataset._check_out(grad, torch.float64, (n, self.d), "grad")
            Dataset._check_out(status, torch.int32, (n,), "status")
        _lib.check(_lib.load().ptafs_std_logp_grad(
            self._h, n, C.c_void_p(x.data_ptr()), self._beta(beta, n), C.c_void_p(logp.data_ptr()),
            C.c_void_p(grad.data_ptr()), C.c_void_p(status.data_ptr()), _stream_handle(stream)),
            "ptafs_std_logp_grad")
        return logp, grad, status

    STD_STAGES = ("transform", "prior", "adjoint", "finalize")

    def ptafs_std_profile_stages(self, x, beta=None, reps=10, stream=None):
        """Mean ms per stage of the standardized evaluation (HIP events)."""
        x = self._x(x)
        n = x.shape[0]
        logp = torch.empty(n, dtype=torch.float64, device=x.device)
        grad = torch.empty_like(x)
        status = torch.empty(n, dtype=torch.int32, device=x.device)
        ms = (C.c_double * 4)()
        _lib.check(_lib.load().ptafs_std_profile_stages(
            self._h, n, C.c_void_p(x.data_ptr()), self._beta(beta, n), C.c_void_p(logp.data_ptr()),
            C.c_void_p(grad.data_ptr()), C.c_void_p(status.data_ptr()), int(reps), ms,
            _stream_handle(stream)), "ptafs_std_profile_stages")
        return dict(zip(self.STD_STAGES, list(ms)))

    def ptafs_std_coefficients(self, x, beta=None, stream=None):
        """Fourier coefficients a = a_hat + L z, (C, n_psr, p); with split
        coefficients [a_G | a_R], (C, n_psr, pz)."""
        x = self._x(x)
        n = x.shape[0]
        lay = self.layout
        a = torch.empty((n, int(lay.n_psr), int(lay.pz)), dtype=torch.float64, device=x.device)
        _lib.check(_lib.load().ptafs_std_coefficients(
            self._h, n, C.c_void_p(x.data_ptr()), self._beta(beta, n), C.c_void_p(a.data_ptr()),
            _stream_handle(stream)), "ptafs_std_coefficients")
        return a

    def ptafs_std_hmc_run(self, x, logp, grad, n_accept, *, n_traj, n_leapfrog, eps, seed, traj0=0,
                          inv_mass=None, beta=None, samples=None, n_invalid=None, use_graph=True,
                          stream=None):
        x = self._x(x, inplace=True)
        n = x.shape[0]
        Dataset._check_out(logp, torch.float64, (n,), "logp")
        Dataset._check_out(grad, torch.float64, (n, self.d), "grad")
        Dataset._check_out(n_accept, torch.int64, (n,), "n_accept")
        if inv_mass is not None:
            Dataset._check_out(inv_mass, torch.float64, (self.d,), "inv_mass")
        if n_invalid is not None:
            Dataset._check_out(n_invalid, torch.int64, (n,), "n_invalid")
        if samples is not None:
            Dataset._check_out(samples, torch.float64, (n_traj, n, self.d), "samples")
        im = C.c_void_p(inv_mass.data_ptr()) if inv_mass is not None else C.c_void_p()
        sm = C.c_void_p(samples.data_ptr()) if samples is not None else C.c_void_p()
        nv = C.c_void_p(n_invalid.data_ptr()) if n_invalid is not None else C.c_void_p()
        _lib.check(_lib.load().ptafs_std_hmc_run(
            self._h, n, int(n_traj), int(n_leapfrog), float(eps), im, C.c_uint64(seed), C.c_uint64(traj0),
            self._beta(beta, n), C.c_void_p(x.data_ptr()), C.c_void_p(logp.data_ptr()),
            C.c_void_p(grad.data_ptr()), C.c_void_p(n_accept.data_ptr()), sm, nv, int(bool(use_graph)),
            _stream_handle(stream)), "ptafs_std_hmc_run")


def ptafs_dataset_create(desc, stream=None):
    return Dataset(desc, stream)


def ptafs_logp_grad(ds: Dataset, x, stream=None):
    return ds.ptafs_logp_grad(x, stream=stream)


def ptafs_logp_grad_plain(ds: Dataset, x, stream=None):
    return ds.ptafs_logp_grad_plain(x, stream=stream)


class LogPosterior(torch.autograd.Function):
    """log p(x) per chain with the hand-written adjoint as its backward.

    forward runs ptafs_logp_grad (which always produces the gradient) and
    saves it; backward returns grad_out[:, None] * d log p / d x."""

    @staticmethod
    def forward(ctx, x, ds):
        logp, grad, status = ds.ptafs_logp_grad(x.detach())
        ctx.save_for_backward(grad)
        ctx.mark_non_differentiable(status)
        return logp, status

    @staticmethod
    def backward(ctx, g_logp, g_status):
        (grad,) = ctx.saved_tensors
        return g_logp[:, None] * grad, None
