"""ptafs_logp_grad_noalloc (the entry point that allocates nothing: its
workspace is the library's static per-device array) against
ptafs_logp_grad, through the C ABI: bit-identical outputs on two calls in a
row, the second with a smaller input, and the size limit."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_06834_amd import _lib, api
    return _lib, api


def _outs(n, d):
    return (torch.empty(n, dtype=torch.float64, device="cuda"),
            torch.empty((n, d), dtype=torch.float64, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda"))


def _abi(lib, fn, ds, x, out):
    lp, gr, st = out
    s = torch.cuda.current_stream().cuda_stream
    return getattr(lib, fn)(ds._h, x.shape[0], C.c_void_p(x.data_ptr()), C.c_void_p(lp.data_ptr()),
                            C.c_void_p(gr.data_ptr()), C.c_void_p(st.data_ptr()), C.c_void_p(s))


def _near(ds, n, seed):
    th = synth.injected_theta(ds, seed, rn=(-14.0, 3.5), dm=(-14.0, 3.5))
    return synth.random_points(ds, n, seed + 1, theta=th, theta_jitter=0.3)


def test_noalloc_equals_allocating_entry_point(mods):
    _lib, api = mods
    lib = _lib.load()
    big = synth.make_array(71, 5, [300, 41, 16, 1, 257], 9 * synth.YEAR_S,
                           backends_per_psr=[1, 2, 3, 4, 1], nu_range=(0.4e9, 2e9),
                           nf_rn=9, nf_gw=6, nf_dm=5)
    small = synth.cfg1()
    cases = [(big, _near(big, 70, 3)), (small, _near(small, 20, 5))]   # second call smaller
    for ds_desc, X in cases:
        ds = api.Dataset(ds_desc)
        x = torch.tensor(X, device="cuda")
        ref, got = _outs(*X.shape), _outs(*X.shape)
        assert _abi(lib, "ptafs_logp_grad", ds, x, ref) == 0
        assert _abi(lib, "ptafs_logp_grad_noalloc", ds, x, got) == 0
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
        assert torch.all(ref[2] == 0)
        ds.close()


def test_noalloc_size_limit(mods):
    _lib, api = mods
    lib = _lib.load()
    ds_desc = synth.cfg1()
    ds = api.Dataset(ds_desc)
    n = 8192                                    # workspace ~200 MB > 128 MiB
    assert ds.ptafs_layout(n).workspace_bytes > (128 << 20)
    x = torch.tensor(_near(ds_desc, n, 7), device="cuda")
    out = _outs(n, ds.d)
    assert _abi(lib, "ptafs_logp_grad_noalloc", ds, x, out) == -4        # PTAFS_E_LIMIT
    ds.close()
