"""The C-ABI library loads and exports every function include/ptafs.h declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ptafs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ptafs_[a-z_]+)\s*\(", src)))


def test_header_declares_boundary():
    names = declared_functions()
    for n in ("ptafs_dataset_create", "ptafs_dataset_destroy", "ptafs_layout", "ptafs_logp_grad",
              "ptafs_logp_grad_plain", "ptafs_hmc_run", "ptafs_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2607_06834_amd import _lib
    assert os.path.exists(_lib.LIB_PATH), "build libptafs.so first (__graft_entry__.build())"
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_strerror_without_gpu():
    from paper_2607_06834_amd import _lib
    lib = _lib.load()
    assert lib.ptafs_strerror(0) == b"success"
    assert lib.ptafs_strerror(-4).startswith(b"size exceeds")
    assert lib.ptafs_strerror(12345) == b"unknown error"


def test_slot_mapping_covers_rows():
    """The basis-row mapping of the TOA pass is a bijection between harmonic
    sin/cos slots (plus the three timing-model columns) and rows."""
    import itertools
    for kb in range(1, 31):
        rows = set()
        for k, sc in itertools.product(range(1, kb + 1), (0, 1)):
            h = k - 1
            rows.add(4 * (2 * (h >> 2) + sc) + (h & 3))
        for ti in range(3):
            h = kb + (ti >> 1)
            rows.add(4 * (2 * (h >> 2) + (ti & 1)) + (h & 3))
        assert len(rows) == 2 * kb + 3
        pairs = kb + 2
        tiles = (2 * ((pairs + 3) // 4) + 3) // 4
        assert max(rows) < 16 * tiles


def test_estimate_without_gpu():
    """ptafs_estimate sizes a data set from its descriptor on the host: the
    layout matches the oracle's, memory grows with the data, and invalid
    descriptors are refused with the create call's error codes."""
    import numpy as np
    import synth
    from oracle import model
    from paper_2607_06834_amd import api
    ds = synth.make_array(5, 4, [30, 40, 50, 60], 8 * synth.YEAR_S, backends_per_psr=[1, 2, 1, 2],
                          nu_range=(0.4e9, 2e9), nf_rn=5, nf_gw=3, nf_dm=4, has_cw=True)
    est = api.ptafs_estimate(ds, 16)
    ref = model.Layout(4, 5, 3, 4, True)
    assert (est.d, est.n_theta, est.off_u, est.off_z, est.off_zdm, est.off_cw) == \
        (ref.d, ref.n_theta, ref.u, ref.z, ref.zdm, ref.cw)
    big = synth.make_array(5, 4, [300, 400, 500, 600], 8 * synth.YEAR_S, backends_per_psr=[1, 2, 1, 2],
                           nu_range=(0.4e9, 2e9), nf_rn=5, nf_gw=3, nf_dm=4, has_cw=True)
    e2 = api.ptafs_estimate(big, 16)
    assert e2.dataset_bytes > est.dataset_bytes and e2.workspace_bytes > est.workspace_bytes
    assert api.ptafs_estimate(ds, 64).workspace_bytes > est.workspace_bytes
    assert api.ptafs_estimate(ds, 64).hmc_bytes > est.hmc_bytes
    bad = dict(ds)
    bad["sigma"] = -np.asarray(ds["sigma"])
    try:
        api.ptafs_estimate(bad, 16)
        raise AssertionError("negative sigma accepted")
    except RuntimeError as e:
        assert "invalid argument" in str(e)
