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
