"""Host logic of the autotuner (no GPU): the chunk sizes that fill whole
rounds of the device's wave slots."""
import numpy as np
import pytest

import synth
from paper_2607_06834_amd import autotune


def waves(offsets, n_chains, tpc, wpb=1):
    tiles = (np.diff(np.asarray(offsets)) + 15) // 16
    return int(np.maximum(1, -(-tiles // tpc)).sum()) * ((n_chains + 15) // 16) * wpb


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("wpb", [1, 4])
def test_round_fitting_is_the_smallest_chunk_that_fits(seed, wpb):
    rng = np.random.default_rng(seed)
    counts = rng.integers(16, 4000, size=int(rng.integers(3, 90)))
    off = np.concatenate([[0], np.cumsum(counts)])
    n_cu, chains = 256, int(rng.integers(1, 129))
    got = autotune.round_fitting_tpcs(off, chains, n_cu, wpb=wpb)
    assert got == sorted(set(got))
    expect = set()
    for r in (1, 2):
        for occ in (1, 2, 3, 4):
            slots = r * n_cu * 4 * occ
            fit = [t for t in range(1, int(((counts + 15) // 16).max()) + 1)
                   if waves(off, chains, t, wpb) <= slots]
            if fit:
                expect.add(min(fit))
    assert set(got) == expect
    for t in got:
        assert waves(off, chains, t, wpb) <= 2 * n_cu * 4 * 4


def test_round_fitting_benchmark_shape():
    """67 pulsars / 250k TOAs / 64 chains on 256 compute units: 33 tiles per
    chunk put 2032 one-wave workgroups on the 2048 slots of two waves per SIMD."""
    import synth
    ds = synth.cfg2()
    got = autotune.round_fitting_tpcs(ds["toa_offsets"], 64, 256)
    assert 33 in got
    assert waves(ds["toa_offsets"], 64, 33) <= 2048 < waves(ds["toa_offsets"], 64, 32)


def test_serving_tuning_is_a_function_of_shape():
    """The serving tuning is fixed by the request's shape and the device's
    compute-unit count alone (never timed), so a request gets the same
    reduction order alone and in any mix."""
    ds = synth.cfg1()
    a = autotune.serving_tuning(ds["toa_offsets"], 16, 256)
    b = autotune.serving_tuning(ds["toa_offsets"], 16, 256)
    assert a == b and a[1] == 1 and a[2] == 2 and 4 <= a[0] <= 32
    big = synth.serving_request(505)
    t = autotune.serving_tuning(big["toa_offsets"], 16, 256)
    assert 4 <= t[0] <= 32
