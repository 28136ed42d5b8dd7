"""CPU-side checks of the C-ABI library (no GPU work is launched).

* libdapt.so loads and exports every function include/da.h declares.
* The library's host-built Metropolis threshold tables and schedule levels --
  the data the device decides against -- are bit-identical to the ones the
  oracle builds independently from the same definition.
* The admission footprint grows with every input it depends on.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "da.h")


@pytest.fixture(scope="module")
def api():
    from paper_1806_08815_amd import api as a
    a.lib()
    return a


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(da_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_exports_every_declared_symbol(api):
    names = _declared()
    assert len(names) >= 20, names
    lib = ctypes.CDLL(api.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("T", [0.0, 0.05, 0.1, 1.0, 3.0, 32.0 * 3, 3277.0, 196608.0, 5e8])
def test_threshold_tables_match_oracle(api, orc, T):
    assert np.array_equal(api.da_threshold_table(T), orc.threshold_table(T))


@pytest.mark.parametrize("kind,L", [("geometric", 128), ("linear_beta", 50), ("geometric", 1)])
def test_schedule_levels_match_oracle(api, orc, kind, L):
    sch = api.schedule(3.0 * 65536, 0.05 * 65536, kind, L)
    k = 0 if kind == "geometric" else 1
    for l in range(L):
        assert api.da_level_temperature(sch, l) == orc.level_temperature(
            3.0 * 65536, 0.05 * 65536, k, L, l)


def test_footprint(api):
    f = api.da_job_footprint
    base = f(1000, 2, 64, 128)
    assert base > 1024 * 1024 * 2
    assert f(2000, 2, 64, 128) > base and f(1000, 4, 64, 128) > base
    assert f(1000, 2, 128, 128) > base and f(1000, 2, 64, 256) > base
    assert f(0, 2, 64, 128) == -1 and f(10, 3, 1, 1) == -1


def test_strerror(api):
    assert api.da_strerror(api.DA_ENOMEM) == "out of memory"
    assert api.da_strerror(12345) == "unknown status"


def test_state_bytes(api):
    # header (32 bytes) + per replica x, best x (N bytes each), h (4N), E, best E,
    # accepted count (8 each), offset (4)
    assert api.da_state_bytes(100, 3) == 32 + 3 * (6 * 100 + 28)
    assert api.da_state_bytes(8192, 1) == 32 + 6 * 8192 + 28
    assert api.da_state_bytes(0, 1) == -1 and api.da_state_bytes(10, 0) == -1
    assert api.da_state_bytes(8193, 1) == -1


def test_ladder_update_matches_oracle(api, orc):
    """The adaptive-ladder update (Sec. II.D, Hukushima's scheme) decides the
    temperatures of later PT runs, so the library's and the oracle's independent
    writings of it must agree to the bit."""
    g = np.random.Generator(np.random.PCG64(17))
    for trial in range(300):
        M = int(g.integers(1, 48))
        temps = np.cumsum(g.uniform(0.01, 5.0, size=M)) + g.uniform(0.01, 1.0)
        proposals = int(g.integers(0, 5000))
        acc = g.integers(0, proposals + 1, size=max(M - 1, 1))
        if trial % 7 == 0:
            acc[:] = 0
        got = api.da_pt_ladder_update(temps, acc[:max(M - 1, 0)] if M > 1 else acc, proposals)
        want = orc.ladder_update(temps, acc, proposals)
        assert np.array_equal(got, want), (M, proposals)
