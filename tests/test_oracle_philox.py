"""Pins the oracle's Philox4x32-10 and its draw layout.

The oracle's generator is checked against rocRAND's Philox4x32-10 engine, an
independent open-source implementation of the same published bijection
(Salmon et al., SC'11), compiled here for the host.  The draw layout (which
16-bit slice feeds which variable) is then checked against the raw bijection.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROCRAND_HDR = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Probe : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  Probe p;
  unsigned a[6];
  while (scanf("%x %x %x %x %x %x", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
    uint4 c = {a[0], a[1], a[2], a[3]};
    uint2 k = {a[4], a[5]};
    uint4 o = p.run(c, k);
    printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_philox():
    if not os.path.exists(ROCRAND_HDR):
        pytest.skip("rocRAND header not installed")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "probe.cpp")
    exe = os.path.join(d, "probe")
    with open(src, "w") as f:
        f.write(PROBE)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", src, "-o", exe])

    def run(cases):
        inp = "\n".join(" ".join(f"{v:x}" for v in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return [tuple(int(t, 16) for t in line.split()) for line in out.strip().splitlines()]

    return run


def test_philox_matches_rocrand(orc, rocrand_philox):
    g = np.random.Generator(np.random.PCG64(7))
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 2, 3, 4, 5, 6)]
    cases += [tuple(int(v) for v in g.integers(0, 2**32, size=6, dtype=np.uint64))
              for _ in range(3000)]
    ref = rocrand_philox(cases)
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        seed = c[4] | (c[5] << 32)
        got = tuple(int(v) for v in orc.philox(c[:4], seed))
        assert got == r, (c, got, r)


def test_metropolis_draw_layout(orc):
    seed = 0x1234_5678_9ABC_DEF0
    for (r, s) in [(0, 0), (3, 17), (1023, 99_999)]:
        for i in range(0, 40):
            blk = orc.philox((i >> 3, s, r, 0), seed)
            word = int(blk[(i & 7) >> 1])
            want = (word >> 16) if (i & 1) else (word & 0xFFFF)
            assert orc.metropolis_draw(seed, r, s, i) == want


def test_other_draw_layouts(orc):
    seed = 99
    assert orc.select_draw(seed, 5, 7) == int(orc.philox((0, 7, 5, 1), seed)[0])
    assert orc.exchange_draw(seed, 2, 9, 4) == int(orc.philox((4, 9, 2, 2), seed)[0]) & 0xFFFF
    for i in range(300):
        blk = orc.philox((i >> 7, 0, 11, 3), seed)
        assert orc.init_bit(seed, 11, i) == (int(blk[(i >> 5) & 3]) >> (i & 31)) & 1


def test_draws_are_uniform(orc):
    # chi-square over 16 equal bins of the 16-bit Metropolis draws
    n = 40_000
    u = np.array([orc.metropolis_draw(5, r % 7, r // 7, r % 1000) for r in range(n)])
    counts = np.bincount(u >> 12, minlength=16)
    exp = n / 16
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 45.0  # 15 dof, p ~ 1e-4
