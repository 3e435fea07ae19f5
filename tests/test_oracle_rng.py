"""Pins of the oracle's random numbers: Philox4x32-10 against rocRAND's engine, the uniform
map, and the Box-Muller transform against special values and a normality test."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    subprocess.check_call([hipcc, "--cuda-host-only", "-x", "hip", "-O1",
                           os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe])

    def run(rows):
        inp = "".join(f"{s} {a} {b} {c} {d}\n" for s, (a, b, c, d) in rows)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
        return np.array([[int(t) for t in line.split()] for line in out.stdout.splitlines()],
                        dtype=np.uint64)
    return run


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(5)
    # rocRAND addresses counter words 0-1 through a 64-bit count of 32-bit outputs, so the
    # helper reaches word 1 only below 2^30 (word 1 is the filter's cycle counter)
    rows = [(0, (0, 0, 0, 0)), (2 ** 64 - 1, (2 ** 32 - 1, 2 ** 30 - 1, 2 ** 32 - 1, 2 ** 32 - 1)),
            (0x0123456789ABCDEF, (7, 3, 1, 0))]
    for _ in range(300):
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        ctr = tuple(int(v) for v in rng.integers(0, 2 ** 32, 4))
        ctr = (ctr[0], ctr[1] % 2 ** 30, ctr[2], ctr[3])
        rows.append((seed, ctr))
    # the counters the filter actually uses: (index, cycle, purpose, grid)
    rows += [(0, (i, k, p, 0)) for i in range(0, 4096, 97) for k in (0, 1, 99) for p in range(4)]
    ref = rocrand_ref(rows)
    got = np.array([orc.philox(list(c), s) for s, c in rows], dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_uniform_map_exact_and_open(orc):
    assert orc.uniform(0) == 0.5 * 2.0 ** -23
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert orc.uniform(0x1FF) == orc.uniform(0)  # the 9 low bits are dropped
    rng = np.random.default_rng(1)
    for b in rng.integers(0, 2 ** 32, 2000):
        u = orc.uniform(int(b))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # representable in FP32: both sides get the same u


def test_box_muller_special_values(orc):
    # radius sqrt(-2 ln u1) = 1 at u1 = e^{-1/2}; angle 2 pi u2
    u1 = math.exp(-0.5)
    n1, n2 = orc.box_muller(u1, 0.0)
    assert n1 == pytest.approx(1.0, abs=1e-15) and n2 == pytest.approx(0.0, abs=1e-15)
    n1, n2 = orc.box_muller(u1, 0.25)
    assert n1 == pytest.approx(0.0, abs=1e-15) and n2 == pytest.approx(1.0, abs=1e-15)
    n1, n2 = orc.box_muller(u1, 0.5)
    assert n1 == pytest.approx(-1.0, abs=1e-15) and n2 == pytest.approx(0.0, abs=1e-15)
    n1, n2 = orc.box_muller(math.exp(-2.0), 0.125)  # radius 2 at 45 degrees
    assert n1 == pytest.approx(math.sqrt(2), abs=1e-14)
    assert n2 == pytest.approx(math.sqrt(2), abs=1e-14)


def test_predict_noise_is_standard_normal(orc):
    p = orc.Params(64, 64, 0.2, 0.1, 0.99, 0.02, 0.1, 0.5, 4.0, 0.9, 1, 1, seed=11)
    n = 200_000
    z = orc.predict_noise(p, 3, n)
    for k in range(4):
        col = z[:, k]
        assert abs(col.mean()) < 5 / math.sqrt(n)
        assert abs(col.var() - 1) < 5 * math.sqrt(2 / n)
        assert stats.kstest(col, "norm").pvalue > 1e-4
    c = np.corrcoef(z.T)
    assert np.all(np.abs(c - np.eye(4)) < 5 / math.sqrt(n))
    # independent streams per cycle and per grid
    z2 = orc.predict_noise(p, 4, 1000)
    assert not np.allclose(z[:1000], z2)
