"""Pins for the oracle's random points (Philox4x32-10 and the counter layout).

The oracle's Philox is checked against (1) the published known-answer vectors
of Philox4x32-10 (SC'11 reference implementation) and (2) rocRAND's header-only
Philox engine run on the host, an implementation independent of the oracle,
over random counters/keys and over the exact counters the Vegas points use.
Uniformity of the resulting y is checked statistically.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_known_answer_vectors(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = orc.philox(ctr, key)
        assert [int(x) for x in got] == want


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "pins", "rocrand_philox_ref.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)

    def run(cases):
        text = "".join("%08x %08x %08x %08x %08x %08x\n" % (*c, *k) for c, k in cases)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    return run


def test_against_rocrand_random_counters(orc, rocrand_ref):
    rng = np.random.default_rng(123)
    cases = []
    for _ in range(200):
        c = [int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        k = [int(x) for x in rng.integers(0, 2**32, 2, dtype=np.uint64)]
        cases.append((c, k))
    cases.append(([0, 0, 0, 0], [0, 0]))
    cases.append(([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2))
    ref = rocrand_ref(cases)
    for (c, k), want in zip(cases, ref):
        assert [int(x) for x in orc.philox(c, k)] == want


def test_point_counter_layout_against_rocrand(orc, rocrand_ref):
    """y of event e, iteration t, problem p, dim i comes from word i%4 of
    Philox(ctr=(e lo, e hi, t, p*256 + i//4), key=(seed lo, seed hi))."""
    cases, meta = [], []
    for seed in (0, 1, 0xDEADBEEF12345678):
        for (t, p, e) in ((0, 0, 0), (3, 0, 12345), (9, 7, 2**32 + 5), (1, 255, 10**8 - 1)):
            d = 20
            for j in range(5):
                cases.append(([e & 0xFFFFFFFF, e >> 32, t, p * 256 + j], [seed & 0xFFFFFFFF, seed >> 32]))
            meta.append((seed, t, p, e, d))
    ref = rocrand_ref(cases)
    pos = 0
    for seed, t, p, e, d in meta:
        y = orc.point(seed, t, p, e, d)
        for j in range(5):
            words = ref[pos + j]
            for q in range(4):
                k = words[q]
                assert y[4 * j + q] == (k + 0.5) / 2**32
        pos += 5


def test_uniformity(orc):
    """y over many events: mean 1/2 and a flat histogram (chi^2, 64 cells)."""
    n, d = 20000, 8
    ys = np.array([orc.point(0, 0, 0, e, d) for e in range(n)])
    assert ys.min() > 0.0 and ys.max() < 1.0
    m = ys.mean()
    assert abs(m - 0.5) < 5 * np.sqrt(1 / 12 / ys.size)
    counts, _ = np.histogram(ys.ravel(), bins=64, range=(0, 1))
    expect = ys.size / 64
    chi2 = ((counts - expect) ** 2 / expect).sum()
    # 63 dof: mean 63, sd ~11.2; a 6 sd band
    assert 63 - 6 * 11.3 < chi2 < 63 + 6 * 11.3
    # dimensions are uncorrelated
    c = np.corrcoef(ys.T)
    off = c[~np.eye(d, dtype=bool)]
    assert np.abs(off).max() < 5 / np.sqrt(n)
