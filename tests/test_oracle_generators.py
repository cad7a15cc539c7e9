"""Pins of the oracle's generators against things other than itself.

Philox4x32-10: the published known-answer vectors and rocRAND's independent
engine.  FP32 Gaussian transform: exhaustive comparison over every possible
uniform with binary64 libm.  GUE: exact Hermiticity, partition invariance,
moments, the semicircle edge and E||H psi||^2 = 1.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(orc):
    for ctr, key, out in _kat():
        assert orc.philox(ctr, key).tolist() == out


def test_philox_matches_rocrand_engine(orc, tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = tmp_path / "rr_ref"
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    rng = np.random.default_rng(7)
    ctrs = rng.integers(0, 2 ** 32, size=(200, 4), dtype=np.uint64)
    keys = rng.integers(0, 2 ** 32, size=(200, 2), dtype=np.uint64)
    ctrs[:50, 2:] = 0  # the counter layout the GUE generator uses
    text = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k))
                     for c, k in zip(ctrs, keys)) + "\n"
    res = subprocess.run([str(exe)], input=text, capture_output=True,
                         text=True, check=True)
    got = [list(map(int, l.split())) for l in res.stdout.strip().splitlines()]
    for c, k, g in zip(ctrs, keys, got):
        assert orc.philox(c, k).tolist() == g


def test_philox_uniformity(orc):
    n = 1 << 16
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 12345
    out = orc.philox_many(ctr, (1, 0))
    words = out.ravel()
    # each of the 32 bit positions is set with probability 1/2
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(words.size))
    # chi-square of the top byte
    hist = np.bincount(words >> 24, minlength=256)
    assert stats.chisquare(hist).pvalue > 1e-4


def _all_uniforms():
    k = np.arange(1 << 23, dtype=np.uint64)
    return ((2 * k + 1).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def test_u01_exact(orc):
    for x in [0, 1, 511, 512, 0xFFFFFFFF, 0x80000000, 123456789]:
        want = ((x >> 9) * 2 + 1) * 2.0 ** -24
        assert float(orc.u01(x)) == want
        assert 0.0 < want < 1.0


def test_logf32_exhaustive(orc):
    u = _all_uniforms()
    got = orc.logf32(u).astype(np.float64)
    ref = np.log(u.astype(np.float64))
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(got - ref) / ulp) <= 2.0


def test_sincos2pi_exhaustive(orc):
    u = _all_uniforms()
    s, c = orc.sincos2pi_f32(u)
    th = 2 * np.pi * u.astype(np.float64)
    assert np.max(np.abs(s - np.sin(th))) <= 2.0 * 2.0 ** -24
    assert np.max(np.abs(c - np.cos(th))) <= 2.0 * 2.0 ** -24
    # quadrant symmetry holds exactly: sin(2 pi (1-u)) = -sin(2 pi u)
    s2, c2 = orc.sincos2pi_f32((1.0 - u.astype(np.float64)).astype(np.float32))
    assert np.array_equal(s2, -s) and np.array_equal(c2, c)


def test_box_muller_distribution(orc):
    rng = np.random.default_rng(11)
    x0 = rng.integers(0, 2 ** 32, 400000, dtype=np.uint64).astype(np.uint32)
    x1 = rng.integers(0, 2 ** 32, 400000, dtype=np.uint64).astype(np.uint32)
    z0, z1 = orc.box_muller_f32(x0, x1)
    for z in (z0, z1):
        assert abs(z.mean()) < 5 / np.sqrt(z.size)
        assert abs(z.var() - 1) < 0.02
        assert stats.kstest(z.astype(np.float64), "norm").pvalue > 1e-4
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 0.01
    # against binary64 evaluation of the same uniforms: a few ulp of r
    u0 = ((x0 >> 9).astype(np.float64) * 2 + 1) * 2.0 ** -24
    u1 = ((x1 >> 9).astype(np.float64) * 2 + 1) * 2.0 ** -24
    r = np.sqrt(-2 * np.log(u0))
    ulp_r = np.spacing(r.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(z0 - r * np.cos(2 * np.pi * u1)) / ulp_r) < 4
    assert np.max(np.abs(z1 - r * np.sin(2 * np.pi * u1)) / ulp_r) < 4


def test_gue_hermitian_bitwise(orc):
    D = 300
    H = orc.gue_entries(1, 0, 0, D, D, D=D)
    assert np.array_equal(H, H.conj().T)
    assert np.all(np.diag(H).imag == 0)


def test_gue_partition_invariance(orc):
    """Windows cut at different places see the same global entries."""
    D = 1000
    full = orc.gue_entries(5, 0, 0, D, D, D=D)
    for (r0, c0, nr, nc) in [(0, 0, 128, 128), (128, 512, 128, 256),
                             (700, 3, 300, 97), (999, 0, 1, 1000)]:
        w = orc.gue_entries(5, r0, c0, nr, nc, D=D)
        assert np.array_equal(w, full[r0:r0 + nr, c0:c0 + nc])


def test_gue_entry_statistics(orc):
    D = 2048
    H = orc.gue_dense(1, D)
    iu = np.triu_indices(D, 1)
    off = H[iu]
    assert abs(off.real.var() * 2 * D - 1) < 0.01
    assert abs(off.imag.var() * 2 * D - 1) < 0.01
    assert abs(np.diag(H).real.var() * D - 1) < 0.1
    assert stats.kstest(off.real[:200000] * np.sqrt(2 * D), "norm").pvalue > 1e-4
    # semicircle on [-2, 2]: extreme eigenvalues near the edges
    w = np.linalg.eigvalsh(H)
    assert 1.9 < w[-1] < 2.1 and -2.1 < w[0] < -1.9
    assert abs(np.trace(H).real) / D < 0.1
    # second moment of the spectrum: Tr(H^2)/D -> 1
    assert abs(np.mean(w ** 2) - 1) < 0.01


def test_gue_seeds_differ(orc):
    a = orc.gue_entries(1, 0, 0, 16, 16, D=16)
    b = orc.gue_entries(2, 0, 0, 16, 16, D=16)
    assert not np.any(a == b)
