"""Pins of the oracle's RNG and samplers (no GPU).

* Philox4x32-10 against rocRAND's engine, compiled here for the host and run
  as a library (a third-party implementation of the published generator).
* Uniformity of the 24-bit uniforms by chi-square.
* Cosine-hemisphere sampler (paper, Section 3.2: rays drawn with a cosine
  weighting remove the dot product of eq. (1)): moments of cos(theta).
* Cone sampler (Section 3.1: directions inside the light's solid angle):
  support and the moments of a uniform-in-solid-angle cone.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    if shutil.which("hipcc") is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    subprocess.run(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "rocrand_philox_host.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_kat):
    rng = np.random.default_rng(1234)
    n = 2000
    keys = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    ctrs = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    ctrs[:, 1] %= 2 ** 30          # rocRAND's offset argument counts 32-bit words in 64 bits
    ctrs[:5] = 0                   # include the zero counter and small pixel-like counters
    ctrs[5:10, :2] = [[0, 0], [1, 0], [0, 1], [1919, 1079], [63, 63]]
    inp = "\n".join(" ".join(str(int(v)) for v in (*keys[i], *ctrs[i])) for i in range(n))
    out = subprocess.run([rocrand_kat], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array(out.split(), dtype=np.uint64).reshape(n, 4)
    mine = np.stack([orc.philox4x32_10(keys[i], ctrs[i:i + 1])[0] for i in range(n)]).astype(np.uint64)
    assert np.array_equal(ref, mine)


def test_philox_uniform_chi2(orc):
    from scipy import stats
    n = 1 << 18
    i = np.arange(n, dtype=np.uint64)
    ctr = np.stack([i % 1920, i // 1920, np.full(n, 7), np.full(n, 3)], axis=1).astype(np.uint32)
    r = orc.philox4x32_10((5, 11), ctr)
    for word in range(4):
        u = (r[:, word] >> 8).astype(np.float64) * 2.0 ** -24
        assert u.min() >= 0.0 and u.max() < 1.0
        counts = np.bincount((u * 256).astype(np.int64), minlength=256)
        chi2 = ((counts - n / 256) ** 2 / (n / 256)).sum()
        assert stats.chi2.sf(chi2, 255) > 1e-4, (word, chi2)
    # distinct keys give distinct streams
    r2 = orc.philox4x32_10((5, 12), ctr)
    assert (r2 != r).mean() > 0.99


def _uniforms(n, seed):
    rng = np.random.default_rng(seed)
    return rng.random((n, 2))


def test_cosine_sampler_moments(orc):
    n = 400_000
    rng = np.random.default_rng(3)
    normals = rng.normal(size=(n, 3))
    normals[:8] = [[0, 0, 1], [0, 0, -1], [0, 1, 0], [1, 0, 0], [0, 0, -1 + 1e-12], [0, 1e-9, -1], [1, 1, 1], [-1, 0, 0]]
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    d = orc.sample_cosine(normals, _uniforms(n, 4))
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    c = (d * normals).sum(1)
    assert c.min() >= 0.0
    # cos(theta) has density 2c on [0,1]: E[c] = 2/3, E[c^2] = 1/2
    se = np.sqrt(1 / 18 / n)
    assert abs(c.mean() - 2 / 3) < 5 * se
    assert abs((c ** 2).mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    # azimuth is uniform: the tangential component has zero mean in a fixed frame
    t = d - c[:, None] * normals
    z = np.array([0.0, 0.0, 1.0])
    m = np.abs(normals[:, 2]) < 0.5
    e1 = np.cross(normals[m], z); e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    assert abs((t[m] * e1).sum(1).mean()) < 5 * np.sqrt(1 / 4 / m.sum())


def test_onb_orthonormal(orc):
    # the sampler output for u0 = 0 is the normal itself; for u0 -> 1 it lies in the tangent plane
    rng = np.random.default_rng(5)
    n = rng.normal(size=(1000, 3))
    n[:4] = [[0, 0, 1], [0, 0, -1], [0, 0, -1 + 1e-15], [1e-300, 0, -1]]
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    u = np.zeros((1000, 2))
    np.testing.assert_allclose(orc.sample_cosine(n, u), n, atol=1e-12)
    for phi in (0.0, 0.25, 0.5, 0.75):
        u = np.column_stack([np.full(1000, 1.0 - 2.0 ** -24), np.full(1000, phi)])
        d = orc.sample_cosine(n, u)
        assert np.abs((d * n).sum(1)).max() < 1e-3
        np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    # quarter turns give orthogonal tangents
    a = orc.sample_cosine(n, np.column_stack([np.full(1000, 1.0), np.zeros(1000)]))
    b = orc.sample_cosine(n, np.column_stack([np.full(1000, 1.0), np.full(1000, 0.25)]))
    assert np.abs((a * b).sum(1)).max() < 1e-12


@pytest.mark.parametrize("half_deg", [0.0, 0.5, 1.0, 10.0, 60.0])
def test_cone_sampler(orc, half_deg):
    n = 200_000
    axis = np.array([0.3, 0.9, -0.2]); axis /= np.linalg.norm(axis)
    th = np.radians(half_deg)
    k = 2 * np.sin(th / 2) ** 2
    d = orc.sample_cone(axis, k, _uniforms(n, 6))
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    c = d @ axis
    assert c.min() >= np.cos(th) - 1e-12
    if half_deg == 0.0:
        np.testing.assert_allclose(d, np.broadcast_to(axis, d.shape), atol=1e-15)
        return
    # uniform in solid angle: cos(theta) uniform on [1-k, 1]
    assert abs(c.mean() - (1 - k / 2)) < 5 * k / np.sqrt(12 * n)
    frac = (c > 1 - k / 2).mean()
    assert abs(frac - 0.5) < 5 * np.sqrt(0.25 / n)
