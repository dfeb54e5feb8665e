"""Pins of the oracle's intersection and BVH (no GPU).

The paper groups objects in a bounding-volume hierarchy so that rays skip
whole groups (Section 3.2); the plain definition of visibility is brute force
over all triangles.  The oracle's BVH must agree with brute force exactly,
also on grazing rays, rays through shared edges and vertices, and rays along
the coordinate axes.
"""
import numpy as np
import pytest

from paper_2406_06963_amd import workloads as wl


def _grazing_rays(tris, rng, n):
    """Rays aimed at vertices, edge midpoints and along triangle planes."""
    T = tris.shape[0]
    k = rng.integers(0, T, size=n)
    kind = rng.integers(0, 4, size=n)
    tri = tris[k].astype(np.float64)
    bary = np.where(kind[:, None] == 0, np.eye(3)[rng.integers(0, 3, size=n)],
                    np.where(kind[:, None] == 1, np.array([0.5, 0.5, 0.0])[[0, 1, 2]][None].repeat(n, 0),
                             rng.dirichlet([1, 1, 1], size=n)))
    target = np.einsum("ni,nij->nj", bary, tri)
    o = rng.uniform(-2, 2, size=(n, 3))
    # kind 3: origin inside the triangle's plane (ray along the plane)
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    inplane = tri[:, 0] + rng.uniform(-1, 2, size=(n, 1)) * e1 + rng.uniform(-1, 2, size=(n, 1)) * e2
    o = np.where(kind[:, None] == 3, inplane, o)
    d = target - o
    d /= np.linalg.norm(d, axis=1, keepdims=True) + 1e-300
    return o, d


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_bvh_anyhit_equals_brute_force(orc, seed):
    rng = np.random.default_rng(seed)
    T = int(rng.integers(1, 65))
    sc = wl.random_triangles(T, seed=seed)
    s = orc.Scene(sc.tris, sc.obj_id)
    n = 25_000
    o1 = rng.uniform(-2, 2, size=(n, 3))
    d1 = rng.normal(size=(n, 3))
    d1 /= np.linalg.norm(d1, axis=1, keepdims=True)
    o2, d2 = _grazing_rays(sc.tris, rng, n)
    # axis-aligned directions (zero components)
    o3 = rng.uniform(-2, 2, size=(n, 3))
    d3 = np.eye(3)[rng.integers(0, 3, size=n)] * rng.choice([-1.0, 1.0], size=(n, 1))
    # rays starting exactly on a triangle, leaving it
    k = rng.integers(0, T, size=n)
    bary = rng.dirichlet([1, 1, 1], size=n)
    o4 = np.einsum("ni,nij->nj", bary, sc.tris[k].astype(np.float64))
    d4 = rng.normal(size=(n, 3)); d4 /= np.linalg.norm(d4, axis=1, keepdims=True)
    o = np.concatenate([o1, o2, o3, o4])
    d = np.concatenate([d1, d2, d3, d4])
    tmax = np.where(rng.random(4 * n) < 0.5, np.inf, rng.uniform(0.0, 4.0, size=4 * n))
    hb, hf = s.anyhit(o, d, tmax)
    assert hf.sum() > 1000 and (1 - hf).sum() > 1000
    assert np.array_equal(hb, hf)
    t_b, i_b = s.closest(o, d)
    t_f, i_f = s.closest(o, d, brute=True)
    assert np.array_equal(i_b, i_f)
    assert np.array_equal(t_b[i_b >= 0], t_f[i_f >= 0])


def test_moller_trumbore_hand_cases(orc):
    tri = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32)
    s = orc.Scene(tri)
    o = np.array([[0.25, 0.25, 1.0],    # interior, t = 1
                  [0.0, 0.0, 2.0],      # vertex (inclusive), t = 2
                  [0.5, 0.5, 3.0],      # on the hypotenuse (inclusive), t = 3
                  [0.6, 0.6, 1.0],      # outside
                  [0.25, 0.25, -1.0],   # behind the origin (t < 0)
                  [0.25, 0.25, 1.0],    # parallel (det == 0)
                  [0.25, 0.25, -1.0]])  # from below, two-sided, t = 1
    d = np.array([[0, 0, -1], [0, 0, -1], [0, 0, -1], [0, 0, -1], [0, 0, -1], [1, 0, 0], [0, 0, 1]], float)
    t, idx = s.closest(o, d, brute=True)
    np.testing.assert_array_equal(idx, [0, 0, 0, -1, -1, -1, 0])
    np.testing.assert_array_equal(t[[0, 1, 2, 6]], [1.0, 2.0, 3.0, 1.0])
    # any-hit is strict in t: t == tmax is not a hit (eq. (3): beyond the radius is unoccluded)
    hb, hf = s.anyhit(o[:1], d[:1], np.array([1.0]))
    assert hb[0] == 0 and hf[0] == 0
    hb, hf = s.anyhit(o[:1], d[:1], np.array([np.nextafter(1.0, 2.0)]))
    assert hb[0] == 1 and hf[0] == 1


def test_closest_tie_breaks_to_smallest_index(orc):
    # two coincident triangles: the lower original index wins
    t = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]] * 3, np.float32)
    s = orc.Scene(t, np.array([7, 8, 9], np.uint32))
    tt, idx = s.closest(np.array([[0.2, 0.2, 1.0]]), np.array([[0.0, 0.0, -1.0]]))
    assert idx[0] == 0 and tt[0] == 1.0


def test_bvh_depth_reasonable(orc):
    sc = wl.make_scene("room")
    s = orc.Scene(sc.tris, sc.obj_id)
    assert s.depth <= 2 + int(np.ceil(np.log2(sc.n_tris / 4)))
