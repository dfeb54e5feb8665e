"""Pins of the oracle's modified SVGF (no GPU).

Section 3.3 of the paper: temporal accumulation by an exponential moving
average over back-projected history, rejection of inconsistent history,
variance from moments or (without history) from a larger spatial kernel, and
an iterated edge-aware spatial kernel driven by that variance.

* T7  a constant image is left unchanged by the a-trous levels;
* T8  with all edge-stopping weights equal to one every level is a normalised
      dilated B3 convolution (scipy.ndimage.convolve);
* T9  with a static camera the first frames after a reset are the exact
      running mean (the 1/h ramp of the moving average), and the time average
      of the accumulated AO converges to the closed-form visibility of the
      floor beside a wall;
* T10 an integer-pixel motion shifts the history exactly; disocclusion,
      normal, plane-distance and id rejection reset it;
* variance from moments is the sample variance of the accumulated samples;
  the spatial fallback on a flat patch is the variance of the pooled moments;
* T13 the adjoint agrees with a forward-mode (dual number) JVP in the
      dot-product test and with central differences.

The lighter variant (one level of a 3x3 (1,2,1)/4 kernel, the outlook of
Section 3.3) is pinned the same way: constant image, unit weights against
scipy's convolution, one level against a hand-written 3x3 sum, and its
adjoint by the dot-product test.
"""
import numpy as np
import pytest
from scipy import ndimage

H1 = np.array([1, 4, 6, 4, 1]) / 16.0
K1 = np.array([1, 2, 1]) / 4.0
TAPS = {5: H1, 3: K1}


def _geom(W, H, seed, z_const=None, cone=0.3, invalid_frac=0.0):
    rng = np.random.default_rng(seed)
    n = np.column_stack([rng.normal(scale=cone, size=(W * H, 2)), np.ones(W * H)])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    z = np.full(W * H, z_const) if z_const is not None else rng.uniform(2.0, 3.0, W * H)
    nz = np.column_stack([n, z]).astype(np.float32)
    if invalid_frac:
        nz[rng.random(W * H) < invalid_frac] = 0.0
    dz = rng.normal(scale=0.05, size=(W * H, 2)).astype(np.float32)
    return nz, dz


# ---------------------------------------------------------------- a-trous pins

@pytest.mark.parametrize("kw", [5, 3])
def test_constant_image_unchanged(orc, kw):
    W, H = 37, 29
    nz, dz = _geom(W, H, 1, invalid_frac=0.1)
    rng = np.random.default_rng(2)
    cv = np.column_stack([np.full(W * H, 0.37), rng.uniform(0, 0.2, W * H)])
    P = orc.svgf_params(levels=5, kernel_width=kw)
    out = orc.svgf_spatial(P, W, H, cv, nz, dz)
    valid = nz[:, 3] > 0
    np.testing.assert_allclose(out[valid], 0.37, atol=1e-12)
    assert (out[~valid] == 1.0).all()


@pytest.mark.parametrize("kw", [5, 3])
def test_unit_weights_reduce_to_normalised_convolution(orc, kw):
    W, H = 45, 38
    nz, dz = _geom(W, H, 3, z_const=2.0, cone=0.2, invalid_frac=0.15)
    rng = np.random.default_rng(4)
    cv = np.column_stack([rng.random(W * H), rng.uniform(0.01, 0.3, W * H)])
    L = 4
    P = orc.svgf_params(levels=L, sigma_z=1.0, sigma_n=0.0, sigma_l=1e300, fp32=False, kernel_width=kw)
    R = kw // 2
    valid = (nz[:, 3] > 0).reshape(H, W)
    m = valid.astype(np.float64)
    c = cv[:, 0].reshape(H, W).copy()
    v = cv[:, 1].reshape(H, W).copy()
    cur = cv.copy()
    for level in range(L):
        s = 1 << level
        K = np.zeros((2 * R * s + 1, 2 * R * s + 1))
        K[::s, ::s] = np.outer(TAPS[kw], TAPS[kw])
        den = ndimage.convolve(m, K, mode="constant")
        c_ref = ndimage.convolve(c * m, K, mode="constant") / den
        v_ref = ndimage.convolve(v * m, K * K, mode="constant") / den ** 2
        nxt = orc.svgf_atrous(P, W, H, level, cur, nz, dz)
        np.testing.assert_allclose(nxt[:, 0].reshape(H, W)[valid], c_ref[valid], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(nxt[:, 1].reshape(H, W)[valid], v_ref[valid], rtol=1e-12, atol=1e-14)
        c, v, cur = c_ref, v_ref, nxt


def test_light_kernel_one_level_by_hand(orc):
    # one level of the 3x3 kernel written out for a few pixels: prefilter g,
    # the three stopping terms, then the weighted sums (stride 1)
    W, H = 9, 7
    nz, dz = _geom(W, H, 8, invalid_frac=0.1)
    rng = np.random.default_rng(9)
    cv = np.column_stack([rng.random(W * H), rng.uniform(0.01, 0.2, W * H)])
    P = orc.svgf_params(levels=1, sigma_z=0.7, sigma_n=40.0, sigma_l=3.0, fp32=False, kernel_width=3)
    out = orc.svgf_atrous(P, W, H, 0, cv, nz, dz)
    ok = lambda x, y: 0 <= x < W and 0 <= y < H and nz[y * W + x, 3] > 0
    for (x, y) in [(0, 0), (4, 3), (8, 6), (3, 0), (0, 5), (5, 5)]:
        p = y * W + x
        if not ok(x, y):
            continue
        G = sk = 0.0
        for b in (-1, 0, 1):
            for a in (-1, 0, 1):
                if ok(x + a, y + b):
                    k = K1[a + 1] * K1[b + 1]
                    G += k * cv[(y + b) * W + x + a, 1]
                    sk += k
        g = np.sqrt(G / sk)
        D = Sc = Sv = 0.0
        for b in (-1, 0, 1):
            for a in (-1, 0, 1):
                if not ok(x + a, y + b):
                    continue
                q = (y + b) * W + x + a
                w = 1.0
                if (a, b) != (0, 0):
                    zp, zq = float(nz[p, 3]), float(nz[q, 3])
                    wz = np.exp(-abs(zp - zq) / (0.7 * abs(a * float(dz[p, 0]) + b * float(dz[p, 1])) + 1e-4 * zp))
                    d = float(np.dot(nz[p, :3].astype(np.float64), nz[q, :3].astype(np.float64)))
                    wn = min(d, 1.0) ** 40.0 if d > 0 else 0.0
                    wl = np.exp(-abs(cv[p, 0] - cv[q, 0]) / (3.0 * g + 1e-4))
                    w = wz * wn * wl
                h = K1[a + 1] * K1[b + 1]
                D += h * w
                Sc += h * w * cv[q, 0]
                Sv += h * h * w * w * cv[q, 1]
        np.testing.assert_allclose(out[p], [Sc / D, Sv / D ** 2], rtol=1e-12, atol=1e-15)


def test_edge_stopping_blocks_across_depth_edge(orc):
    # two flat regions at very different depths: no leakage across the edge
    W, H = 32, 16
    nz = np.tile(np.array([0, 0, 1, 2.0], np.float32), (W * H, 1))
    nz.reshape(H, W, 4)[:, W // 2:, 3] = 20.0
    dz = np.zeros((W * H, 2), np.float32)
    cv = np.zeros((W * H, 2))
    cv.reshape(H, W, 2)[:, W // 2:, 0] = 1.0
    cv[:, 1] = 0.01
    out = orc.svgf_spatial(orc.svgf_params(levels=5), W, H, cv, nz, dz).reshape(H, W)
    assert out[:, : W // 2].max() < 1e-12 and out[:, W // 2:].min() > 1 - 1e-12


# --------------------------------------------------------------- temporal pins

def _plane_frame(W, H, z=5.0, oid=1):
    pos = np.zeros((W * H, 4), np.float32)
    yy, xx = np.divmod(np.arange(W * H), W)
    pos[:, 0] = xx * 0.01
    pos[:, 1] = yy * 0.01
    pos[:, 3] = np.array([oid], np.uint32).view(np.float32)[0]
    nz = np.tile(np.array([0, 0, 1, z], np.float32), (W * H, 1))
    return pos, nz


def test_static_camera_running_mean(orc):
    W, H, n_ao = 12, 10, 8
    pos, nz = _plane_frame(W, H)
    mv = np.zeros((W * H, 2), np.float32)
    P = orc.svgf_params()
    rng = np.random.default_rng(5)
    samples = rng.integers(0, n_ao + 1, size=(9, W * H)).astype(np.uint8)
    hist = None
    xs_hist = []
    for f in range(9):
        h = orc.svgf_temporal(P, W, H, n_ao, samples[f], pos, nz, mv, pos, nz, hist, 0.001)
        xs = samples[f] / n_ao
        xs_hist.append(xs)
        X = np.array(xs_hist)
        if f < 5:
            # a = max(0.2, 1/h) = 1/h for h <= 5: exact running mean of values and of squares
            np.testing.assert_allclose(h[:, 0], X.mean(0), atol=2e-6)
            np.testing.assert_allclose(h[:, 1], X.mean(0), atol=2e-6)
            np.testing.assert_allclose(h[:, 2], (X ** 2).mean(0), atol=2e-6)
        if f == 3:
            # four frames of history: variance from moments is the sample variance
            cv = orc.svgf_variance(P, W, H, h, nz, np.zeros((W * H, 2), np.float32))
            np.testing.assert_allclose(cv[:, 1], X.var(0), atol=4e-6)
        np.testing.assert_array_equal(h[:, 3], min(f + 1, 255))
        hist = h.astype(np.float32)
    # after the ramp the weight of a new sample stays at alpha = 0.2
    prev = hist[:, 0].astype(np.float64)
    h = orc.svgf_temporal(P, W, H, n_ao, samples[0], pos, nz, mv, pos, nz, hist, 0.001)
    np.testing.assert_allclose(h[:, 0], prev + 0.2 * (samples[0] / n_ao - prev), atol=1e-6)


def test_static_camera_converges_to_the_closed_form(orc):
    # floor beside an infinite wall, static camera: the time average of the
    # accumulated AO c' over many frames converges to each pixel's expected
    # visibility, the closed form V(d / r) of the wall pin
    from paper_2406_06963_amd import workloads as wl
    sc = wl.scene_plane_wall(wall_x=0.0)
    W, H = 40, 40
    cam = wl.Camera((-0.7, 2.5, 2.0), (-0.7, 0.0, -0.3))
    s = orc.Scene(sc.tris, sc.obj_id)
    pos, nz, _, _ = orc.gbuffer(s, cam, None, W, H)
    mv = np.zeros((W * H, 2), np.float32)
    P = orc.svgf_params()
    r, n_ao, F, skip = 1.0, 4, 240, 20
    pix = float(cam.pix_angle(H))
    hist, acc = None, np.zeros(W * H)
    for f in range(F):
        ao, _, _ = orc.trace(s, orc.trace_params(W, H, frame=f, seed=23, n_ao=n_ao, ao_radius=r, n_shadow=0), pos, nz)
        hist = orc.svgf_temporal(P, W, H, n_ao, ao, pos, nz, mv, pos, nz, hist, pix).astype(np.float32)
        if f >= skip:
            acc += hist[:, 0]
    est = acc / (F - skip)
    floor = (orc.id_bits(pos) == 0) & (nz[:, 3] > 0)
    d = -pos[:, 0].astype(np.float64)
    a = np.clip(d / r, 0.0, 1.0)
    V = 1.0 - (np.arccos(a) - a * np.sqrt(1.0 - a * a)) / np.pi
    sel = floor & (d > 0.0)
    bins = np.clip((d / r / 0.1).astype(int), 0, 12)
    checked = 0
    for b in range(13):
        m = sel & (bins == b)
        if m.sum() < 20:
            continue
        # the EMA's time average has about the variance of the plain sample
        # mean over the window; a factor 2 covers the correlation left
        sigma = 2.0 * np.sqrt((V[m] * (1 - V[m])).sum() / (n_ao * (F - skip))) / m.sum()
        assert abs(est[m].mean() - V[m].mean()) <= 5 * sigma + 1e-12, (b, est[m].mean(), V[m].mean(), sigma)
        checked += 1
    assert checked >= 8
    # per pixel too, well inside the noise of one pixel's window
    per_sigma = 2.0 * np.sqrt(V[sel] * (1 - V[sel]) / (n_ao * (F - skip)))
    assert (np.abs(est[sel] - V[sel]) <= 6 * per_sigma + 1e-12).mean() >= 0.999


def test_integer_shift_moves_history_exactly(orc):
    W, H, n_ao = 16, 8, 4
    pos, nz = _plane_frame(W, H)
    rng = np.random.default_rng(6)
    c = rng.random(W * H)
    hist_in = np.column_stack([c, c, c * c + 0.01, rng.integers(1, 9, W * H)]).astype(np.float32)
    ao = rng.integers(0, n_ao + 1, W * H).astype(np.uint8)
    P = orc.svgf_params()
    # previous frame: the world point of pixel x was at pixel x + 2
    prev_pos = pos.copy()
    prev_pos.reshape(H, W, 4)[:, :, 0] -= 0.02
    mv = np.tile(np.array([2.0, 0.0], np.float32), (W * H, 1))
    out = orc.svgf_temporal(P, W, H, n_ao, ao, pos, nz, mv, prev_pos, nz, hist_in, 0.001).reshape(H, W, 4)
    # reference: zero motion against the history rolled by two pixels
    shifted = np.roll(hist_in.reshape(H, W, 4), -2, axis=1).reshape(-1, 4)
    ref = orc.svgf_temporal(P, W, H, n_ao, ao, pos, nz, np.zeros_like(mv), pos, nz, shifted, 0.001).reshape(H, W, 4)
    np.testing.assert_array_equal(out[:, : W - 2], ref[:, : W - 2])
    # the last two columns map outside the image: disocclusion resets
    xs = (ao.reshape(H, W) / n_ao)[:, W - 2:]
    np.testing.assert_array_equal(out[:, W - 2:, 3], 1.0)
    np.testing.assert_array_equal(out[:, W - 2:, 0], xs)
    np.testing.assert_array_equal(out[:, W - 2:, 2], xs * xs)


@pytest.mark.parametrize("case", ["id", "normal30", "normal20", "plane5", "plane3", "nan", "nohist", "prev_invalid"])
def test_history_rejection(orc, case):
    W, H, n_ao = 6, 5, 4
    z, pix = 5.0, 0.002
    pos, nz = _plane_frame(W, H, z=z)
    prev_pos, prev_nz = pos.copy(), nz.copy()
    hist_in = np.tile(np.array([0.5, 0.5, 0.3, 6], np.float32), (W * H, 1))
    mv = np.zeros((W * H, 2), np.float32)
    ao = np.full(W * H, 1, np.uint8)
    accept = True
    if case == "id":
        prev_pos[:, 3] = np.array([7], np.uint32).view(np.float32)[0]
        accept = False
    elif case.startswith("normal"):
        a = np.radians(30.0 if case == "normal30" else 20.0)
        prev_nz[:, :3] = [np.sin(a), 0.0, np.cos(a)]
        accept = case == "normal20"          # cos 20 = 0.94 >= 0.9 > cos 30 = 0.87
    elif case.startswith("plane"):
        k = 5.0 if case == "plane5" else 3.0
        prev_pos[:, 2] += k * z * pix       # along the normal, k pixel footprints
        accept = case == "plane3"
    elif case == "nan":
        mv[:] = np.nan
        accept = False
    elif case == "nohist":
        hist_in = None
        accept = False
    elif case == "prev_invalid":
        prev_nz[:, 3] = 0.0
        accept = False
    out = orc.svgf_temporal(orc.svgf_params(), W, H, n_ao, ao, pos, nz, mv, prev_pos, prev_nz, hist_in, pix)
    if accept:
        np.testing.assert_array_equal(out[:, 3], 7.0)
        np.testing.assert_allclose(out[:, 0], 0.5 + 0.2 * (0.25 - 0.5))
    else:
        np.testing.assert_array_equal(out[:, 3], 1.0)
        np.testing.assert_array_equal(out[:, 0], 0.25)


def test_fallback_variance_is_pooled_moment_variance(orc):
    W, H = 15, 11
    pos, nz = _plane_frame(W, H)
    dz = np.zeros((W * H, 2), np.float32)
    rng = np.random.default_rng(8)
    m1 = rng.random(W * H)
    m2 = m1 ** 2 + rng.uniform(0, 0.05, W * H)
    hist = np.column_stack([m1, m1, m2, np.full(W * H, 2.0)])
    nz[rng.random(W * H) < 0.1] = 0.0            # some invalid pixels are skipped
    P = orc.svgf_params()
    cv = orc.svgf_variance(P, W, H, hist, nz, dz)
    valid = (nz[:, 3] > 0).reshape(H, W)
    M1 = m1.reshape(H, W)
    M2 = m2.reshape(H, W)
    for y in range(H):
        for x in range(W):
            if not valid[y, x]:
                continue
            sl = (slice(max(y - 3, 0), y + 4), slice(max(x - 3, 0), x + 4))
            msk = valid[sl]
            ref = M2[sl][msk].mean() - M1[sl][msk].mean() ** 2
            assert abs(cv[y * W + x, 1] - ref) < 1e-12
    np.testing.assert_array_equal(cv[valid.ravel(), 0], m1[valid.ravel()])


def test_variance_mixed_history_radius_and_depth_edge(orc):
    # pixels with >= 4 frames of history take max(0, mu2 - mu1^2) of their own
    # moments (clamped when rounding made it negative); the others pool the
    # moments of every valid neighbour in the (2R+1)^2 window whose depth
    # matches (with dz = 0 the depth weight is 1 on the same depth and 0 across
    # an edge of 10 units): law of total variance over that set
    W, H = 14, 9
    pos, nz = _plane_frame(W, H, z=2.0)
    nz.reshape(H, W, 4)[:, 9:, 3] = 12.0                   # a depth edge at x = 9
    dz = np.zeros((W * H, 2), np.float32)
    rng = np.random.default_rng(21)
    m1 = rng.random(W * H)
    m2 = m1 ** 2 + rng.uniform(0, 0.05, W * H)
    hl = np.where(rng.random(W * H) < 0.5, 2.0, 6.0)
    neg = (hl >= 4) & (rng.random(W * H) < 0.2)
    m2[neg] = m1[neg] ** 2 - 1e-3                           # rounding below mu1^2: clamped to 0
    hist = np.column_stack([m1, m1, m2, hl])
    valid = np.ones((H, W), bool)
    valid[3, 4] = valid[6, 10] = False
    nz[~valid.ravel()] = 0.0
    Z = nz[:, 3].reshape(H, W)
    M1, M2, HL = m1.reshape(H, W), m2.reshape(H, W), hl.reshape(H, W)
    for R in (1, 3):
        cv = orc.svgf_variance(orc.svgf_params(fallback_radius=R), W, H, hist, nz, dz)
        for y in range(H):
            for x in range(W):
                if not valid[y, x]:
                    continue
                got = cv[y * W + x, 1]
                if HL[y, x] >= 4:
                    assert got == max(0.0, M2[y, x] - M1[y, x] ** 2)
                    continue
                sl = (slice(max(y - R, 0), y + R + 1), slice(max(x - R, 0), x + R + 1))
                msk = valid[sl] & (Z[sl] == Z[y, x])
                ref = M2[sl][msk].mean() - M1[sl][msk].mean() ** 2
                assert abs(got - ref) < 1e-12, (R, x, y, got, ref)


# ------------------------------------------------------------------ adjoint pins

def _vjp_case(W, H, L, seed):
    rng = np.random.default_rng(seed)
    nz, dz = _geom(W, H, seed, invalid_frac=0.05)
    cv = np.column_stack([rng.random(W * H), rng.uniform(0.002, 0.05, W * H)])
    P = orc_params(L, rng)
    return nz, dz, cv, P


def orc_params(L, rng, kernel_width=5):
    import oracle
    return oracle.svgf_params(levels=L, sigma_z=rng.uniform(0.5, 2, L), sigma_n=rng.uniform(16, 128, L),
                              sigma_l=rng.uniform(1, 8, L), fp32=False, kernel_width=kernel_width)


@pytest.mark.parametrize("W,H,L,seed,kw", [(20, 16, 3, 1, 5), (40, 36, 5, 2, 5), (23, 17, 2, 3, 3)])
def test_adjoint_dot_product(orc, W, H, L, seed, kw):
    nz, dz, cv, P = _vjp_case(W, H, L, seed)
    P.kernel_width = kw
    rng = np.random.default_rng(seed + 100)
    v = rng.normal(size=W * H)
    dcv = rng.normal(size=(W * H, 2))
    ds = rng.normal(size=3 * L)
    Ju = orc.svgf_spatial_jvp(P, W, H, cv, nz, dz, dcv, ds)
    gcv, gs = orc.svgf_spatial_vjp(P, W, H, cv, nz, dz, v)
    lhs = Ju @ v
    rhs = (dcv * gcv).sum() + (ds * gs.ravel()).sum()
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + 1e-3), (lhs, rhs)
    # each input family alone (catches compensating errors)
    for mask in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        d2 = dcv * np.array(mask[:2], float)
        s2 = ds * mask[2]
        lhs = orc.svgf_spatial_jvp(P, W, H, cv, nz, dz, d2, s2) @ v
        rhs = (d2 * gcv).sum() + (s2 * gs.ravel()).sum()
        assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + 1e-3), (mask, lhs, rhs)


def test_adjoint_central_differences(orc):
    W, H, L = 24, 20, 4
    nz, dz, cv, P = _vjp_case(W, H, L, 7)
    rng = np.random.default_rng(11)
    g = rng.normal(size=W * H)
    gcv, gs = orc.svgf_spatial_vjp(P, W, H, cv, nz, dz, g)

    def loss(cv_, P_):
        return orc.svgf_spatial(P_, W, H, cv_, nz, dz) @ g

    for k in range(3):
        e = rng.normal(size=(W * H, 2))
        h = 1e-6
        fd = (loss(cv + h * e, P) - loss(cv - h * e, P)) / (2 * h)
        an = (e * gcv).sum()
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    import ctypes
    for fam, name in enumerate(("sigma_z", "sigma_n", "sigma_l")):
        for l in range(L):
            base = getattr(P, name)[l]
            h = 1e-6 * max(1.0, abs(base))
            Pp, Pm = type(P)(), type(P)()
            ctypes.pointer(Pp)[0] = P
            ctypes.pointer(Pm)[0] = P
            getattr(Pp, name)[l] = base + h
            getattr(Pm, name)[l] = base - h
            fd = (loss(cv, Pp) - loss(cv, Pm)) / (2 * h)
            assert abs(fd - gs[fam, l]) <= 1e-6 * max(1.0, abs(gs[fam, l])), (name, l, fd, gs[fam, l])


def test_tiny_negative_motion_uses_the_pixel_itself(orc):
    # mv = -1e-10 px: the fraction 1 - 1e-10 rounds to 1 in fp32, so only tap
    # 1 (at x - 1 + 1 = x) has a nonzero bilinear factor; the history must
    # come from the pixel itself with weight one
    W, H, n_ao = 6, 4, 4
    pos, nz = _plane_frame(W, H)
    rng = np.random.default_rng(12)
    c = rng.random(W * H)
    hist_in = np.column_stack([c, c, c * c, np.full(W * H, 3.0)]).astype(np.float32)
    ao = np.full(W * H, 2, np.uint8)
    P = orc.svgf_params()
    mv = np.full((W * H, 2), -1e-10, np.float32)
    out = orc.svgf_temporal(P, W, H, n_ao, ao, pos, nz, mv, pos, nz, hist_in, 0.001)
    ref = orc.svgf_temporal(P, W, H, n_ao, ao, pos, nz, np.zeros_like(mv), pos, nz, hist_in, 0.001)
    np.testing.assert_array_equal(out, ref)
    assert (out[:, 3] == 4.0).all()


# ------------------------------------------- fractional back-projection pins
#
# Section 3.3 back-projects each pixel with its motion vector into the
# previous frame and blends the history found there.  The blend is bilinear
# over the 2 x 2 pixels around the back-projected point, renormalised over
# the taps that survive the consistency tests, and the history length of the
# result is one more than the largest length among those taps (the reading
# of the history-length rule recorded in the design notes).  The expected
# values below come from facts that do not depend on how the weights are
# coded: a bilinear blend reproduces any function that is linear in x and y
# exactly, so over a linearly varying history the blend at p + mv is the
# linear function at p + mv; a partial blend is written out by hand.

def _linear_history(W, H):
    """History channels linear in (x, y); lengths 2, 7, 3, 5 by pixel parity
    (x even / odd, y even / odd), so any 2 x 2 footprint holds all four."""
    yy, xx = np.divmod(np.arange(W * H), W)
    c = 0.1 + 0.05 * xx + 0.02 * yy
    m1 = 0.2 + 0.03 * xx - 0.01 * yy
    m2 = 0.3 + 0.01 * xx + 0.04 * yy
    hl = np.array([[2.0, 7.0], [3.0, 5.0]])[yy % 2, xx % 2]
    return np.column_stack([c, m1, m2, hl]).astype(np.float32)


def _lin(x, y):
    """The three history channels at a continuous position (x, y)."""
    return (0.1 + 0.05 * x + 0.02 * y, 0.2 + 0.03 * x - 0.01 * y, 0.3 + 0.01 * x + 0.04 * y)


def _ema(hist_c, hist_m1, hist_m2, xs, a):
    return hist_c + a * (xs - hist_c), hist_m1 + a * (xs - hist_m1), hist_m2 + a * (xs * xs - hist_m2)


def _run_motion(orc, W, H, mv_xy, prev_pos=None):
    n_ao = 4
    pos, nz = _plane_frame(W, H)
    hist_in = _linear_history(W, H)
    ao = np.full(W * H, 1, np.uint8)            # x_s = 0.25 everywhere
    mv = np.tile(np.array(mv_xy, np.float32), (W * H, 1))
    pp = pos if prev_pos is None else prev_pos
    out = orc.svgf_temporal(orc.svgf_params(), W, H, n_ao, ao, pos, nz, mv, pp, nz, hist_in, 0.001)
    return out.reshape(H, W, 4), mv[0]


def test_fractional_motion_blends_a_linear_history_exactly(orc):
    # motion (0.25, 0.75): taps at x, x + 1 and y, y + 1 with fractions
    # 0.25 / 0.75; every interior pixel sees history lengths {2, 7, 3, 5}
    W, H = 8, 6
    out, _ = _run_motion(orc, W, H, (0.25, 0.75))
    # one pixel by hand: (2, 1) back-projects to (2.25, 1.75)
    #   c = 0.1 + 0.05 * 2.25 + 0.02 * 1.75 = 0.2475, mu1 = 0.25, mu2 = 0.3925
    #   h' = 1 + max(2, 7, 3, 5) = 8, a = max(0.2, 1 / 8) = 0.2
    #   c' = 0.2475 + 0.2 * (0.25 - 0.2475) = 0.248
    #   mu1' = 0.25, mu2' = 0.3925 + 0.2 * (0.0625 - 0.3925) = 0.3265
    np.testing.assert_allclose(out[1, 2], [0.248, 0.25, 0.3265, 8.0], rtol=0, atol=1e-6)
    # every pixel whose four taps lie inside the image
    for y in range(H - 1):
        for x in range(W - 1):
            ref = _ema(*_lin(x + 0.25, y + 0.75), 0.25, 0.2)
            np.testing.assert_allclose(out[y, x, :3], ref, rtol=0, atol=1e-6, err_msg=f"{(x, y)}")
            assert out[y, x, 3] == 8.0, (x, y)


def test_fractional_negative_motion_and_the_image_border(orc):
    # motion (-0.6, 0.3) in fp32: floor (-1, 0), fractions (0.4, 0.3)
    W, H = 8, 6
    out, mv = _run_motion(orc, W, H, (-0.6, 0.3))
    mx, my = float(mv[0]), float(mv[1])
    for y in range(H - 1):
        for x in range(1, W):
            ref = _ema(*_lin(x + mx, y + my), 0.25, 0.2)
            np.testing.assert_allclose(out[y, x, :3], ref, rtol=0, atol=1e-6, err_msg=f"{(x, y)}")
            assert out[y, x, 3] == 8.0, (x, y)
    # column 0: the taps at x = -1 are outside, the two at x = 0 remain with
    # weights 0.4 * 0.7 and 0.4 * 0.3, renormalised by their sum 0.4: a linear
    # blend along y only.  Their lengths are 2 and 3 (x even), so h' = 4 and
    # the ramp gives a = max(0.2, 1 / 4) = 0.25.
    for y in range(H - 1):
        hl = 1.0 + max(2.0 if y % 2 == 0 else 3.0, 3.0 if y % 2 == 0 else 2.0)
        assert hl == 4.0
        ref = _ema(*_lin(0.0, y + my), 0.25, 0.25)
        np.testing.assert_allclose(out[y, 0, :3], ref, rtol=0, atol=1e-6, err_msg=f"{y}")
        assert out[y, 0, 3] == 4.0
    # by hand for (0, 2): c = 0.1 + 0.02 * 2.3 = 0.146, c' = 0.146 + 0.25 * (0.25 - 0.146) = 0.172
    assert abs(out[2, 0, 0] - 0.172) <= 1e-6
    # bottom row: the taps at y = H are outside, a blend along x only
    for x in range(1, W):
        hl = 1.0 + max(2.0, 7.0) if (H - 1) % 2 == 0 else 1.0 + max(3.0, 5.0)
        a = max(0.2, 1.0 / hl)
        ref = _ema(*_lin(x + mx, H - 1), 0.25, a)
        np.testing.assert_allclose(out[H - 1, x, :3], ref, rtol=0, atol=1e-6, err_msg=f"{x}")
        assert out[H - 1, x, 3] == hl


def test_rejected_tap_renormalises_the_rest(orc):
    # motion (0.25, 0.75); the history sample at (3, 2) belongs to another
    # object, so pixel (2, 1) keeps three of its four taps
    W, H = 8, 6
    pos, _ = _plane_frame(W, H)
    prev_pos = pos.copy()
    prev_pos[2 * W + 3, 3] = np.array([9], np.uint32).view(np.float32)[0]
    out, _ = _run_motion(orc, W, H, (0.25, 0.75), prev_pos=prev_pos)
    # bilinear factors of (2, 1), (3, 1), (2, 2), (3, 2): 3/16, 1/16, 9/16, 3/16;
    # without the last the weights are 3/13, 1/13, 9/13
    c = (3 * 0.22 + 0.27 + 9 * 0.24) / 13            # c at (2,1), (3,1), (2,2)
    m1 = (3 * 0.25 + 0.28 + 9 * 0.24) / 13
    m2 = (3 * 0.36 + 0.37 + 9 * 0.40) / 13
    # lengths of the surviving taps: 3, 5, 2 -> h' = 6, a = max(0.2, 1/6) = 0.2
    np.testing.assert_allclose(out[1, 2], [c + 0.2 * (0.25 - c), m1 + 0.2 * (0.25 - m1),
                                           m2 + 0.2 * (0.0625 - m2), 6.0], rtol=0, atol=1e-6)
    # the rejected sample is also the (0, 0) tap of pixel (3, 2), the (1, 0)
    # tap of (2, 2), the (0, 1) tap of (3, 1) and the (1, 1) tap of (2, 1);
    # pixels whose footprint avoids it are unaffected
    ref = _ema(*_lin(5 + 0.25, 3 + 0.75), 0.25, 0.2)
    np.testing.assert_allclose(out[3, 5, :3], ref, rtol=0, atol=1e-6)
    # (3, 2): its own sample (3/16) is rejected; (4, 2) 1/16, (3, 3) 9/16 and
    # (4, 3) 3/16 remain -> weights 1/13, 9/13, 3/13 on c = 0.34, 0.31, 0.36;
    # lengths 2, 5, 3 -> h' = 6
    c = (0.34 + 9 * 0.31 + 3 * 0.36) / 13
    np.testing.assert_allclose(out[2, 3, 0], c + 0.2 * (0.25 - c), rtol=0, atol=1e-6)
    assert out[2, 3, 3] == 6.0


def test_short_histories_take_the_ramp_of_the_longest_tap(orc):
    # lengths {1, 2, 1, 3} by parity: h' = 1 + 3 = 4, so a = 1/4 > alpha;
    # a blend of the lengths would give a non-integer h' and another a
    W, H, n_ao = 6, 4, 4
    pos, nz = _plane_frame(W, H)
    hist_in = _linear_history(W, H)
    yy, xx = np.divmod(np.arange(W * H), W)
    hist_in[:, 3] = np.array([[1.0, 2.0], [1.0, 3.0]])[yy % 2, xx % 2]
    ao = np.full(W * H, 3, np.uint8)            # x_s = 0.75
    mv = np.tile(np.array([0.5, 0.25], np.float32), (W * H, 1))
    out = orc.svgf_temporal(orc.svgf_params(), W, H, n_ao, ao, pos, nz, mv, pos, nz, hist_in, 0.001)
    out = out.reshape(H, W, 4)
    for y in range(H - 1):
        for x in range(W - 1):
            ref = _ema(*_lin(x + 0.5, y + 0.25), 0.75, 0.25)
            np.testing.assert_allclose(out[y, x, :3], ref, rtol=0, atol=1e-6, err_msg=f"{(x, y)}")
            assert out[y, x, 3] == 4.0
