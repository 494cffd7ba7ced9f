"""Pins for the oracle renderers (Section 4): majorant grid, emission-
absorption marching, delta tracking and the path tracer.  Closed forms,
brute force, library interpolation and an independent analytic Monte Carlo
estimator stand against the oracle."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import scenes

TF5 = dict(tf=[(0.2, 0.3, 0.9, 0.0), (0.9, 0.1, 0.2, 0.8), (0.4, 0.4, 0.4, 0.3),
               (1.0, 1.0, 0.0, 1.0), (0.0, 1.0, 1.0, 0.5)], tf_range=(0.1, 0.9))


def _f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def _alpha(med, s):
    tf = _f32(med["tf"])
    lo, hi = _f32(med.get("tf_range", (0.0, 1.0)))
    xs = lo + np.arange(len(tf)) * (hi - lo) / (len(tf) - 1)
    return np.interp(s, xs, tf[:, 3])


def _rgb(med, s):
    tf = _f32(med["tf"])
    lo, hi = _f32(med.get("tf_range", (0.0, 1.0)))
    xs = lo + np.arange(len(tf)) * (hi - lo) / (len(tf) - 1)
    return np.array([np.interp(s, xs, tf[:, c]) for c in range(3)])


def _vol(shape, seed, zero=0.5):
    rng = np.random.default_rng(seed)
    v = rng.random(shape, dtype=np.float32)
    v[rng.random(shape) < zero] = 0.0
    return v


# ------------------------------ majorant ------------------------------

@pytest.mark.parametrize("C", [4, 8, 16])
def test_majorant_bruteforce(C):
    v = _vol((21, 26, 30), 1)
    buf, st = oracle.encode(v, 0.5)
    R = oracle.reconstruct(v, 0.5)
    B = st["background"]
    med = dict(sigma_scale=5.0, **TF5)
    maj = oracle.majorant(oracle.VdbField(buf), med, C)
    nz, ny, nx = v.shape
    gz, gy, gx = maj.shape
    pad = np.full((gz * C + 2, gy * C + 2, gx * C + 2), B, np.float32)
    pad[1:nz + 1, 1:ny + 1, 1:nx + 1] = R
    ds = 5.0 / max(v.shape)
    tf = np.asarray(med["tf"])
    lo, hi = _f32(med["tf_range"])
    knots = lo + np.arange(len(tf)) * (hi - lo) / (len(tf) - 1)
    for cz in range(gz):
        for cy in range(gy):
            for cx in range(gx):
                blk = pad[cz * C:cz * C + C + 2, cy * C:cy * C + C + 2, cx * C:cx * C + C + 2]
                a, b = float(blk.min()), float(blk.max())
                s = np.concatenate([[a, b], knots[(knots > a) & (knots < b)],
                                    np.linspace(a, b, 257)])
                assert maj[cz, cy, cx] == pytest.approx(ds * _alpha(med, s).max(), abs=1e-15)


def test_majorant_cell_ranges_and_threads_assemble_the_grid():
    # the cell-range entry point computes each cell by the same definition:
    # ragged ranges and the threaded split reassemble the whole grid bitwise
    v = _vol((21, 30, 37), 8, zero=0.4)
    buf, _ = oracle.encode(v, 0.5)
    f = oracle.VdbField(buf)
    med = dict(sigma_scale=20.0, tf=[(0, 0, 0, 0.1), (1, 1, 1, 0.9), (1, 1, 1, 0.4)])
    full = oracle.majorant(f, med, 4)
    part = np.full_like(full, -1.0)
    cuts = [0, 1, 17, 200, 201, full.size]
    for a, b in zip(cuts[:-1], cuts[1:]):
        oracle.majorant(f, med, 4, cells=(a, b), out=part)
    assert np.array_equal(part.view(np.uint64), full.view(np.uint64))
    assert np.array_equal(oracle.majorant_threads(f, med, 4, 3).view(np.uint64), full.view(np.uint64))


def test_majorant_bounds_every_sample():
    v = _vol((40, 33, 27), 2)
    buf, _ = oracle.encode(v, 0.3)
    f = oracle.VdbField(buf)
    med = dict(sigma_scale=7.0, **TF5)
    C = 8
    maj = oracle.majorant(f, med, C)
    rng = np.random.default_rng(3)
    p = (rng.random((50000, 3)) * [27, 33, 40] - 0.5).astype(np.float32)
    sig = 7.0 / 40 * _alpha(med, oracle.sample(f, p))
    cell = np.floor((p.astype(np.float64) + 0.5) / C).astype(int)
    assert np.all(sig <= maj[cell[:, 2], cell[:, 1], cell[:, 0]] * (1 + 1e-12))


# ------------------------------ emission-absorption ------------------------------

def test_ea_homogeneous_slab_closed_form():
    c = 0.6
    n = 32
    v = np.full((n, n, n), c, np.float32)
    buf, st = oracle.encode(v, 1.0)
    med = scenes.ea_medium(8.0)
    cam = scenes.ortho_z_camera(n, n, 16, 16)
    for step in (0.5, 0.25, 1.0):
        img = oracle.render_ea(oracle.VdbField(buf), cam, med, dict(step=step))
        sigma = 8.0 / n * float(np.float32(c))
        alpha = 1 - math.exp(-sigma * step)
        T = (1 - alpha) ** int(round(n / step))
        rgb = _rgb(med, float(np.float32(c)))
        np.testing.assert_allclose(img[..., 3], 1 - T, rtol=1e-12)
        for ch in range(3):
            np.testing.assert_allclose(img[..., ch], rgb[ch] * (1 - T), rtol=1e-12)
    # small steps approach Beer-Lambert exp(-sigma d)
    img = oracle.render_ea(oracle.VdbField(buf), cam, med, dict(step=1 / 64))
    assert img[0, 0, 3] == pytest.approx(1 - math.exp(-8.0 * float(np.float32(c))), rel=1e-9)


def test_ea_front_to_back_two_layers():
    n, m = 16, 6
    a, b = 0.9, 0.3
    v = np.full((n, n, n), b, np.float32)
    v[:m] = a          # front layer (small z) first along +z
    med = scenes.ea_medium(8.0)
    f = oracle.DenseField(v, 0.0)
    cam = scenes.ortho_z_camera(n, n, 4, 4)
    img = oracle.render_ea(f, cam, med, dict(step=1.0))  # samples on voxel centres
    sa, sb = 8.0 / n * float(np.float32(a)), 8.0 / n * float(np.float32(b))
    Ta, Tb = math.exp(-sa) ** m, math.exp(-sb) ** (n - m)
    ca, cb = _rgb(med, float(np.float32(a))), _rgb(med, float(np.float32(b)))
    want = ca * (1 - Ta) + Ta * cb * (1 - Tb)
    for ch in range(3):
        np.testing.assert_allclose(img[..., ch], want[ch], rtol=1e-12)
    np.testing.assert_allclose(img[..., 3], 1 - Ta * Tb, rtol=1e-12)


def test_ea_early_termination_threshold():
    v = np.full((32, 32, 32), 1.0, np.float32)
    f = oracle.DenseField(v, 1.0)
    med = scenes.ea_medium(80.0)
    cam = scenes.ortho_z_camera(32, 32, 4, 4)
    full = oracle.render_ea(f, cam, med, dict(step=0.5))
    cut = oracle.render_ea(f, cam, med, dict(step=0.5, t_terminate=1e-3))
    assert np.all(cut[..., 3] >= 1 - 1e-3)
    assert np.all(np.abs(cut - full) <= 1e-3 + 1e-12)


# ------------------------------ delta tracking ------------------------------

def _chord(n, o, d):
    # brute force: inside-length of the parametric line sampled finely
    t = np.linspace(0, 4 * n, 4_000_001)
    pts = np.asarray(o)[None, :] + t[:, None] * np.asarray(d)[None, :]
    inside = np.all((pts >= -0.5) & (pts <= n - 0.5), axis=1)
    return inside.sum() * (t[1] - t[0])


@pytest.mark.parametrize("C", [4, 8, 16])
def test_transmittance_homogeneous_beer_lambert(C):
    n = 24
    v = np.full((n, n, n), 1.0, np.float32)
    buf, _ = oracle.encode(v, 1.0)
    f = oracle.VdbField(buf)
    med = dict(sigma_scale=30.0, tf=[(1, 1, 1, 0), (1, 1, 1, 1)])
    d = np.array([1.0, 2.0, 3.0])
    d /= np.linalg.norm(d)
    o = np.array([3.3, -0.9, -5.0]) - 0.0
    o = o - 10 * d
    L = _chord(n, o, d)
    trials = 200_000
    T = oracle.transmittance(f, med, o, d, trials, seed=C, C_=C)
    want = math.exp(-30.0 / n * L)
    se = math.sqrt(want * (1 - want) / trials)
    assert abs(T - want) < 4 * se + 1e-4


@pytest.mark.parametrize("n,seed", [(6, 1), (8, 2)])
def test_transmittance_heterogeneous_matches_ray_marched(n, seed):
    v = _vol((n, n, n), seed, zero=0.3)
    f = oracle.DenseField(v, 0.0)
    med = dict(sigma_scale=3.0 * n, tf=[(1, 1, 1, 0), (1, 1, 1, 1)])
    rng = np.random.default_rng(seed)
    for ray in range(3):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        o = np.full(3, (n - 1) / 2.0) + rng.uniform(-1, 1, 3) - 2 * n * d
        o32, d32 = o.astype(np.float32), d.astype(np.float32)
        o64, d64 = o32.astype(np.float64), d32.astype(np.float64)
        d64 = d64 / np.linalg.norm(d64)
        # ray-marched optical depth, midpoint rule at 1/256 voxel
        dt = 1.0 / 256
        t = (np.arange(int(4 * n / dt)) + 0.5) * dt
        pts = o64[None] + t[:, None] * d64[None]
        inside = np.all((pts >= -0.5) & (pts <= n - 0.5), axis=1)
        s = ndimage.map_coordinates(v.astype(np.float64), pts[inside][:, ::-1].T, order=1,
                                    mode="grid-constant", cval=0.0)
        tau = (3.0 * n / n) * s.sum() * dt
        want = math.exp(-tau)
        trials = 200_000
        T = oracle.transmittance(f, med, o32, d32, trials, seed=seed * 10 + ray, C_=4)
        se = math.sqrt(max(want * (1 - want), 1e-6) / trials)
        assert abs(T - want) < 4 * se + 2e-3, (T, want)


# ------------------------------ path tracer ------------------------------

def test_isotropic_directions_uniform_on_sphere():
    # midpoint grid over the unit square -> quadrature of the sphere moments:
    # |d| = 1, E[d] = 0, E[d d^T] = I / 3, E[d_x^4] = 1 / 5
    m = 200
    u = (np.arange(m) + 0.5) / m
    D = np.array([oracle.isotropic(a, b) for a in u for b in u])
    np.testing.assert_allclose(np.linalg.norm(D, axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(D.mean(axis=0), 0.0, atol=1e-3)
    np.testing.assert_allclose(D.T @ D / len(D), np.eye(3) / 3, atol=1e-3)
    np.testing.assert_allclose((D ** 4).mean(axis=0), 0.2, atol=1e-3)


def _homog(n, value=1.0):
    v = np.full((n, n, n), value, np.float32)
    buf, _ = oracle.encode(v, 1.0)
    return oracle.VdbField(buf)


def test_pt_zero_density_is_ambient():
    n = 16
    f = oracle.DenseField(np.zeros((n, n, n), np.float32), 0.0)
    med = scenes.pt_medium(64.0)
    cam = scenes.orbit_camera((n, n, n), 8, 8)
    rgba, aov = oracle.render_pt(f, cam, med, dict(spp=4, max_bounces=4, seed=3), aov=True)
    assert np.all(rgba[:, :3] == np.asarray(med["ambient"], np.float32).astype(np.float64))
    assert np.all(rgba[:, 3] == 0) and np.all(aov == 1.0)


def test_pt_white_furnace():
    # albedo 1, white medium, no light, constant ambient: every path that
    # escapes carries exactly the ambient radiance
    n = 16
    f = _homog(n)
    med = dict(sigma_scale=40.0, albedo=1.0, tf=[(1, 1, 1, 0), (1, 1, 1, 1)],
               light_dir=(0, 1, 0), light_E=(0, 0, 0), ambient=(0.25, 0.5, 1.0))
    cam = scenes.orbit_camera((n, n, n), 8, 8)
    rgba = oracle.render_pt(f, cam, med, dict(spp=8, max_bounces=10_000, seed=4))
    np.testing.assert_allclose(rgba[:, :3], np.tile([0.25, 0.5, 1.0], (64, 1)), rtol=1e-12)


def test_pt_albedo_zero_is_attenuated_ambient():
    n, sigma_scale = 16, 24.0
    f = _homog(n)
    med = dict(sigma_scale=sigma_scale, albedo=0.0, tf=[(1, 1, 1, 0), (1, 1, 1, 1)],
               light_dir=(0, 0, -1), light_E=(5, 5, 5), ambient=(1.0, 1.0, 1.0))
    cam = scenes.ortho_z_camera(n, n, 16, 16)
    spp = 64
    rgba, aov = oracle.render_pt(f, cam, med, dict(spp=spp, max_bounces=4, seed=5), aov=True)
    tau = sigma_scale
    T = math.exp(-tau / n * n)
    N = 256 * spp
    se = math.sqrt(T * (1 - T) / N)
    assert abs(rgba[:, 0].mean() - T) < 4 * se
    assert abs(aov[:, 1].mean() - T) < 4 * se
    # mean first-scatter depth fraction: (1 - e^-tau) / tau
    dmean = (1 - math.exp(-tau)) / tau
    assert abs(aov[:, 0].mean() - dmean) < 4 * math.sqrt(1.0 / (12 * N)) + 4 * se


def test_pt_single_scatter_closed_form():
    # light from the camera side, one scattering event, no ambient:
    # E[L] = albedo * E / (4 pi) * (1 - exp(-2 sigma d)) / 2
    n, sigma_scale, albedo, E = 16, 12.0, 0.8, 2.0
    f = _homog(n)
    med = dict(sigma_scale=sigma_scale, albedo=albedo, tf=[(1, 1, 1, 0), (1, 1, 1, 1)],
               light_dir=(0, 0, -1), light_E=(E, E, E), ambient=(0, 0, 0))
    cam = scenes.ortho_z_camera(n, n, 16, 16)
    spp = 64
    rgba = oracle.render_pt(f, cam, med, dict(spp=spp, max_bounces=1, seed=6))
    sd = sigma_scale
    p = (1 - math.exp(-2 * sd)) / 2
    k = albedo * E / (4 * math.pi)
    N = 256 * spp
    se = k * math.sqrt(p * (1 - p) / N)
    assert abs(rgba[:, 1].mean() - k * p) < 4 * se


def _single_scatter_channels(med, s0, n, spp, seed):
    """Oracle image of a homogeneous cube of value s0 lit from the camera
    side with one scattering event, and the per-channel closed form
    E[L_ch] = albedo * c_ch(s0) * E_ch / (4 pi) * (1 - exp(-2 sigma d)) / 2,
    sigma d = sigma_scale * alpha(s0); colour and alpha by np.interp."""
    f = _homog(n, s0)
    cam = scenes.ortho_z_camera(n, n, 16, 16)
    rgba = oracle.render_pt(f, cam, med, dict(spp=spp, max_bounces=1, seed=seed))
    sd = float(np.float32(med["sigma_scale"])) * _alpha(med, float(np.float32(s0)))
    p = (1 - math.exp(-2 * sd)) / 2
    k = (float(np.float32(med["albedo"])) * _rgb(med, float(np.float32(s0))) *
         _f32(med["light_E"]) / (4 * math.pi))
    return rgba, k, p


def test_pt_single_scatter_coloured_closed_form():
    # a constant TF colour c and a coloured light: channel ch carries
    # albedo * c_ch * E_ch of the same single-scatter indicator, so the three
    # channels of every pixel are that indicator times their own constant and
    # their means follow the per-channel closed form (a swapped or dropped
    # colour channel, or alpha used as colour, fails)
    c = (0.9, 0.5, 0.2)
    med = dict(sigma_scale=12.0, albedo=0.8, tf=[c + (0.0,), c + (1.0,)],
               light_dir=(0, 0, -1), light_E=(2.0, 1.0, 3.0), ambient=(0, 0, 0))
    n, spp = 16, 64
    rgba, k, p = _single_scatter_channels(med, 1.0, n, spp, 6)
    ind = rgba[:, 0] / k[0]
    for ch in range(3):
        np.testing.assert_allclose(rgba[:, ch] / k[ch], ind, rtol=1e-12, atol=1e-15)
        se = k[ch] * math.sqrt(p * (1 - p) / (256 * spp))
        assert abs(rgba[:, ch].mean() - k[ch] * p) < 4 * se, ch
    assert np.all(rgba[:, :3] >= 0) and ind.max() > 0.5


@pytest.mark.parametrize("s0", [0.15, 0.45, 0.62, 0.85])
def test_pt_single_scatter_five_point_tf_at_density(s0):
    # TF5: five coloured control points with alpha 0, .8, .3, 1, .5 over
    # [0.1, 0.9]; a homogeneous cube of value s0 in each interval: extinction
    # from the interpolated alpha, throughput from the interpolated colour
    med = dict(TF5, sigma_scale=12.0, albedo=0.9, light_dir=(0, 0, -1),
               light_E=(1.5, 2.5, 1.0), ambient=(0, 0, 0))
    n, spp = 16, 64
    rgba, k, p = _single_scatter_channels(med, s0, n, spp, 60 + int(100 * s0))
    ind = rgba[:, 1] / k[1]
    for ch in range(3):
        if k[ch] == 0.0:
            assert np.all(rgba[:, ch] == 0.0)
            continue
        np.testing.assert_allclose(rgba[:, ch] / k[ch], ind, rtol=1e-12, atol=1e-15)
        se = k[ch] * math.sqrt(p * (1 - p) / (256 * spp))
        assert abs(rgba[:, ch].mean() - k[ch] * p) < 4 * se, (ch, rgba[:, ch].mean(), k[ch] * p)


def _numpy_homog_pt(n, sigma, albedo, E, ldir, amb, bounces, N, seed):
    """Independent analytic estimator for a homogeneous cube: exponential
    free flights, exact shadow transmittance, isotropic scattering."""
    rng = np.random.default_rng(seed)
    o = np.stack([rng.uniform(-0.5, n - 0.5, N), rng.uniform(-0.5, n - 0.5, N),
                  np.full(N, -0.5)], 1)
    d = np.tile([0.0, 0.0, 1.0], (N, 1))
    L = np.zeros(N)
    beta = np.ones(N)
    alive = np.ones(N, bool)
    ldir = np.asarray(ldir, np.float64)

    def exit_dist(p, dd):
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = np.where(dd > 0, (n - 0.5 - p) / dd, np.where(dd < 0, (-0.5 - p) / dd, np.inf))
        return t1.min(axis=1)

    for b in range(bounces):
        te = exit_dist(o, d)
        t = -np.log(1 - rng.random(N)) / sigma
        esc = alive & (t >= te)
        L[esc] += beta[esc] * amb
        alive &= ~esc
        x = o + t[:, None] * d
        beta = beta * albedo
        tl = exit_dist(x, np.tile(ldir, (N, 1)))
        L[alive] += beta[alive] * E / (4 * math.pi) * np.exp(-sigma * tl[alive])
        if b + 1 == bounces:
            break
        z = 1 - 2 * rng.random(N)
        phi = 2 * math.pi * rng.random(N)
        r = np.sqrt(np.maximum(0, 1 - z * z))
        d = np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)
        o = x
    return L


def test_pt_multiple_scattering_matches_analytic_estimator():
    n, sigma_scale, albedo = 16, 32.0, 0.9
    E, amb, bounces = 3.0, 0.1, 8
    ldir = np.array([-0.4, 0.8, 0.45])
    ldir /= np.linalg.norm(ldir)
    f = _homog(n)
    med = dict(sigma_scale=sigma_scale, albedo=albedo, tf=[(1, 1, 1, 0), (1, 1, 1, 1)],
               light_dir=tuple(ldir), light_E=(E, E, E), ambient=(amb, amb, amb))
    cam = scenes.ortho_z_camera(n, n, 16, 16)
    spp = 256
    L1 = oracle.render_pt(f, cam, med, dict(spp=spp, max_bounces=bounces, seed=7))[:, 0]
    L2 = oracle.render_pt(f, cam, med, dict(spp=spp, max_bounces=bounces, seed=8))[:, 0]
    Lo = 0.5 * (L1 + L2)
    # Monte Carlo noise of the mean from two independent renders
    se_o = math.sqrt(np.var(L1 - L2) / 4 / len(Lo))
    ld32 = np.asarray(ldir, np.float32).astype(np.float64)
    Ln = _numpy_homog_pt(n, sigma_scale / n, albedo, E, ld32, amb, bounces, 1_000_000, 8)
    se = math.sqrt(se_o ** 2 + Ln.var() / len(Ln))
    assert abs(Lo.mean() - Ln.mean()) < 4 * se, (Lo.mean(), Ln.mean(), se)
    # multiple scattering matters at this albedo: single scattering differs
    S = _numpy_homog_pt(n, sigma_scale / n, albedo, E, ld32, amb, 1, 400_000, 9)
    assert abs(S.mean() - Ln.mean()) > 10 * se


def test_pt_multiple_scattering_coloured_matches_analytic_estimator():
    # a constant TF colour scales each channel's throughput by albedo * c_ch
    # at every real collision: channel ch must match the analytic estimator
    # run with albedo * c_ch, E_ch and ambient_ch
    n, sigma_scale, albedo, bounces = 16, 32.0, 0.9, 8
    c = np.array([1.0, 0.7, 0.35])
    E = np.array([3.0, 2.0, 4.0])
    amb = np.array([0.1, 0.3, 0.05])
    ldir = np.array([-0.4, 0.8, 0.45])
    ldir /= np.linalg.norm(ldir)
    f = _homog(n)
    med = dict(sigma_scale=sigma_scale, albedo=albedo, tf=[tuple(c) + (0.0,), tuple(c) + (1.0,)],
               light_dir=tuple(ldir), light_E=tuple(E), ambient=tuple(amb))
    cam = scenes.ortho_z_camera(n, n, 16, 16)
    spp = 256
    L1 = oracle.render_pt(f, cam, med, dict(spp=spp, max_bounces=bounces, seed=17))[:, :3]
    L2 = oracle.render_pt(f, cam, med, dict(spp=spp, max_bounces=bounces, seed=18))[:, :3]
    ld32 = np.asarray(ldir, np.float32).astype(np.float64)
    c32, E32, a32 = _f32(c), _f32(E), _f32(amb)
    means = []
    for ch in range(3):
        Lo = 0.5 * (L1[:, ch] + L2[:, ch])
        se_o = math.sqrt(np.var(L1[:, ch] - L2[:, ch]) / 4 / len(Lo))
        Ln = _numpy_homog_pt(n, sigma_scale / n, float(np.float32(albedo)) * c32[ch], E32[ch], ld32,
                             a32[ch], bounces, 400_000, 30 + ch)
        se = math.sqrt(se_o ** 2 + Ln.var() / len(Ln))
        assert abs(Lo.mean() - Ln.mean()) < 4 * se, (ch, Lo.mean(), Ln.mean(), se)
        means.append(Ln.mean())
    # the channels differ by far more than the noise: the colour matters
    assert abs(means[0] - means[2]) > 0.05


def _texel_of(d, w, h):
    u = (np.arctan2(d[..., 2], d[..., 0]) + math.pi) / (2 * math.pi)
    v = np.arccos(np.clip(d[..., 1], -1, 1)) / math.pi
    return (np.clip(np.floor(v * h), 0, h - 1).astype(int),
            np.clip(np.floor(u * w), 0, w - 1).astype(int))


def pinhole_texel_cases():
    """A pinhole camera looking through an empty volume at a lat-long map
    with distinguishable texels, and for every pixel the texel its rays see
    (or -1 where the pixel's footprint straddles two texels): directions of
    17 x 17 points spanning each pixel square widened by 10 % on every side,
    from the camera's definition (lower_left + x du + y dv, normalised), in
    float64."""
    n = 8
    w, h = 32, 16
    env = np.zeros((h, w, 3), np.float32)
    for y in range(h):
        for x in range(w):
            env[y, x] = (x, y, 100 + x + w * y)
    # off-centre, non-square, tilted view so that a du/dv swap or a missing
    # normalisation moves pixels to other texels
    cam = scenes.pinhole_camera((3.5, 2.0, -30.0), (9.0, 8.5, 3.5), (0.2, 1.0, 0.1), 60.0, 40, 26)
    ll, du, dv = (np.asarray(cam[k], np.float32).astype(np.float64) for k in ("lower_left", "du", "dv"))
    sub = np.linspace(-0.1, 1.1, 17)   # the pixel square and a 10 % margin
    want = np.full((cam["height"], cam["width"]), -1, np.int64)
    for py in range(cam["height"]):
        for px in range(cam["width"]):
            x = px + sub[:, None]
            y = py + sub[None, :]
            d = ll + x[..., None] * du + y[..., None] * dv
            d /= np.linalg.norm(d, axis=-1, keepdims=True)
            ty, tx = _texel_of(d, w, h)
            if np.all(ty == ty.flat[0]) and np.all(tx == tx.flat[0]):
                want[py, px] = ty.flat[0] * w + tx.flat[0]
    return n, env, cam, want


def test_pt_pinhole_camera_rays_see_their_texels():
    # the pinhole camera's ray directions, pinned through the image-based
    # light: every escaping camera ray returns the texel of its own direction
    n, env, cam, want = pinhole_texel_cases()
    f = oracle.DenseField(np.zeros((n, n, n), np.float32), 0.0)
    med = dict(scenes.pt_medium(16.0), env=env)
    rgba = oracle.render_pt(f, cam, med, dict(spp=5, max_bounces=2, seed=2))
    ok = want >= 0
    assert ok.sum() >= 0.4 * ok.size and len(np.unique(want[ok])) >= 8
    flat = env.reshape(-1, 3).astype(np.float64)
    got = rgba[:, :3].reshape(cam["height"], cam["width"], 3)
    assert np.array_equal(got[ok], flat[want[ok]])


def test_pt_deterministic_per_pixel():
    # a pixel's estimate depends only on (seed, pixel, sample), not on which
    # other pixels are rendered in the same call
    n = 16
    v = _vol((n, n, n), 12, zero=0.4)
    buf, _ = oracle.encode(v, 0.5)
    f = oracle.VdbField(buf)
    med = scenes.pt_medium(32.0)
    cam = scenes.orbit_camera((n, n, n), 12, 10)
    prm = dict(spp=3, max_bounces=5, seed=99)
    full = oracle.render_pt(f, cam, med, prm)
    sub = oracle.render_pt(f, cam, med, prm, pixels=np.array([119, 5, 60], np.uint32))
    assert np.array_equal(sub, full[[119, 5, 60]])


def test_pt_with_a_given_majorant_equals_the_built_one():
    # the entry point that takes a precomputed majorant walks the same grid
    n = 16
    v = _vol((n, n, n), 13, zero=0.4)
    buf, _ = oracle.encode(v, 0.5)
    f = oracle.VdbField(buf)
    med = scenes.pt_medium_tf5(32.0)
    cam = scenes.orbit_camera((n, n, n), 12, 10)
    prm = dict(spp=3, max_bounces=5, seed=99, macrocell=4)
    a, aa = oracle.render_pt(f, cam, med, prm, aov=True)
    maj = oracle.majorant(f, med, 4)
    b, ba = oracle.render_pt(f, cam, med, prm, aov=True, majorant=maj)
    assert np.array_equal(a, b) and np.array_equal(aa, ba)
    with pytest.raises(ValueError):
        oracle.render_pt(f, cam, med, dict(prm, macrocell=8), majorant=maj)


def test_pt_russian_roulette_is_unbiased():
    # a thick white medium lit only by ambient: deep paths carry most of the
    # radiance, so roulette from bounce 2 on (survival max(beta), survivors
    # divided by it) must keep the mean of the plain estimator; dropping the
    # division or the survival test moves it by far more than the noise
    n, sigma_scale, albedo, amb, bounces = 16, 96.0, 0.8, 1.0, 48
    f = _homog(n)
    med = dict(sigma_scale=sigma_scale, albedo=albedo, tf=[(1, 1, 1, 0), (1, 1, 1, 1)],
               light_dir=(0, 1, 0), light_E=(0, 0, 0), ambient=(amb, amb, amb))
    cam = scenes.ortho_z_camera(n, n, 16, 16)
    spp = 256
    runs = [oracle.render_pt(f, cam, med, dict(spp=spp, max_bounces=bounces, seed=s, rr=True))[:, 0]
            for s in (11, 12)]
    Lo = 0.5 * (runs[0] + runs[1])
    se_o = math.sqrt(np.var(runs[0] - runs[1]) / 4 / len(Lo))
    Ln = _numpy_homog_pt(n, sigma_scale / n, albedo, 0.0, (0.0, 1.0, 0.0), amb, bounces, 600_000, 12)
    se = math.sqrt(se_o ** 2 + Ln.var() / len(Ln))
    assert abs(Lo.mean() - Ln.mean()) < 4 * se, (Lo.mean(), Ln.mean(), se)
    # the roulette changes the draws: the image differs from the plain one
    plain = oracle.render_pt(f, cam, med, dict(spp=spp, max_bounces=bounces, seed=11))[:, 0]
    assert not np.array_equal(plain, runs[0])
    # deep paths matter here: cutting them at 2 bounces loses far more than the noise
    S = _numpy_homog_pt(n, sigma_scale / n, albedo, 0.0, (0.0, 1.0, 0.0), amb, 2, 300_000, 13)
    assert Ln.mean() - S.mean() > 20 * se


def test_pt_russian_roulette_white_furnace_never_kills():
    # albedo 1 and a white medium keep beta = 1, so the survival probability
    # is 1 and every path still returns exactly the ambient radiance
    n = 16
    f = _homog(n)
    med = dict(sigma_scale=40.0, albedo=1.0, tf=[(1, 1, 1, 0), (1, 1, 1, 1)],
               light_dir=(0, 1, 0), light_E=(0, 0, 0), ambient=(0.25, 0.5, 1.0))
    cam = scenes.orbit_camera((n, n, n), 8, 8)
    rgba = oracle.render_pt(f, cam, med, dict(spp=8, max_bounces=10_000, seed=4, rr=True))
    np.testing.assert_allclose(rgba[:, :3], np.tile([0.25, 0.5, 1.0], (64, 1)), rtol=1e-12)


def _env_unique(w=8, h=4):
    # texel (y, x) carries (x, y, 100 + x + w y): every texel is distinguishable
    e = np.zeros((h, w, 3), np.float32)
    for y in range(h):
        for x in range(w):
            e[y, x] = (x, y, 100 + x + w * y)
    return e


@pytest.mark.parametrize("direction,texel", [((1, 0, 0), (4, 2)), ((-1, 0, 0), (7, 2)),
                                             ((0, 1, 0), (4, 0)), ((0, -1, 0), (4, 3)),
                                             ((0, 0, 1), (6, 2)), ((0, 0, -1), (2, 2))])
def test_pt_env_map_axis_directions(direction, texel):
    # empty volume: every camera ray escapes along the camera direction, so
    # the pixel is the texel the lat-long mapping assigns to that axis:
    # u = (atan2(z, x) + pi) / 2pi, v = acos(y) / pi, nearest texel, clamped
    n = 8
    f = oracle.DenseField(np.zeros((n, n, n), np.float32), 0.0)
    env = _env_unique()
    med = dict(scenes.pt_medium(16.0), env=env)
    d = np.asarray(direction, np.float64)
    a = np.roll(d, 1)                       # two axes orthogonal to d
    b = np.cross(d, a)
    cam = dict(kind=0, width=4, height=4, lower_left=tuple(-20.0 * d - a - b),
               du=tuple(0.5 * a), dv=tuple(0.5 * b), dir=tuple(d))
    rgba = oracle.render_pt(f, cam, med, dict(spp=3, max_bounces=2, seed=1))
    want = env[texel[1], texel[0]].astype(np.float64)
    assert np.array_equal(rgba[:, :3], np.tile(want, (16, 1)))


def test_pt_constant_env_map_equals_ambient():
    # a constant map is the ambient term: same draws, same sums, bit for bit
    n = 16
    v = _vol((n, n, n), 21, zero=0.3)
    buf, _ = oracle.encode(v, 0.5)
    f = oracle.VdbField(buf)
    med = scenes.pt_medium(48.0)
    env = np.broadcast_to(np.asarray(med["ambient"], np.float32), (6, 12, 3)).copy()
    cam = scenes.orbit_camera((n, n, n), 10, 9)
    prm = dict(spp=4, max_bounces=6, seed=17)
    a = oracle.render_pt(f, cam, med, prm)
    b = oracle.render_pt(f, cam, dict(med, env=env), prm)
    assert np.array_equal(a, b)
    # a brighter map adds exactly (escaped throughput) x 1 per channel: no
    # pixel loses light and pixels whose camera rays all escape gain 1
    c = oracle.render_pt(f, cam, dict(med, env=env + 1.0), prm)
    assert np.all(c[:, :3] >= a[:, :3]) and np.any(c[:, :3] > a[:, :3])
    clear = a[:, 3] == 0.0
    assert clear.any()
    np.testing.assert_allclose(c[clear, :3] - a[clear, :3], 1.0, rtol=1e-6)
