"""Pins of the oracle's iso-surface marcher (reading of the interval-based
implicit iso-surface ray marcher, Section 5.4).  A linear field is
reproduced exactly by trilinear interpolation, so planes give closed forms:
the hit lies on the plane to within the bisection width step / 2^refine, the
normal is minus the normalised gradient exactly, and with no refinement the
hit is the midpoint of the first lattice interval that crosses."""
import math

import numpy as np
import pytest

import oracle
from synth import scenes

NX, NY, NZ = 20, 18, 40


def _field(fn):
    z, y, x = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
    return np.ascontiguousarray(fn(x.astype(np.float64), y.astype(np.float64),
                                   z.astype(np.float64)).astype(np.float32))


def _interior(cam):
    """Pixel-centre masks whose footprint (and normal stencil) stays inside."""
    w, h = cam["width"], cam["height"]
    xs = -0.5 + (np.arange(w) + 0.5) * NX / w
    ys = -0.5 + (np.arange(h) + 0.5) * NY / h
    mx = (xs >= 0.5) & (xs <= NX - 1.5)
    my = (ys >= 0.5) & (ys <= NY - 1.5)
    return np.outer(my, mx), xs, ys


def _render(v, iso=0.5, step=0.37, refine=12, background=0.0):
    cam = scenes.ortho_z_camera(NX, NY, 2 * NX, 2 * NY)
    img, aux = oracle.render_iso(oracle.DenseField(v, background), cam, iso, step, refine, aux=True)
    return cam, img, aux


def test_ramp_plane_hit_position_and_normal():
    v = _field(lambda x, y, z: z / (NZ - 1))
    step, refine = 0.37, 12
    cam, img, aux = _render(v, step=step, refine=refine)
    m, _, _ = _interior(cam)
    t_star = 0.5 * (NZ - 1) + 0.5          # z = -0.5 + t on the plane z = (NZ-1)/2
    assert np.all(img[m][:, 3] == 1.0)
    assert np.max(np.abs(aux[m][:, 0] - t_star)) <= step / 2 ** refine + 1e-12
    # gradient +z: normal -z, colour 0.5 (n + 1) = (0.5, 0.5, 0)
    assert np.allclose(img[m][:, :3], [0.5, 0.5, 0.0], atol=1e-12)


def test_tilted_plane_normal_and_hit():
    a, b, c = 0.3, -0.2, 1.0
    v = _field(lambda x, y, z: (a * x + b * y + c * z) / NZ)
    step, refine = 0.5, 14
    cam, img, aux = _render(v, iso=0.45, step=step, refine=refine)
    m, xs, ys = _interior(cam)
    X, Y = np.meshgrid(xs, ys)
    t_star = (0.45 * NZ - a * X - b * Y) / c + 0.5
    hit = m & (t_star > 1.0) & (t_star < NZ - 1.0)
    assert hit.sum() > 100
    assert np.all(img[hit][:, 3] == 1.0)
    assert np.max(np.abs(aux[hit][:, 0] - t_star[hit])) <= step / 2 ** refine + 1e-9
    n = -np.array([a, b, c]) / math.sqrt(a * a + b * b + c * c)
    assert np.allclose(img[hit][:, :3], 0.5 * (n + 1.0), atol=1e-9)


def test_entering_inside_crosses_outward():
    v = _field(lambda x, y, z: 1.0 - z / (NZ - 1))
    cam, img, aux = _render(v)
    m, _, _ = _interior(cam)
    assert np.allclose(aux[m][:, 0], 0.5 * (NZ - 1) + 0.5, atol=0.37 / 2 ** 12 + 1e-12)
    assert np.allclose(img[m][:, :3], [0.5, 0.5, 1.0], atol=1e-12)   # normal +z


def test_first_crossing_of_a_tent_is_the_near_one():
    cz, w = NZ / 2.0, NZ / 3.0
    v = _field(lambda x, y, z: np.maximum(1.0 - np.abs(z - cz) / w, 0.0))
    cam, img, aux = _render(v)
    m, _, _ = _interior(cam)
    near = cz - 0.5 * w + 0.5
    assert np.max(np.abs(aux[m][:, 0] - near)) <= 0.37 / 2 ** 12 + 1e-12
    assert np.allclose(img[m][:, :3], [0.5, 0.5, 0.0], atol=1e-12)


def test_without_refinement_the_hit_is_the_interval_midpoint():
    v = _field(lambda x, y, z: z / (NZ - 1))
    step = 0.37
    cam, img, aux = _render(v, step=step, refine=0)
    m, _, _ = _interior(cam)
    t_star = 0.5 * (NZ - 1) + 0.5
    k = math.ceil(t_star / step - 0.5)        # first lattice sample past the plane
    assert np.allclose(aux[m][:, 0], step * k, atol=1e-12)   # ((k-1/2) + (k+1/2)) step / 2


@pytest.mark.parametrize("value", [0.3, 0.5, 0.9])
def test_constant_volume_never_crosses(value):
    # background = the value: the field is constant everywhere, so no pair of
    # samples straddles the iso value (f == iso counts as inside)
    v = np.full((NZ, NY, NX), value, np.float32)
    _, img, aux = _render(v, background=value)
    assert np.all(img == 0.0) and np.all(aux[..., 0] == -1.0)
    assert np.all(aux[..., 1] == abs(np.float32(value) - 0.5))
