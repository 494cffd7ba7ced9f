"""Scene descriptions (cameras, media, render settings) as plain numbers.

These are inputs shared by the oracle tests, the GPU tests and the benchmark:
dictionaries of floats and ints, no rendering arithmetic.  Cameras are in the
volume's index space, where voxel centres sit on integers and the volume fills
the box [-0.5, n-0.5]^3.
"""
from __future__ import annotations

import math

import numpy as np


def ortho_z_camera(nx: int, ny: int, width: int, height: int) -> dict:
    """Orthographic camera looking along +z; pixel (px, py) centre maps to
    x = -0.5 + (px + 0.5) * nx / width (y likewise), rays start on z = -0.5."""
    return dict(kind=0, width=width, height=height,
                lower_left=(-0.5, -0.5, -0.5),
                du=(nx / width, 0.0, 0.0), dv=(0.0, ny / height, 0.0),
                dir=(0.0, 0.0, 1.0))


def pinhole_camera(eye, target, up, fov_y_deg: float, width: int, height: int) -> dict:
    """Pinhole camera: ray direction of image point (x, y) in pixel units is
    lower_left + x * du + y * dv (then normalised)."""
    eye = np.asarray(eye, np.float64)
    w = np.asarray(target, np.float64) - eye
    w /= np.linalg.norm(w)
    u = np.cross(w, np.asarray(up, np.float64))
    u /= np.linalg.norm(u)
    v = np.cross(u, w)
    h = math.tan(math.radians(fov_y_deg) / 2.0)
    aspect = width / height
    du = u * (2.0 * h * aspect / width)
    dv = v * (2.0 * h / height)
    ll = w - u * (h * aspect) - v * h
    return dict(kind=1, width=width, height=height, origin=tuple(eye),
                lower_left=tuple(ll), du=tuple(du), dv=tuple(dv))


def orbit_camera(dims, width: int, height: int, fov_y_deg: float = 40.0,
                 azimuth_deg: float = 30.0, elevation_deg: float = 20.0,
                 distance: float = 1.9) -> dict:
    """Pinhole camera orbiting the volume centre at `distance` x the longest
    side."""
    nx, ny, nz = dims
    c = np.array([(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
    r = distance * max(dims)
    az, el = math.radians(azimuth_deg), math.radians(elevation_deg)
    eye = c + r * np.array([math.sin(az) * math.cos(el), math.sin(el),
                            -math.cos(az) * math.cos(el)])
    return pinhole_camera(eye, c, (0.0, 1.0, 0.0), fov_y_deg, width, height)


def ea_medium(sigma_scale: float = 8.0) -> dict:
    """Emission-absorption medium: extinction sigma_scale * density per unit
    of the longest axis; colour ramps linearly from (0.1, 0.2, 0.8) at
    density 0 to (1.0, 0.9, 0.6) at density 1."""
    return dict(sigma_scale=sigma_scale, albedo=1.0,
                tf=[(0.1, 0.2, 0.8, 0.0), (1.0, 0.9, 0.6, 1.0)], tf_range=(0.0, 1.0))


def pt_medium(sigma_scale: float = 64.0, albedo: float = 0.9) -> dict:
    """Scattering medium: white transfer function with alpha = density,
    one directional light and a constant ambient term."""
    d = np.array([-0.4, 0.8, 0.45])
    d /= np.linalg.norm(d)
    return dict(sigma_scale=sigma_scale, albedo=albedo,
                tf=[(1.0, 1.0, 1.0, 0.0), (1.0, 1.0, 1.0, 1.0)], tf_range=(0.0, 1.0),
                light_dir=tuple(d), light_E=(3.0, 3.0, 3.0),
                ambient=(0.06, 0.07, 0.10))


# Five coloured control points over densities [0.1, 0.9] with alpha
# 0, 0.8, 0.3, 1, 0.5: every interval of the transfer function has its own
# colour and slope, so a wrong interval, channel or colour shows.
TF5 = [(0.2, 0.3, 0.9, 0.0), (0.9, 0.1, 0.2, 0.8), (0.4, 0.4, 0.4, 0.3),
       (1.0, 1.0, 0.0, 1.0), (0.0, 1.0, 1.0, 0.5)]
TF5_RANGE = (0.1, 0.9)


def pt_medium_tf5(sigma_scale: float = 64.0, albedo: float = 0.9) -> dict:
    """The scattering medium of pt_medium() with the coloured five-point
    transfer function TF5 (alpha = extinction, RGB = scattering colour)."""
    return dict(pt_medium(sigma_scale, albedo), tf=list(TF5), tf_range=TF5_RANGE)


TINY = dict(name="tiny-64^3-ea-128x128", rate=0.25, width=128, height=128, step=0.5)
MID = dict(name="mid-512^3-pt-1024x1024x16spp", rates=(0.25, 0.10, 0.05), width=1024,
           height=1024, spp=16, max_bounces=8, seed=0x5EED)
PAPER = dict(name="paper-1987x1351x2449-pt-1920x1080x64spp",
             dims=(1987, 1351, 2449), rates=(0.05, 0.10, 0.15, 0.20, 0.25),
             width=1920, height=1080, spp=64, max_bounces=16, seed=0x5EED)
