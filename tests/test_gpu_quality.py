"""GPU parity of the compression-error statistics (Section 5.2's MSE and
PSNR): vdbc_compare_dense against the oracle's reconstruction of the same
grid and numpy sums.  Differing-voxel counts, max error and value range are
exact; the sum of squared errors agrees to 1e-12 relative (fp64 sums in
another order)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2504_04564_amd import _build, vdbc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def lib():
    _build.ensure_built()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return vdbc.load()


def _expected(v, q, metric=2):
    rec = oracle.reconstruct(v, q, metric)
    e = rec.astype(np.float64) - v.astype(np.float64)
    return dict(sse=float(np.sum(e * e)), max_abs=float(np.max(np.abs(e))),
                differing=int(np.count_nonzero(rec.view(np.uint32) != v.view(np.uint32))),
                min=float(v.min()), max=float(v.max()))


CASES = [((37, 29, 45), 0.25, 2, "cloud"), ((64, 64, 64), 0.10, 1, "cloud"),
         ((40, 33, 19), 0.5, 3, "noise"), ((48, 48, 48), 1.0, 2, "cloud"), ((8, 8, 8), 0.05, 2, "cloud")]


@pytest.mark.parametrize("shape,q,metric,kind", CASES)
def test_compare_dense_vs_oracle(shape, q, metric, kind):
    v = synth.cloud_volume(shape, seed=sum(shape)) if kind == "cloud" else \
        synth.dense_noise(shape, seed=sum(shape))
    buf, _ = vdbc.encode(v, q, metric=metric)
    got = vdbc.compare_dense(vdbc.Grid(buf), torch.from_numpy(v).cuda())
    want = _expected(v, q, metric)
    assert got["differing"] == want["differing"]
    assert got["max_abs"] == want["max_abs"]
    assert got["min"] == want["min"] and got["max"] == want["max"]
    assert abs(got["sse"] - want["sse"]) <= 1e-12 * max(want["sse"], 1e-300)
    if q == 1.0:
        assert got["differing"] == 0 and got["mse"] == 0.0 and got["psnr"] == float("inf")


def test_compare_dense_is_deterministic_and_counts_every_voxel():
    v = synth.dense_noise((70, 9, 130), seed=4)
    g = vdbc.Grid(vdbc.encode(v, 0.3)[0])
    d = torch.from_numpy(v).cuda()
    a = vdbc.compare_dense(g, d)
    b = vdbc.compare_dense(g, d)
    assert a == b
    # a grid compared with a volume shifted by one everywhere differs at
    # every voxel by exactly one
    c = vdbc.compare_dense(vdbc.Grid(vdbc.encode(v, 1.0)[0]), d + 1.0)
    assert c["differing"] == v.size
    assert abs(c["sse"] - v.size * 1.0) <= 1e-9 * v.size
