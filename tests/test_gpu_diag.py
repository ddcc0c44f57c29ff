"""The atomic-layout microbenchmark (mpm_diag_box_atomics), measurement
support (GPU): one launch of each layout on a zeroed grid leaves the expected
sums, each node holding the number of workgroup boxes that cover it (both
atomic layouts), 1 where covered (plain stores), nothing (empty launch); the
box geometry is recomputed here from its description; bad arguments are
refused."""
import numpy as np
import pytest
import torch

from paper_1910_00935_amd import _lib as L

pytestmark = pytest.mark.gpu


def _coverage(n):
    cov = np.zeros((n, n, n), np.int64)
    for w in range(128):
        bx, by, bz = w & 3, (w >> 2) & 3, w >> 4
        x0, y0, z0 = 15 + 4 * bx, 15 + 4 * by, 15 + 2 * bz
        cov[x0:x0 + 7, y0:y0 + 7, z0:z0 + 5] += 1
    return cov


@pytest.mark.parametrize("layout", [0, 1, 2, 3])
def test_box_sums(layout):
    n = 40
    g = torch.zeros(4 * n ** 3, device="cuda")
    L.call("mpm_diag_box_atomics", layout, g.data_ptr(), n, 1, torch.cuda.current_stream().cuda_stream)
    got = g.cpu().numpy().reshape(n, n, n, 4)
    cov = _coverage(n)
    want = {0: cov, 1: cov, 2: (cov > 0).astype(np.int64), 3: np.zeros_like(cov)}[layout]
    for c in range(4):
        assert np.array_equal(got[..., c], want.astype(np.float32)), (layout, c)
    if layout in (0, 1):
        assert cov.max() == 12 and cov.sum() == 128 * 245  # up to 2 x 2 x 3 boxes per node


def test_refusals():
    g = torch.zeros(4 * 40 ** 3, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    for layout, n, k in ((4, 40, 1), (1, 33, 1), (1, 40, -1)):
        assert L.lib().mpm_diag_box_atomics(layout, g.data_ptr(), n, k, s) == L.MPM_E_ARG
    assert L.lib().mpm_diag_box_atomics(1, None, 40, 1, s) == L.MPM_E_ARG
