"""The allocation-free gradient-L0 step (dect_l0_step_static) against the
allocating entry point (dect_l0_step with unit weight), through the C-ABI."""
import numpy as np
import pytest

from paper_2308_01290_amd import dect
from tests.gpu_util import cuda, host

pytestmark = pytest.mark.gpu


def inputs(batch, ny, nx, seed):
    rng = np.random.default_rng(seed)
    clean = np.zeros((batch, ny, nx))
    clean[:, :, nx // 3: 2 * nx // 3] = 1.0
    gt = (clean + 0.05 * rng.standard_normal(clean.shape)).astype(np.float32)
    g0 = (clean + 0.02 * rng.standard_normal(clean.shape)).astype(np.float32)
    return gt, g0


def run_both(batch, ny, nx, beta, seed):
    import torch
    gt, g0 = inputs(batch, ny, nx, seed)
    lam = 0.01
    a = cuda(g0)
    ha, va = torch.empty_like(a), torch.empty_like(a)
    dect.l0_step_static(cuda(gt), a, lam, beta, h=ha, v=va)
    b, hb, vb = dect.l0_step(cuda(gt), cuda(g0), lam, beta, return_hv=True)
    return [host(x) for x in (a, ha, va)], [host(x) for x in (b, hb, vb)]


def test_static_equals_allocating_two_calls():
    """Two calls in a row on the shared static scratch, the second smaller:
    each equals the allocating entry point's output bit for bit (same kernels
    and order), including the thresholded (h, v)."""
    for batch, ny, nx, beta, seed in ((4, 512, 512, 0.05, 1), (1, 96, 64, 40.0, 2)):
        got, ref = run_both(batch, ny, nx, beta, seed)
        for g_, r_ in zip(got, ref):
            assert np.array_equal(g_, r_), (batch, ny, nx)


def test_static_rejects_sizes_beyond_its_scratch():
    """batch*n_y*n_x above the static scratch fails on the host, before
    anything is enqueued, and leaves g untouched."""
    import torch
    cap = int(dect.lib().dect_l0_step_static_max_values())
    assert cap == 1 << 21
    n = 1024
    batch = cap // (n * n) + 1
    g = torch.zeros((batch, n, n), device="cuda")
    with pytest.raises(dect.DectError, match="static scratch"):
        dect.l0_step_static(torch.ones_like(g), g, 0.01, 1.0)
    assert float(g.abs().max()) == 0.0
    # empty batch is a no-op
    e = torch.zeros((0, 64, 64), device="cuda")
    dect.l0_step_static(e, e, 0.01, 1.0)
