"""Shared helpers of the GPU tests (inputs are seeded; nothing here computes
the method)."""
import functools

import numpy as np

from paper_2308_01290_amd import phantoms as P


def cuda(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel_inf(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def ragged_geometry():
    """Non-square image, bins not a multiple of 256, offset detector, odd views."""
    return P.FanGeometry(n_x=40, n_y=24, pixel_mm=1.3, n_views=37, n_det=300, sid_mm=400.0,
                         sdd_mm=700.0, det_offset_mm=0.37, angle0_rad=0.3).resolved()


@functools.lru_cache(maxsize=None)
def workload(name):
    """(geometry, phantom, p_lo, p_hi) with FP32-rounded sinograms."""
    from oracle.physics import Physics
    phys = Physics()
    if name == "small":
        g, ph, pL, pH = P.workload_small(phys.mu_pair)
    elif name == "slice512":
        g, ph, pL, pH = P.workload_slice512(phys.mu_pair)
    else:
        raise KeyError(name)
    return g, ph, pL.astype(np.float32), pH.astype(np.float32)
