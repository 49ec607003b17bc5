"""Writes the stored oracle results used by the full-size GPU parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generator; nothing
here touches the GPU library.  Inputs are rounded to FP32 as the GPU receives
them.  Outputs (the oracle's Z and rho_e after 50 outer iterations):
  slice512_K50.npz  sinogram form, 512^2 / 720-view / 736-bin slice
                    (elliptical water body, 40 inserts, Poisson 5e4 / 1e5)
  image512_K50.npz  image-domain form (--image), the same phantom as noisy
                    attenuation images (15 / 10 HU white noise)

    python tests/golden/make_golden.py [--threads N] [--image]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import solve as S  # noqa: E402
from oracle.physics import Physics  # noqa: E402
from paper_2308_01290_amd import phantoms as P  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--image", action="store_true")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    phys = Physics()
    if args.image:
        return image(args, phys)
    args.out = args.out or os.path.join(HERE, "slice512_K50.npz")
    g, ph, pL, pH = P.workload_slice512(phys.mu_pair)
    pL = pL.astype(np.float32).astype(np.float64)
    pH = pH.astype(np.float32).astype(np.float64)
    params = S.Params(n_iter=50)
    t0 = time.time()
    Z, R, st = S.solve(pL, pH, g, phys, params, nthreads=args.threads or None, return_state=True)
    dt = time.time() - t0
    np.savez_compressed(args.out, Z=Z.astype(np.float32), rho=R.astype(np.float32),
                        seconds=np.float64(dt), n_iter=np.int32(50))
    print(f"wrote {args.out} in {dt:.1f} s")


def image(args, phys):
    from oracle import image as I
    out = args.out or os.path.join(HERE, "image512_K50.npz")
    g, ph, muL, muH = P.workload_image512(phys.mu_pair)
    muL = muL.astype(np.float32).astype(np.float64)
    muH = muH.astype(np.float32).astype(np.float64)
    t0 = time.time()
    Z, R = I.solve(muL, muH, phys, S.Params(n_iter=50))
    dt = time.time() - t0
    np.savez_compressed(out, Z=Z.astype(np.float32), rho=R.astype(np.float32),
                        seconds=np.float64(dt), n_iter=np.int32(50))
    print(f"wrote {out} in {dt:.1f} s")


if __name__ == "__main__":
    main()
