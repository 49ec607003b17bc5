"""Writes the stored oracle results used by the full-size GPU parity test.

Calls only the FP64 oracle (oracle/) and the seeded input generator; nothing
here touches the GPU library.  Output: tests/golden/slice512_K50.npz with the
oracle's Z and rho_e after 50 outer iterations on the 512^2 / 720-view /
736-bin slice (elliptical water body, 40 inserts, Poisson 5e4 / 1e5), inputs
rounded to FP32 as the GPU receives them.

    python tests/golden/make_golden.py [--threads N]
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
    ap.add_argument("--out", default=os.path.join(HERE, "slice512_K50.npz"))
    args = ap.parse_args()
    phys = Physics()
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


if __name__ == "__main__":
    main()
