"""Writes the stored oracle results used by the full-size GPU parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generator; nothing
here touches the GPU library.  Inputs are rounded to FP32 as the GPU receives
them.  Each file holds the oracle's Z and rho_e (FP32) after the stated number
of outer iterations and the seconds the oracle took.

  slice512   slice512_K50.npz   sinogram form, 512^2 / 720-view / 736-bin slice
                                (elliptical water body, 40 inserts, Poisson 5e4 / 1e5), K = 50
  image512   image512_K50.npz   image-domain form, the same phantom as noisy
                                attenuation images (15 / 10 HU white noise), K = 50
  uneven     uneven_<seed>_K50.npz  four slices of the uneven batch (image 256,
                                384, 384, 512; 984, 360, 720, 984 views; 882, 535,
                                864, 829 bins), K = 50
  served     served_<n>_<views>_K20.npz  two serving requests: 768^2 with 1152
                                views and 256^2 with 360 views, K = 20 (the low end
                                of the requests' iteration budgets)

    python tests/golden/make_golden.py MODE [MODE ...] [--threads N]
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

UNEVEN_SEEDS = (3038, 3002, 3030, 3016)
SERVED = ((768, 12680, 1152), (256, 7560, 360))   # (image n, seed, views)
SERVED_K = 20


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


OUT_DIR = [HERE]


def save(name, Z, R, dt, n_iter, **meta):
    out = os.path.join(OUT_DIR[0], name)
    np.savez_compressed(out, Z=Z.astype(np.float32), rho=R.astype(np.float32),
                        seconds=np.float64(dt), n_iter=np.int32(n_iter), **meta)
    print(f"wrote {out} in {dt:.1f} s", flush=True)


def sino_case(name, g, pL, pH, n_iter, threads, phys, **meta):
    """The oracle's solve (init, n_iter iterations, output), one progress line
    per iteration."""
    t0 = time.time()
    a, b = f32(pL), f32(pH)
    params = S.Params(n_iter=n_iter).resolved(phys, g)
    st = S.init_state(a, b, g, phys, params, threads or None)
    for k in range(n_iter):
        st = S.iterate(st, a, b, g, phys, params, threads or None)
        print(f"{name}: iteration {k + 1}/{n_iter} ({time.time() - t0:.0f} s)", flush=True)
    Z, R = S.finalize(st, phys, params)
    save(name, Z, R, time.time() - t0, n_iter, **meta)


def slice512(args, phys):
    g, ph, pL, pH = P.workload_slice512(phys.mu_pair)
    sino_case("slice512_K50.npz", g, pL, pH, 50, args.threads, phys)


def image512(args, phys):
    from oracle import image as I
    g, ph, muL, muH = P.workload_image512(phys.mu_pair)
    t0 = time.time()
    Z, R = I.solve(f32(muL), f32(muH), phys, S.Params(n_iter=50))
    save("image512_K50.npz", Z, R, time.time() - t0, 50)


def uneven(args, phys):
    for seed in UNEVEN_SEEDS:
        g, ph, pL, pH = P.slice_uneven(seed, phys.mu_pair)
        sino_case(f"uneven_{seed}_K50.npz", g, pL, pH, 50, args.threads, phys, seed=np.int32(seed))


def served_one(args, phys, n, seed, views):
    g, ph, pL, pH = P.slice_served(n, seed, phys.mu_pair, n_views=views)
    sino_case(f"served_{n}_{views}_K{SERVED_K}.npz", g, pL, pH, SERVED_K, args.threads, phys,
              seed=np.int32(seed))


def served(args, phys):
    for n, seed, views in SERVED:
        served_one(args, phys, n, seed, views)


def uneven_one(args, phys, seed):
    g, ph, pL, pH = P.slice_uneven(seed, phys.mu_pair)
    sino_case(f"uneven_{seed}_K50.npz", g, pL, pH, 50, args.threads, phys, seed=np.int32(seed))


MODES = {"slice512": slice512, "image512": image512, "uneven": uneven, "served": served}
MODES.update({f"uneven{seed}": (lambda a, p, s=seed: uneven_one(a, p, s)) for seed in UNEVEN_SEEDS})
MODES.update({f"served{n}": (lambda a, p, c=(n, seed, v): served_one(a, p, *c)) for n, seed, v in SERVED})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("modes", nargs="+", choices=sorted(MODES))
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out-dir", default=HERE, help="where the .npz files go")
    args = ap.parse_args()
    OUT_DIR[0] = args.out_dir
    os.makedirs(args.out_dir, exist_ok=True)
    phys = Physics()
    for m in args.modes:
        MODES[m](args, phys)


if __name__ == "__main__":
    main()
