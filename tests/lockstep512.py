"""Lockstep of the 512^2 / 720-view / 736-bin slice over all 50 outer
iterations: the FP64 oracle runs its own trajectory on the host, and from each
of its states (rounded to FP32) the GPU runs one outer iteration; per
iteration the script prints the near-tie counts of eq. (9) and the GPU's
deviation from the oracle's next state (f, rho_e relative to their sup-norm;
t' on the eroded body relative to max(1, sup)).  A study, not a test (about
8 minutes on 16 host cores): the oracle's trajectory is too long for the test
suite, whose lockstep tests cover the first iteration at 512^2.

    python -u -m tests.lockstep512 [--iters 50]
"""
import argparse
import sys
import time

import numpy as np

from oracle import solve as S
from oracle.physics import Physics
from paper_2308_01290_amd import dect
from tests import e2e
from tests import ht_flips as HF
from tests.gpu_util import cuda, host, workload


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=50)
    args = ap.parse_args()
    g, ph, pL, pH = workload("slice512")
    phys = Physics()
    params = S.Params(n_iter=50).resolved(phys, g)
    _, body = e2e.body_mask(ph, g)
    a, b = f32(pL), f32(pH)
    lo, hi = cuda(pL[None]), cuda(pH[None])
    st = S.init_state(a, b, g, phys, params)
    worst = {"f": 0.0, "rho": 0.0, "t": 0.0}
    t0 = time.time()
    print("k  near-ties(f1,f2,rho,t)  df/sup  drho/sup  dt'(body)/max(1,sup)", flush=True)
    for k in range(args.iters):
        s32 = S.State(f32(st.f1), f32(st.f2), f32(st.rho), f32(st.t), st.beta, k)
        ref = S.iterate(s32, a, b, g, phys, params)
        sol = dect.Solver(g, dect.default_params(n_iter=50)).set_state(
            lo, hi, *(cuda(x[None]) for x in (s32.f1, s32.f2, s32.rho, s32.t)), k=k)
        sol.iterate(1)
        f1, f2, rho, t = (host(x)[0] for x in sol.state())
        sol.close()
        ties = [int(HF.near_ties(getattr(s32, n), params.lam, s32.beta).sum()) for n in ("f1", "f2", "rho", "t")]
        df = max(float(np.abs(f1 - ref.f1).max() / np.abs(ref.f1).max()),
                 float(np.abs(f2 - ref.f2).max() / np.abs(ref.f2).max()))
        dr = float(np.abs(rho - ref.rho).max() / np.abs(ref.rho).max())
        dt = float(np.abs(t - ref.t)[body].max() / max(1.0, np.abs(ref.t[body]).max()))
        worst = {"f": max(worst["f"], df), "rho": max(worst["rho"], dr), "t": max(worst["t"], dt)}
        print(f"{k:2d} {ties} {df:.2e} {dr:.2e} {dt:.2e}  beta={s32.beta:.3g} ({time.time() - t0:.0f} s)",
              flush=True)
        st = ref
    print(f"worst over {args.iters} iterations: f {worst['f']:.2e}, rho_e {worst['rho']:.2e}, "
          f"t' {worst['t']:.2e}", flush=True)
    ok = worst["f"] <= 1e-5 and worst["rho"] <= 1e-5 and worst["t"] <= 5e-4
    print("within the lockstep tolerances (1e-5, 1e-5, 5e-4):", ok, flush=True)
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
