"""Writes rollout_fd_forced_periodic_64.json: FP64 central differences of the
differentiable workload's objective, computed with the oracle alone.

Workload: 64^3 periodic box, tau = 0.8 (binary32-rounded, as the library
receives it), body-force field g ~ N(0, (1e-6)^2) per component, initial
velocity u0 = Taylor-Green (0.01) + N(0, (1e-3)^2), rho = 1, Pi^neq = 0,
400 steps; loss L = 1/2 sum rho |u|^2 at the final level (FP64).  The
inputs are rounded to binary32 first, so the derivatives are taken at the
point the GPU rollout starts from.

For each of two seeded standard-normal directions d of g and two of u0 the
file holds (L(theta + s d) - L(theta - s d)) / (2 s), with the step
s = h * rms(theta) and h = 1e-4 (a relative perturbation of 1e-4).

Run from the repository root: python tests/golden/make_rollout_fd.py
(nine 400-step oracle runs of 2.6e5 nodes; about half an hour on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

H = 1e-4
DIRECTION_SEED = 4242
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rollout_fd_forced_periodic_64.json")


def main():
    case = W.adjoint_case()
    st0, g = W.adjoint_inputs(case)
    st0 = W.to_fp32(st0)
    g = g.astype(np.float32).astype(np.float64)
    tau = float(np.float32(case.tau))
    G = oracle.make_grid(case.nx, case.ny, case.nz, tau)

    def loss(st, gg):
        t0 = time.time()
        fin = oracle.run(G, st, case.steps, gg)
        sums, bad = oracle.reduce(G, fin)
        assert bad == 0
        print("  loss %.17g (%.0f s)" % (sums[4], time.time() - t0), flush=True)
        return float(sums[4])

    rms = lambda a: float(np.sqrt((a * a).mean()))  # noqa: E731
    sg, su = H * rms(g), H * rms(st0[1:4])
    dgs, dus = W.gradient_directions(case, DIRECTION_SEED)
    rec = {"workload": case.name, "steps": case.steps, "tau": tau, "h": H, "direction_seed": DIRECTION_SEED,
           "step_g": sg, "step_u0": su, "threads": oracle.num_threads()}
    print("L at the base point", flush=True)
    rec["loss"] = loss(st0, g)
    rec["fd_g"], rec["fd_u0"] = [], []
    for k, d in enumerate(dgs):
        print("direction g%d" % k, flush=True)
        lp, lm = loss(st0, g + sg * d), loss(st0, g - sg * d)
        rec["fd_g"].append((lp - lm) / (2.0 * sg))
    for k, d in enumerate(dus):
        print("direction u0_%d" % k, flush=True)
        sp, sm = st0.copy(), st0.copy()
        sp[1:4] += su * d
        sm[1:4] -= su * d
        lp, lm = loss(sp, g), loss(sm, g)
        rec["fd_u0"].append((lp - lm) / (2.0 * su))
    json.dump(rec, open(OUT, "w"), indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
