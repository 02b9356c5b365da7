"""Writes precision_ref_channel_64.npz: the FP64 oracle's u and Pi^neq at
steps 10, 100 and 2000 of the 64^3 laminar channel subcase of the precision
workload, at a seeded sample of 2048 fluid nodes (the whole field at 2000
steps is too slow for the oracle inside a test and too large to store).

Subcase: 64^3 nodes, x and z periodic, half-way walls on y = 0 and 63,
tau = 0.5045 (binary32-rounded), body force 2 nu U_c / h^2 along x with
U_c = 0.05 and h = 31, initial parabolic profile plus seeded +-5 %
perturbations, rounded to binary32 (the state the GPU starts from).

Run from the repository root: python tests/golden/make_precision_ref.py
(2000 oracle steps of 2.6e5 nodes; about a quarter of an hour on 8 cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

HORIZONS = (10, 100, 2000)
SAMPLES, SAMPLE_SEED = 2048, 606
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_ref_channel_64.npz")


def main():
    case = W.precision_subcase()
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    G = oracle.make_grid(case.nx, case.ny, case.nz, f32(case.tau), faces=case.faces,
                         force=[f32(v) for v in case.force])
    kinds = oracle.node_kinds(G)
    idx = W.sample_nodes(case, SAMPLES, SAMPLE_SEED, fluid_mask=(kinds == 0))
    st = W.to_fp32(W.channel_state(case))
    out = {"idx": idx, "horizons": np.array(HORIZONS)}
    done = 0
    for t in HORIZONS:
        t0 = time.time()
        st = oracle.run(G, st, t - done, t0=done)
        done = t
        out["moments_%d" % t] = st.reshape(10, -1)[:, idx]
        print("step %d (%.0f s)" % (t, time.time() - t0), flush=True)
    np.savez(OUT, **out)


if __name__ == "__main__":
    main()
