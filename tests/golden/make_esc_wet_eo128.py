"""Writes esc_wet_eo128_sample1500.txt: the oracle's wet step (midpoint scheme of eq step1
and eq step2 with the stochastic stress and the random finite difference of eq
thermforce) of the 128^3 electro-osmosis channel with 262,144 ions, the ESC pair of
App. B (cations w = 7, beta = 7; anions w = 4, beta = 8) as hydrodynamic kernels, at
1,500 ions sampled with a fixed seed.  The inputs are the seeded synthetic workload;
the values come from oracle/ alone (about four minutes on one core).

    python -m tests.golden.make_esc_wet_eo128
"""
import os

import numpy as np

from oracle import dynamics, electrostatics as es
import workloads

WORKLOAD = "eo_stokes_128x128x128_n262144"
KERNELS = [(7, 7.0), (4, 8.0)]
STEP = 0
SAMPLE, SAMPLE_SEED = 1500, 23
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "esc_wet_eo128_sample1500.txt")


def case():
    """(workload, params, ions, sampled indices, rfd delta) shared with the GPU test."""
    w = workloads.WORKLOADS[WORKLOAD]
    p = workloads.make_params(w)
    p["hydro_kernel"] = np.asarray(KERNELS, dtype=np.float64)
    delta = 1e-4 * w.h
    p["rfd_delta"] = delta
    ions = workloads.make_ions(w)
    targets = np.sort(np.random.default_rng(SAMPLE_SEED).choice(w.n, SAMPLE, replace=False))
    return w, p, ions, targets, delta


def main():
    w, p, (pos, q, ids, species), targets, delta = case()
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    ref, _, _ = dynamics.wet_step(grid, pos, q, species, ids, p, STEP, rfd_delta=delta,
                                  near="pairs", targets=targets)
    with open(OUT, "w") as f:
        f.write(f"# oracle wet step + RFD, {WORKLOAD}, ESC pair {KERNELS}, step {STEP}, "
                f"rfd_delta {delta!r}, {SAMPLE} ions sampled with seed {SAMPLE_SEED}\n")
        f.write("# id x y z (new positions)\n")
        for t, k in enumerate(targets):
            x, y, z = (float(v) for v in ref[:, t])
            f.write(f"{int(ids[k])} {x!r} {y!r} {z!r}\n")


if __name__ == "__main__":
    main()
