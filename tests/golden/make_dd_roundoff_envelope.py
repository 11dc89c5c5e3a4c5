"""Write dd2d_roundoff_envelope.txt: how far the oracle's own trajectory of
the 200k-cell drift-diffusion workload moves when its initial densities are
perturbed at the level of rounding (relative 1e-15, four seeds), per
checkpoint of 100 steps up to 1000.

The limited Lax-Wendroff flux switches its limiter off when the jump b across
an edge changes sign (Sec. "Limited Lax-Wendroff scheme"), and its time-step
term does not vanish with b, so the face value jumps there: a rounding
difference can move a node across the switch and the trajectory then
departs by more than rounding.  The envelope measures that sensitivity with
the oracle alone; the GPU trajectory test bounds its difference from the
oracle by it.

    python tests/golden/make_dd_roundoff_envelope.py     (about 2 minutes)
"""
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

import numpy as np  # noqa: E402

SEEDS = (1, 2, 3, 4)
MAG = 1e-15
CHECKS = 10
EVERY = 100
OUT = os.path.join(HERE, "dd2d_roundoff_envelope.txt")


def _trajectory(seed):
    import cases
    import oracle
    from paper_2201_01291_amd import workloads as wl
    m = wl.dd_streamer_mesh()
    n, E = wl.dd_fields(m)
    case = cases.Case("dd2d", m, n, E, dict(cases.DD2))
    if seed >= 0:
        n = n * (1.0 + MAG * np.random.default_rng(seed).standard_normal(n.shape))
    om = oracle.OracleMesh(m)
    ph = case.oracle_phys()
    U, t, out = n.copy(), 0.0, []
    for _ in range(CHECKS):
        U, t, _, _ = om.step(ph, U, E, nsteps=EVERY, t0=t)
        out.append(U.copy())
    return out


def main():
    import cases
    from paper_2201_01291_amd import workloads as wl
    with Pool(len(SEEDS) + 1) as pool:
        runs = pool.map(_trajectory, (-1,) + SEEDS)
    m = wl.dd_streamer_mesh()
    n, E = wl.dd_fields(m)
    case = cases.Case("dd2d", m, n, E, dict(cases.DD2))
    base = runs[0]
    with open(OUT, "w") as fh:
        fh.write("# oracle trajectory of the 200k-cell drift-diffusion workload (LLW-minmod,\n"
                 "# RK1, CFL 0.5): largest norm-wise state difference, over seeds 1-4, between\n"
                 "# the run from the seeded densities and runs from densities perturbed by a\n"
                 "# relative 1e-15 N(0,1); written by make_dd_roundoff_envelope.py\n"
                 "# step  envelope\n")
        for k in range(CHECKS):
            env = max(cases.state_err(case, r[k], base[k]).max() for r in runs[1:])
            fh.write(f"{EVERY * (k + 1)} {env:.3e}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
