"""Writes the FP64 oracle's time averages that the mixed-precision path is
compared with (statistically, over independent seeds):

- f1_oracle_shock_density.txt: density of the 1D Ma 3 shock averaged over
  the 30 snapshots at steps 550, 600, ..., 2000, one row per seed;
- f1_oracle_cylinder_wall.txt: the coarse Ma 15 cylinder (40 x 30 O-grid,
  N_ref 50, Shakhov Pr 2/3) after 1500 steps, one row per seed: C_d, then the
  cumulative-average C_p, C_F and C_Q of the 40 wall faces (Sec. V.A).

Seeds 101..106; calls only the oracle.  Run from the repository root:
    python tests/golden/make_f1_oracle.py
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

SEEDS = list(range(101, 107))
HERE = os.path.dirname(os.path.abspath(__file__))


def shock_mean_density(seed):
    import oracle
    import workloads as wl
    w = wl.shock1d()
    w["seed"] = seed
    o = oracle.Oracle(w)
    o.step(500)
    acc = np.zeros(w["n_cells"])
    for _ in range(30):
        o.step(50)
        acc += o.fields()[:, 0]
    return acc / 30


def cylinder_wall(seed):
    import oracle
    import workloads as wl
    w = wl.cylinder(n_theta=40, n_r=30, n_ref=50, Pr=2.0 / 3.0, seed=seed)
    o = oracle.Oracle(w)
    o.step(1500)
    surf, cd = o.surface(1)
    return np.concatenate([[cd], surf[:, 3].ravel(), surf[:, 4].ravel(), surf[:, 5].ravel()])


def main():
    import oracle
    oracle.build()
    with ProcessPoolExecutor(max_workers=6) as ex:
        shock = np.array(list(ex.map(shock_mean_density, SEEDS)))
        cyl = np.array(list(ex.map(cylinder_wall, SEEDS)))
    hdr = "seeds " + " ".join(map(str, SEEDS))
    np.savetxt(os.path.join(HERE, "f1_oracle_shock_density.txt"), shock, fmt="%.17g",
               header=hdr + "; density averaged over steps 550..2000 (every 50), one row per seed")
    np.savetxt(os.path.join(HERE, "f1_oracle_cylinder_wall.txt"), cyl, fmt="%.17g",
               header=hdr + "; after 1500 steps: C_d, C_p[40], C_F[40], C_Q[40], one row per seed")


if __name__ == "__main__":
    main()
