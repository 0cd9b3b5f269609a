"""Write c2_mean_energies_1000.txt: the FP64 oracle's 1000-step mean energies
of the 1M-bead A20B20 melt, as an ensemble mean and spread.

python tests/golden/make_mean_energies.py      (about 6 minutes on 8 cores)

The oracle integrates the seeded workload for 1000 velocity Verlet steps
(Integration methods section; forces of eq. 6 and eq. 7) and records KE,
E_bond, W and E_tot at every step; a run's "mean energy" is the mean over
steps 1..1000. The trajectory is chaotic, so the means of runs that differ
by one rounding are themselves spread: the ensemble is the unperturbed run
plus 7 runs whose initial coordinates are scaled by (1 + 1e-7 g), g standard
normal (seeds 11..17), about one FP32 rounding. The file holds, per energy,
the ensemble mean and standard deviation of the 8 means, the unperturbed
run's mean and the energy at step 0. Only oracle/ and the seeded generators
are called.
"""
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

STEPS = 1000
EPS = 1e-7
SEEDS = [None, 11, 12, 13, 14, 15, 16, 17]
OUT = os.path.join(HERE, "c2_mean_energies_1000.txt")


def trajectory(seed):
    import oracle
    from synth import workloads as wl
    s = wl.build(wl.SPECS["c2"])
    R = s.R.copy()
    if seed is not None:
        rng = np.random.default_rng(seed)
        xyz = R[:, :3].astype(np.float64) * (1.0 + EPS * rng.standard_normal((s.N, 3)))
        R[:, :3] = xyz.astype(np.float32)
    _, _, E = oracle.run(s, STEPS, R=R)
    return E


def main():
    with mp.Pool(len(SEEDS)) as pool:
        runs = pool.map(trajectory, SEEDS)
    means = np.array([E[1:].mean(0) for E in runs])
    ens, sd = means.mean(0), means.std(0, ddof=1)
    names = ["KE", "E_bond", "W", "E_tot"]
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, 1M-bead A20B20 melt (seeded), velocity Verlet, %d steps\n" % STEPS)
        f.write("# written by tests/golden/make_mean_energies.py; a run's mean is over steps 1..%d\n"
                % STEPS)
        f.write("# ensemble: the unperturbed run + %d runs with coordinates scaled by (1 + %.0e g)\n"
                % (len(SEEDS) - 1, EPS))
        f.write("# name  ensemble_mean  ensemble_sd  unperturbed_mean  energy_at_step_0\n")
        for i, n in enumerate(names):
            f.write("%s %.17g %.6g %.17g %.17g\n" % (n, ens[i], sd[i], means[0, i], runs[0][0, i]))
    print(open(OUT).read())


if __name__ == "__main__":
    main()
