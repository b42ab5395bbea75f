"""Writes rarefaction_4000_t0p6.npz: the oracle's run of the N = 4000 double
rarefaction (Example 3.8's configuration at h = 2/4000, transmissive, to
t = 0.6, CFL rule with w1 = 1/12), and as the yardstick of a GPU comparison
the relative L1 distance per component between that run and the same run
from initial data perturbed by 1e-15 relative.  Calls only the oracle;
takes about two minutes on one core."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    n = 4000
    h = 2.0 / n
    U0 = W.double_rarefaction_1d(n)
    U, info = oracle.run_1d(U0, (1, 1), h, 0.6)
    rng = np.random.default_rng(1402)
    Up, infop = oracle.run_1d(U0 * (1.0 + 1e-15 * rng.standard_normal(U0.shape)), (1, 1), h, 0.6)
    spread = np.array([np.abs(U[k] - Up[k]).sum() / np.abs(U[k]).sum() for k in range(3)])
    np.savez_compressed(os.path.join(HERE, "rarefaction_4000_t0p6.npz"), U=U, spread=spread,
                        t=info["t"], steps=info["steps"], min_rho=info["min_rho"],
                        min_p=info["min_p"], steps_perturbed=infop["steps"])
    print(info, infop)


if __name__ == "__main__":
    main()
