"""Writes the exact density profiles of the two-phase shock tube (the
1D workload and its planar 2048-cell form) at t = 240 us, used as the
reference of the L1 errors that bench.py reports.

Calls only the oracle's exact stiffened-gas Riemann solver (oracle/
exact_riemann.py, Toro ch. 4 with p -> p + p_inf); run from the repository
root:  python tests/golden/make_exact_profiles.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import exact_riemann as ER  # noqa: E402

# the shock tube of the workloads: liquid (gamma 4.4, p_inf 6e8, rho 1000,
# p 1e9) | air (gamma 1.4, rho 50, p 1e5) at x = 0.7 on [0, 1], at rest
LEFT = dict(rho=1000.0, u=0.0, p=1e9, gamma=4.4, pinf=6e8)
RIGHT = dict(rho=50.0, u=0.0, p=1e5, gamma=1.4, pinf=0.0)
T_END = 240e-6


def main():
    for n in (400, 2048):
        x = (np.arange(n) + 0.5) / n
        rho, _, _ = ER.solve(x, T_END, 0.7, LEFT, RIGHT)
        path = os.path.join(HERE, f"exact_rho_shock_tube_{n}.txt")
        with open(path, "w") as f:
            f.write(f"# exact density (kg/m^3) at t = 240 us, cell centres (i + 1/2)/{n} on [0, 1]; "
                    f"written by make_exact_profiles.py (oracle/exact_riemann.py)\n")
            for v in rho:
                f.write("%.17g\n" % v)
        print(path)


if __name__ == "__main__":
    main()
