"""Writes vortex80k_t2_oracle.txt: the FP64 oracle's state of the configured
isentropic-vortex case (200 x 200 split/jittered periodic [0,10]^2, seed 2,
cubic CTENOZ, lambda1' = 1e4, SSP-RK3 at CFL 0.3) at t = 2, on 400 sampled
cells.  Calls the oracle and the input generators only.

    python tests/golden/make_vortex80k_t2.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2312_17042_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "vortex80k_t2_oracle.txt")


def main():
    mesh, u0 = W.vortex_case(200, seed=2)
    o = O.Oracle.from_mesh(mesh, physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4)
    t0 = time.time()
    u, steps, t = o.solve(u0, 2.0, cfl=0.3)
    cells = np.sort(np.random.default_rng(7).choice(mesh.n_cells, 400, replace=False))
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle, isentropic vortex 200x200 seed 2, cubic CTENOZ lambda1'=1e4, CFL 0.3\n")
        fh.write(f"# written by tests/golden/make_vortex80k_t2.py; steps {steps} t {t!r} "
                 f"({time.time() - t0:.0f} s, {O.threads()} threads)\n")
        fh.write("# cell rho rho_u rho_v E\n")
        fh.write(f"steps {steps}\n")
        for c in cells:
            fh.write(f"{c} " + " ".join(repr(float(x)) for x in u[:, c]) + "\n")
    print("wrote", OUT, steps, "steps")


if __name__ == "__main__":
    main()
