"""Write tests/golden/thermal12_v48_nh4_harmonics.txt: the oracle's converged
harmonics (Eq. 40) of rho, U, V and T for the heated cavity of the mixed-form
benchmark shape on a grid the oracle converges in minutes.

Case: 12 x 12 cells, 48 x 48 velocities on [-5, 5], N_H = 4 (nine levels),
Shakhov (Pr = 2/3), Kn = 1, St = 1, bottom wall T = T0 (1 + 0.5 sin wt), other
walls at T0, default numerics (CFL 0.5, min face step, level-mass projection),
from rest to R_rho <= 1e-11.  (Stopping at the usual 1e-8 leaves this case about
3e-5 of its density signal away from the fixed point, more than the mixed
form's 1e-5 bound; at 1e-11 the stored state is within 1e-7 of it.)

The values come from the oracle alone (this script imports nothing but the
oracle and the case definitions).  Run: python tests/golden/make_thermal12.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import hbcases  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "thermal12_v48_nh4_harmonics.txt")


def case():
    return hbcases.Case(12, 12, 48, 5.0, 1.0, 1.0, 4, hbcases.thermal_walls(0.5, 0, "sin"), name="thermal12_v48_nh4")


def main():
    c = case()
    o = oracle.Oracle(c)
    t0 = time.time()
    k = 0
    while True:
        o.step(200)
        k += 200
        r = o.residual()
        if k % 2000 == 0:
            print(f"step {k}: R_rho {r[0]:.3e} ({time.time() - t0:.0f} s)", flush=True)
        if r[0] <= 1e-11:
            break
        if k >= 60000:
            raise RuntimeError(f"no convergence: R = {r}")
    re, im = o.harmonics()
    rows = []
    for v in range(4):
        for kk in range(c.NH + 1):
            rows.append(re[v, kk])
            rows.append(im[v, kk])
    header = (f"Oracle harmonics (Eq. 40) of rho, U, V, T/T0 for {c.name}: {c.nx} x {c.ny} cells, "
              f"{c.M}^2 velocities on [-{c.umax:g}, {c.umax:g}], N_H = {c.NH}, Kn = {c.Kn:g}, St = {c.St:g}, "
              f"Pr = 2/3, bottom wall T0 (1 + 0.5 sin wt).\n"
              f"Converged from rest by the oracle in {k} pseudo steps to R = {r.tolist()}; written by "
              f"tests/golden/make_thermal12.py.\n"
              f"Rows: for var in (rho, U, V, T), for k in 0..N_H: Re then Im of qhat_k over the {c.nc} cells "
              f"(c = j nx + i).")
    np.savetxt(OUT, np.array(rows), fmt="%.17e", header=header)
    print(f"wrote {OUT} after {k} steps, R = {r}")


if __name__ == "__main__":
    main()
