"""Error of computed macroscopic harmonics against expected ones, as the
mixed-form tolerance reads it: the relative L-infinity norm over the stacked
vector of the nondimensional harmonics of rho, U, V and T (Eq. 40), that is
max |computed - expected| over every variable, level and cell, divided by the
largest harmonic signal (the expected harmonics minus the rest state rho = 1,
U = V = 0, T = 1).  Each variable's error against its own signal is returned
too, for reporting: a variable with a small signal (the thermal-creep velocity
of a heated cavity) sees the rounding of the others' deviations magnified."""
import numpy as np


def macro_errors(hg, ho):
    """hg, ho: complex arrays [4][N_H + 1][cells] (rho, U, V, T).  Returns
    (stacked relative error, list of per-variable relative errors)."""
    dev = np.array(ho, dtype=np.complex128)
    dev[0, 0] -= 1.0
    dev[3, 0] -= 1.0
    diff = np.abs(np.asarray(hg) - np.asarray(ho))
    per = [float(np.max(diff[v]) / np.max(np.abs(dev[v]))) for v in range(4)]
    return float(np.max(diff) / np.max(np.abs(dev))), per
