"""Host check of the mixed-form harmonic error measure (tests/harmerr.py):
the stacked relative L-infinity error over rho, U, V, T harmonics, with the
rest state (rho = 1, U = V = 0, T = 1 at k = 0) taken out of the signal."""
import numpy as np

from harmerr import macro_errors


def test_stacked_and_per_variable_errors():
    ncell, nk = 5, 3
    ho = np.zeros((4, nk, ncell), dtype=complex)
    ho[0, 0] = 1.0 + 0.02  # density 1.02: signal 0.02
    ho[1, 1] = 1e-4j       # small velocity signal
    ho[2, 2] = 5e-3
    ho[3, 0] = 1.0 - 0.1   # temperature signal 0.1 (the largest)
    hg = ho.copy()
    hg[1, 1, 2] += 2e-9    # 2e-9 on a 1e-4 signal: 2e-5 of U, 2e-8 of the stacked signal
    hg[3, 0, 4] -= 3e-8    # 3e-8 on the 0.1 signal
    err, per = macro_errors(hg, ho)
    assert np.isclose(err, 3e-8 / 0.1)
    assert np.isclose(per[1], 2e-9 / 1e-4)
    assert np.isclose(per[3], 3e-8 / 0.1)
    assert per[0] == 0.0 and per[2] == 0.0


def test_rest_state_is_not_signal():
    ho = np.zeros((4, 2, 3), dtype=complex)
    ho[0, 0] = 1.0
    ho[3, 0] = 1.0
    ho[0, 1, 0] = 1e-3
    hg = ho + 1e-9
    err, _ = macro_errors(hg, ho)
    assert np.isclose(err, 1e-9 / 1e-3)
