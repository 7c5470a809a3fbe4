"""Host-side logic of the warm start (no device): the series ratio that decides the
order of the lattice-wave start."""
import numpy as np


def test_series_ratio_of_known_amplitudes():
    from paper_2212_07494_amd import warmstart as W
    n = 4
    amp = np.zeros((n + n * (n + 1) + 48, 27), complex)
    amp[:n] = 1e-3                       # a1 = sqrt(4 * 27) 1e-3
    amp[n:n + 20] = 1e-5j                # a2 = sqrt(20 * 27) 1e-5
    amp[n + 20:] = -1e-7                 # a3 = sqrt(48 * 27) 1e-7
    a1, a2, a3 = np.sqrt(108) * 1e-3, np.sqrt(540) * 1e-5, np.sqrt(1296) * 1e-7
    assert np.isclose(W.series_ratio(n, amp), a3 * a3 / (a2 * a1), rtol=1e-12)
    # no second order (a single mode without self-interaction) -> 0, never a division by 0
    assert W.series_ratio(n, np.zeros_like(amp)) == 0.0
