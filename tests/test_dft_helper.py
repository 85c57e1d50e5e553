"""Pin of the closed-form QFT helper against numpy's inverse FFT."""
import math

import numpy as np

from circuits import random_state
from tests.dft_closed_form import qft_output


def test_matches_scaled_ifft():
    for n in (1, 5, 12):
        psi = random_state(n, seed=n, workload=9)
        want = np.fft.ifft(psi) * math.sqrt(1 << n)
        for y in sorted({0, 1, (1 << n) - 1, (1 << n) // 3}):
            assert abs(qft_output(psi, y) - want[y]) < 1e-13
