"""Closed form of the QFT used at sizes the oracle cannot replay in full.

With qubit q = index bit q, the QFT circuit maps psi to
  out[y] = 2^(-n/2) sum_x exp(+2 pi i x y / 2^n) psi[x].
The phase factorises over the bits of x, exp(2 pi i x y / N) =
prod_q w_q^(x_q) with w_q = exp(2 pi i 2^q y / N), so one output is a chain
of n halvings of the state vector (about 2N flops, no length-N exp)."""
import math

import numpy as np


def qft_output(psi, y):
    n = int(psi.size).bit_length() - 1
    N = 1 << n
    v = psi
    for q in range(n - 1, -1, -1):          # split off the top bit each time
        half = v.size // 2
        w = np.exp(2j * math.pi * ((y << q) % N) / N)
        v = v[:half] + w * v[half:]
    return complex(v[0]) / math.sqrt(N)
