"""x1 current correction for charge conservation with a wide Ampere stencil.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passage followed
----------------------
* Sec. 3.3, Eq. (correction) and the continuity/Gauss argument after it: the
  charge-conserving (Esirkepov) current satisfies continuity with the Yee
  divergence; to keep Gauss's law with the Ampere operator [k]_B1, the x1
  current is rescaled per Fourier mode along x1 (an FFT along x1 only).

Reading taken (the direction of the ratio)
------------------------------------------
The paper's second line of the continuity argument holds only if the current
that enters Ampere's law, J_A1, obeys  i[k]_B1 J_A1 = i[k]_Yee J_dep1,  where
J_dep1 is the deposited current.  So

    J_A1 = ([k]_Yee / [k]_B1) J_dep1   per mode along x1,

which is the identity when C^B = e1 (the Yee stencil).  The k1 = 0 mode takes
the limit of the ratio, 1 / sum_j (2j-1) C^B_j, which the order constraint of
App. B makes 1.
"""
from __future__ import annotations

import numpy as np

from . import stencil


def correction_ratio(CB, n1, dx1):
    """[k]_Yee/[k]_B1 on the n1 discrete wavenumbers of a periodic x1 axis
    (numpy FFT order).  Raises if [k]_B1 vanishes (to 1e-12 of its largest
    value) at a nonzero mode."""
    CB = np.asarray(CB, dtype=np.float64)
    k = 2 * np.pi * np.fft.fftfreq(n1, d=dx1)
    kY = stencil.yee_symbol(k, dx1)
    kB = stencil.symbol(CB, k, dx1)
    ratio = np.empty(n1)
    ratio[0] = 1.0 / np.sum((2 * np.arange(1, CB.size + 1) - 1) * CB)
    if np.any(np.abs(kB[1:]) <= 1e-12 * np.max(np.abs(kB))):
        raise ValueError("[k]_B1 vanishes at a nonzero x1 mode")
    ratio[1:] = kY[1:] / kB[1:]
    return ratio


def correct_x1(J1, CB, dx1):
    """Sec. 3.3, Eq. (correction): the Ampere-law x1 current from the
    deposited one, J1 indexed [..., i] along x1 (FFT along the last axis)."""
    J1 = np.asarray(J1, dtype=np.float64)
    ratio = correction_ratio(CB, J1.shape[-1], dx1)
    return np.real(np.fft.ifft(np.fft.fft(J1, axis=-1) * ratio, axis=-1))
