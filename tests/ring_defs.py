"""The ring sums of synthesis and of its transpose written out by their
definitions (Sec. 2.3, Eqs. 8-11), for tests of the ring kernels on
arbitrary inputs.  Plain numpy in FP64; the phase m (2j + s) is reduced
mod 2J in integers before it is scaled by pi / J."""
import numpy as np


def _phase(L1, J, s):
    m = np.arange(L1)[:, None]
    j = np.arange(J)[None, :]
    return np.pi * np.mod(m * (2 * j + s), 2 * J) / J  # (L+1, J)


def ring_direct(qr, J, s):
    """f_j = Re q_0 + 2 Re sum_{m>=1} q_m e^{i m phi_j}, phi_j = pi (2j + s) / J;
    qr: (L+1, B) complex -> (B, J)."""
    L1 = qr.shape[0]
    q = qr.copy()
    q[0] = q[0].real
    w = np.full(L1, 2.0)
    w[0] = 1.0
    return np.real((q * w[:, None]).T @ np.exp(1j * _phase(L1, J, s)))


def ring_direct_adjoint(y, L, J, s, wpos):
    """ybar_m = w_m sum_j y_j e^{-i m phi_j}, w_0 = 1, w_m = wpos (2: the
    transpose of ring_direct under sum Re q Re g + Im q Im g); y: (B, J) real
    -> (L+1, B) complex."""
    w = np.full(L + 1, float(wpos))
    w[0] = 1.0
    return (np.exp(-1j * _phase(L + 1, J, s)) @ y.T) * w[:, None]
