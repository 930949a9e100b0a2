"""Feed-angle (parallactic-angle-equivalent) correction of dual-polarisation products.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper lists, among the space-VLBI correlator's capabilities, the
equivalent of the parallactic-angle correction for the spaceborne antenna,
computed from the spacecraft orientation in its telemetry (section 2, the
capability list).  The telemetry is not available, so the feed angles are
inputs here.  Conventions fixed (the paper gives none):

P1  a feed turned by chi (per station and sub-integration) sees, for linear
    feeds, X' = X cos chi + Y sin chi, Y' = -X sin chi + Y cos chi; for
    circular feeds (R = (X + iY)/sqrt2, L = (X - iY)/sqrt2) that is
    R' = exp(-i chi) R, L' = exp(+i chi) L.
P2  products V_ij = <Y_i conj(Y_j)> of inputs i = 2 s + p (p = 0: X or R,
    p = 1: Y or L), packed upper triangle i <= j as the correlator writes them.
P3  the correction returns the products the unrotated feeds would give:
    circular V_ij exp(+i (s_p chi_a - s_q chi_b)) with s_R = +1, s_L = -1;
    linear, per station pair (a, b), the 2 x 2 block V <- Rot(chi_a)^T V Rot(chi_b)
    with Rot(chi) = [[cos, sin], [-sin, cos]] (for a = b the stored entries
    (0,0), (0,1), (1,1) of the Hermitian block).
"""
from __future__ import annotations

import numpy as np

CIRCULAR, LINEAR = 0, 1


def bl_index(i: int, j: int, M: int) -> int:
    """Packed row-major upper-triangle index of (i <= j)."""
    return i * M - i * (i - 1) // 2 + (j - i)


def rot(chi: float) -> np.ndarray:
    """P1: voltage rotation of a linear feed turned by chi."""
    c, s = np.cos(chi), np.sin(chi)
    return np.array([[c, s], [-s, c]])


def correct(V: np.ndarray, angles: np.ndarray, feed: int) -> np.ndarray:
    """P3 on V[T, n_sb, nbl, n_chan] with angles[T, S] (radians); returns a new array."""
    V = np.array(V, dtype=np.complex128)
    T, n_sb, nbl, _ = V.shape
    S = angles.shape[1]
    M = 2 * S
    assert nbl == M * (M + 1) // 2
    sgn = (1.0, -1.0)
    for t in range(T):
        chi = angles[t]
        for a in range(S):
            for b in range(a, S):
                idx = {(p, q): bl_index(2 * a + p, 2 * b + q, M)
                       for p in range(2) for q in range(2) if 2 * a + p <= 2 * b + q}
                if feed == CIRCULAR:
                    for (p, q), k in idx.items():
                        V[t, :, k, :] *= np.exp(1j * (sgn[p] * chi[a] - sgn[q] * chi[b]))
                else:
                    blk = np.empty((2, 2) + V.shape[1:2] + V.shape[3:], complex)
                    for p in range(2):
                        for q in range(2):
                            if (p, q) in idx:
                                blk[p, q] = V[t, :, idx[p, q], :]
                            else:                          # a = b: the Hermitian partner
                                blk[p, q] = np.conj(V[t, :, idx[q, p], :])
                    out = np.einsum("mp,mn...,nq->pq...", rot(chi[a]), blk, rot(chi[b]))
                    for (p, q), k in idx.items():
                        V[t, :, k, :] = out[p, q]
    return V
