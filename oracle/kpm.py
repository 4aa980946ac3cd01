"""Oracle: Chebyshev moments, Jackson kernel and KPM reconstruction (test infrastructure only).

Section 3.3: the resolution operator delta(E - H) is expanded in Chebyshev
polynomials of the scaled Hamiltonian H~ = H / DeltaE (Section 3.2), giving
moments C_n = <phi_L| T_n(H~) |phi_R> and the reconstruction

    f(E) = 2 / (pi Omega DeltaE sqrt(1 - E~^2)) * sum_{n<N_m} g_n (2 - delta_n0) T_n(E~) C_n

with E~ = E / DeltaE and the Jackson damping g_n.  The moments use the
three-term recurrence T_m = 2 H~ T_{m-1} - T_{m-2}, T_0 = 1, T_1 = H~
(Section 3.2).  The reconstruction evaluates T_n(E~) as cos(n arccos E~),
the closed form, on purpose not by recurrence.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    """<a|b> per column, numpy pairwise summation."""
    return np.sum(np.conj(a) * b, axis=0)


def chebyshev_moments(Ht, phiL, phiR, M):
    """mu[n, b] = <phiL_b | T_n(Ht) | phiR_b> for n < M (Section 3.3, Chebyshev moments).

    Ht is the already-scaled Hamiltonian (sparse); phiL, phiR are [n, B].
    """
    phiL = np.asarray(phiL, dtype=np.complex128)
    phiR = np.asarray(phiR, dtype=np.complex128)
    if phiL.ndim == 1:
        phiL = phiL[:, None]
        phiR = phiR[:, None]
    B = phiR.shape[1]
    mu = np.zeros((M, B), dtype=np.complex128)
    if M == 0:
        return mu
    v_prev = phiR                       # T_0 phi_R
    mu[0] = _dot(phiL, v_prev)
    if M == 1:
        return mu
    v = Ht @ phiR                       # T_1 phi_R
    mu[1] = _dot(phiL, v)
    for n in range(2, M):
        v_next = 2.0 * (Ht @ v) - v_prev
        mu[n] = _dot(phiL, v_next)
        v_prev, v = v, v_next
    return mu


def chebyshev_series(Ht, c, psi):
    """sum_n c[n] T_n(Ht) psi for a coefficient list c (complex allowed), by the Section 3.2 recurrence."""
    psi = np.asarray(psi, dtype=np.complex128)
    c = np.asarray(c)
    out = c[0] * psi
    if len(c) == 1:
        return out
    t_prev, t_cur = psi, Ht @ psi
    out = out + c[1] * t_cur
    for n in range(2, len(c)):
        t_prev, t_cur = t_cur, 2.0 * (Ht @ t_cur) - t_prev
        out = out + c[n] * t_cur
    return out


def jackson(M):
    """Jackson damping g_n = (1 - n a) cos(pi n a) + a sin(pi n a) cot(pi a), a = 1/(M+1) (Section 3.3)."""
    a = 1.0 / (M + 1)
    n = np.arange(M, dtype=np.float64)
    return (1.0 - n * a) * np.cos(np.pi * n * a) + a * np.sin(np.pi * n * a) / np.tan(np.pi * a)


def chebyshev_T(n, x):
    """T_n(x) = cos(n arccos x) for |x| <= 1 (closed form)."""
    return np.cos(np.multiply.outer(np.asarray(n, dtype=np.float64), np.arccos(x)))


def kpm_reconstruct(C, energies, energy_max, volume, damping=None):
    """KPM sum of Section 3.3 (same prefactor for DOS, rho*C_vv and rho*DeltaX^2).

    C: moments [M] or [M, ...] (real parts are used), energies: [n_E].
    Returns f with shape [n_E] + C.shape[1:].
    """
    C = np.real(np.asarray(C))
    M = C.shape[0]
    g = jackson(M) if damping is None else np.asarray(damping)
    Et = np.asarray(energies, dtype=np.float64) / energy_max
    if np.any(np.abs(Et) >= 1.0):
        raise ValueError("every energy must satisfy |E| < DeltaE")
    w = g * np.where(np.arange(M) == 0, 1.0, 2.0)
    T = chebyshev_T(np.arange(M), Et)                    # [M, n_E]
    pref = 2.0 / (np.pi * volume * energy_max * np.sqrt(1.0 - Et ** 2))
    s = np.tensordot(T * w[:, None], C, axes=([0], [0]))  # [n_E, ...]
    return s * pref.reshape((-1,) + (1,) * (s.ndim - 1))
