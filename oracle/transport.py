"""Oracle: Chebyshev-Bessel time evolution and the VAC / MSD moments (test infrastructure only).

Section 3.2:
  U(+-dt)|psi>      = sum_{m<Np} (2 - delta_0m) (-+i)^m J_m(DeltaE dt) T_m(H~) |psi>
  [X, U(dt)]|psi>   = sum_{m<Np} (2 - delta_0m) (-i)^m J_m(DeltaE dt) [X, T_m(H~)] |psi>
with H~ = H / DeltaE, hbar = 1, and the recurrences
  T_m = 2 H~ T_{m-1} - T_{m-2},                  T_0 = 1, T_1 = H~
  [X,T_m] = 2 [X,H~] T_{m-1} + 2 H~ [X,T_{m-1}] - [X,T_{m-2}],  [X,T_0] = 0, [X,T_1] = [X,H~].

Section 3.3 moments (one random vector phi, Section 3.1):
  C_n^DOS    = <phi| T_n |phi>
  C_n^VAC(t) = Re <phi| U(t) V T_n U(t)^+ V |phi>
  C_n^MSD(t) = <phi| [X,U(t)]^+ T_n [X,U(t)] |phi>

Readings where the paper is silent (each listed in the design notes):
  * VAC: with U(t)^+ = U(-t) and V Hermitian, <phi|U(t) V = (V U(-t) phi)^+, so
    C_n^VAC(t) = Re <V psi_L | T_n | psi_R> with psi_L = U(-t) phi and
    psi_R = U(-t) V phi, both advanced step by step with U(-dt_k).
    Row k is at t_k = dt_0 + ... + dt_{k-1} (row 0 at t = 0).
  * MSD: the commutator over a sequence of steps follows the product rule
    [X, U2 U1] = [X, U2] U1 + U2 [X, U1], i.e.
    chi_{k+1} = [X, U(dt_k)] psi_k + U(dt_k) chi_k,  psi_{k+1} = U(dt_k) psi_k,
    chi_0 = 0, psi_0 = phi.  Row k is at t_{k+1} = dt_0 + ... + dt_k.
  * The number of terms Np: when not given, the smallest m > DeltaE |dt| with
    |J_m(DeltaE |dt|)| < 1e-16 (the paper: up to machine precision, Np
    proportional to dt).
"""
from __future__ import annotations

import numpy as np
import scipy.special

from .kpm import chebyshev_moments


def auto_terms(tau, tol=1e-16):
    """Smallest m > tau with |J_m(tau)| < tol (number of terms kept: m)."""
    m = int(np.floor(tau)) + 1
    while abs(scipy.special.jv(m, tau)) >= tol:
        m += 1
    return m


def evolution_coefficients(dt, energy_max, Np):
    """c_m = (2 - delta_0m) (-i sgn(dt))^m J_m(DeltaE |dt|), m < Np (Section 3.2, first expansion)."""
    tau = energy_max * abs(dt)
    m = np.arange(Np)
    J = scipy.special.jv(m, tau)
    phase = (-1j * np.sign(dt) if dt != 0 else 1.0) ** m
    return np.where(m == 0, 1.0, 2.0) * phase * J


def _np_for(dt, energy_max, Np):
    return Np if Np > 0 else auto_terms(energy_max * abs(dt))


def evolve(Ht, psi, dt, energy_max, Np=0):
    """U(dt)|psi> = e^{-i H dt}|psi> (dt < 0 gives e^{+i H |dt|}); Section 3.2."""
    Np = _np_for(dt, energy_max, Np)
    c = evolution_coefficients(dt, energy_max, Np)
    psi = np.asarray(psi, dtype=np.complex128)
    t_prev = psi                                     # T_0 psi
    out = c[0] * t_prev
    if Np == 1:
        return out
    t_cur = Ht @ psi                                 # T_1 psi
    out = out + c[1] * t_cur
    for m in range(2, Np):
        t_next = 2.0 * (Ht @ t_cur) - t_prev
        out = out + c[m] * t_next
        t_prev, t_cur = t_cur, t_next
    return out


def commutator_evolve(Ht, XHt, psi, dt, energy_max, Np=0):
    """[X, U(dt)]|psi> by the [X, T_m] recurrence (Section 3.2, second expansion).

    XHt is [X, H~] = [X, H] / DeltaE.
    """
    Np = _np_for(dt, energy_max, Np)
    c = evolution_coefficients(dt, energy_max, Np)
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.zeros_like(psi)                         # c_0 [X, T_0] psi = 0
    if Np == 1:
        return out
    t_prev, t_cur = psi, Ht @ psi                    # T_0 psi, T_1 psi
    d_prev = np.zeros_like(psi)                      # [X, T_0] psi
    d_cur = XHt @ psi                                # [X, T_1] psi
    out = out + c[1] * d_cur
    for m in range(2, Np):
        d_next = 2.0 * (XHt @ t_cur) + 2.0 * (Ht @ d_cur) - d_prev
        t_next = 2.0 * (Ht @ t_cur) - t_prev
        out = out + c[m] * d_next
        d_prev, d_cur = d_cur, d_next
        t_prev, t_cur = t_cur, t_next
    return out


def dos_moments(H, phi, energy_max, M):
    """C_n^DOS = <phi|T_n(H~)|phi> (Section 3.3)."""
    return chebyshev_moments(H / energy_max, phi, phi, M)


def vac_moments(H, V, phi, dts, energy_max, M, Np=0):
    """C_n^VAC(t_k), k < len(dts), shape [N_t, M, B] (real; Section 3.3)."""
    Ht = H / energy_max
    phi = np.asarray(phi, dtype=np.complex128)
    if phi.ndim == 1:
        phi = phi[:, None]
    psiL = phi
    psiR = V @ phi
    out = []
    for k, dt in enumerate(dts):
        phiL = V @ psiL
        out.append(chebyshev_moments(Ht, phiL, psiR, M).real)
        if k + 1 < len(dts):
            psiL = evolve(Ht, psiL, -dt, energy_max, Np)
            psiR = evolve(Ht, psiR, -dt, energy_max, Np)
    return np.array(out)


def msd_moments(H, XH, phi, dts, energy_max, M, Np=0, return_states=False):
    """C_n^MSD(t_{k+1}), k < len(dts), shape [N_t, M, B] (real; Section 3.3)."""
    Ht = H / energy_max
    XHt = XH / energy_max
    phi = np.asarray(phi, dtype=np.complex128)
    if phi.ndim == 1:
        phi = phi[:, None]
    psi = phi
    chi = np.zeros_like(phi)
    out = []
    for dt in dts:
        chi = commutator_evolve(Ht, XHt, psi, dt, energy_max, Np) \
            + evolve(Ht, chi, dt, energy_max, Np)
        psi = evolve(Ht, psi, dt, energy_max, Np)
        out.append(chebyshev_moments(Ht, chi, chi, M).real)
    if return_states:
        return np.array(out), psi, chi
    return np.array(out)
