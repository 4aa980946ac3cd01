"""Oracle: gradients by the plain reverse of the recurrences, every vector stored (test infrastructure only).

The paper computes the moments mu_n = <phi_L|T_n(H~)|phi_R> by the forward
recurrence v_0 = phi_R, v_1 = H~ v_0, v_n = 2 H~ v_{n-1} - v_{n-2}
(Sections 3.2-3.3); it has no derivatives.  For a loss
L = sum_n Re(w_n mu_n) (w_n real for moment losses, complex for the
evolution series) the reverse of that recurrence (DeltaE held fixed) is

  lam_M = lam_{M+1} = 0,  lam_n = conj(w_n) phi_L + 2 H~ lam_{n+1} - lam_{n+2}   (n = M-1 .. 1)
  dL/dp = Re[ sum_{n>=2} 2 <lam_n| dH~/dp v_{n-1}> + <lam_1| dH~/dp v_0> ]

and the adjoint of phi_R is lam_0 = sum_n conj(w_n) T_n(H~) phi_L.

Parameters:
  * on-site U_i:  dH~/dU_i = e_i e_i^T / DeltaE;
  * hopping class c, as the relative change H_ij -> (1 + eps_c) H_ij on every
    bond of class c, at eps_c = 0:  dH~/deps_c = H_c / DeltaE, and the velocity
    V = i dx H changes by V_c = i dx H_c;
  * one stored entry H_ij on its own (complex): a change dH_ij = delta changes L
    by Re(delta g_ij) with g_ij = sum_n f_n <lam_n|e_i> <e_j|v_{n-1}> / DeltaE
    (+ i dx_ij conj(a_i) x_j for every velocity application a^+ V x), so
    dL/dRe H_ij = Re g_ij and dL/dIm H_ij = -Im g_ij.  For a Hermitian H whose
    bond carries h = H_ij = conj(H_ji), dL/dRe h and dL/dIm h add the two
    entries' values with the sign of Im flipped on the partner (tie_hermitian).

The VAC gradient reverses the whole computation of vac_moments (the reading
C_n(t_k) = Re <V psi_L(k)|T_n|psi_R(k)>, psi_{L,R}(k+1) = U(-dt_k) psi_{L,R}(k),
psi_L(0) = phi, psi_R(0) = V phi): per row the two moment adjoints, through the
velocity V (Hermitian, so its adjoint is V itself), and through each evolution
U(-dt) = sum_m c_m T_m(H~), whose adjoint is U(+dt).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .kpm import chebyshev_series
from .operators import position_differences
from .transport import evolution_coefficients, evolve, _np_for


def _entries(nn, nbr, hop, hop_class):
    n, k = nbr.shape
    slot = np.arange(k)[None, :]
    valid = slot < np.asarray(nn)[:, None]
    rows = np.broadcast_to(np.arange(n)[:, None], (n, k))[valid]
    cols = np.asarray(nbr)[valid].astype(np.int64)
    vals = (np.full(rows.shape[0], -1.0 + 0j) if hop is None
            else np.asarray(hop)[valid].astype(np.complex128))
    cls = (np.zeros(rows.shape[0], dtype=np.int64) if hop_class is None
           else np.asarray(hop_class)[valid])
    return n, rows, cols, vals, cls


def class_parts(nn, nbr, hop, hop_class, n_class):
    """H_c: the hoppings of class c as separate sparse matrices."""
    n, rows, cols, vals, cls = _entries(nn, nbr, hop, hop_class)
    return [sp.coo_matrix((np.where(cls == c, vals, 0), (rows, cols)), shape=(n, n)).tocsr()
            for c in range(n_class)]


def velocity_class_parts(nn, nbr, hop, hop_class, n_class, x, length_x):
    """V_c = i dx H_c: the velocity operator restricted to the hoppings of class c."""
    n, rows, cols, vals, cls = _entries(nn, nbr, hop, hop_class)
    dx = position_differences(x, rows, cols, length_x)
    return [sp.coo_matrix((np.where(cls == c, 1j * dx * vals, 0), (rows, cols)), shape=(n, n)).tocsr()
            for c in range(n_class)]


def _as_cols(a):
    a = np.asarray(a, dtype=np.complex128)
    return a[:, None] if a.ndim == 1 else a


def entry_list(nn, nbr, x=None, length_x=0.0):
    """The stored entries of a neighbour list in the input layout: (rows, cols, slots, dx),
    slot s of row i at flat index i * max_nn + s."""
    n, k = nbr.shape
    slot = np.broadcast_to(np.arange(k)[None, :], (n, k))
    valid = slot < np.asarray(nn)[:, None]
    rows = np.broadcast_to(np.arange(n)[:, None], (n, k))[valid]
    cols = np.asarray(nbr)[valid].astype(np.int64)
    flat = (rows * k + slot[valid]).astype(np.int64)
    dx = None if x is None else position_differences(x, rows, cols, length_x)
    return rows, cols, flat, dx


def tie_hermitian(nn, nbr, g):
    """Per-entry gradient pairs (dL/dRe, dL/dIm) [n, max_nn, 2] of independent entries ->
    the gradient of each Hermitian bond h = H_ij = conj(H_ji), stored at both entries of
    the pair (the partner's Im with the opposite sign).  The q-th entry of row i that
    points to j pairs with the q-th entry of row j that points to i; an entry without a
    partner keeps its own value."""
    n, k = nbr.shape
    out = np.array(g, dtype=np.float64, copy=True)
    for i in range(n):
        for s in range(nn[i]):
            j = nbr[i, s]
            q = sum(1 for t in range(s) if nbr[i, t] == j)
            hits = [t for t in range(nn[j]) if nbr[j, t] == i]
            if q < len(hits):
                p = hits[q]
                out[i, s, 0] = g[i, s, 0] + g[j, p, 0]
                out[i, s, 1] = g[i, s, 1] - g[j, p, 1]
    return out


def _add_entries(gH, entries, lam, v, f, scale):
    """gH[flat] += f (Re g, -Im g), g = sum_b conj(lam[i, b]) v[j, b] * scale."""
    rows, cols, flat, _ = entries
    g = np.sum(np.conj(lam[rows]) * v[cols], axis=1) * scale * f
    gH[flat, 0] += np.real(g)
    gH[flat, 1] += -np.imag(g)


def _add_velocity_entries(gH, entries, a, xv):
    """The velocity's share a^+ V x (V_ij = i dx_ij H_ij, unscaled): g_ij = i dx_ij conj(a_i) x_j."""
    rows, cols, flat, dx = entries
    g = 1j * dx * np.sum(np.conj(a[rows]) * xv[cols], axis=1)
    gH[flat, 0] += np.real(g)
    gH[flat, 1] += -np.imag(g)


def moments_gradient(H, phiL, phiR, energy_max, weights, H_classes=(), entries=None, gH=None):
    """Gradient of L = sum_{n,b} Re(w[n,b] mu[n,b]) w.r.t. on-site energies and class scales,
    and (entries = entry_list(...), gH [n * max_nn, 2] accumulated) w.r.t. each stored entry.

    Returns (grad_onsite [n], grad_class [len(H_classes)]).
    """
    Ht = H / energy_max
    phiL, phiR = _as_cols(phiL), _as_cols(phiR)
    w = np.asarray(weights)
    if w.ndim == 1:
        w = w[:, None]
    M = w.shape[0]
    v = [phiR]
    if M > 1:
        v.append(Ht @ phiR)
    for n in range(2, M):
        v.append(2.0 * (Ht @ v[n - 1]) - v[n - 2])
    lam = [None] * (M + 2)
    lam[M] = np.zeros_like(phiR)
    lam[M + 1] = np.zeros_like(phiR)
    for n in range(M - 1, 0, -1):
        lam[n] = np.conj(w[n]) * phiL + 2.0 * (Ht @ lam[n + 1]) - lam[n + 2]
    gU = np.zeros(H.shape[0])
    gC = np.zeros(len(H_classes))
    for n in range(1, M):
        f = 1.0 if n == 1 else 2.0
        gU += f * np.sum(np.real(np.conj(lam[n]) * v[n - 1]), axis=1)
        for c, Hc in enumerate(H_classes):
            gC[c] += f * np.sum(np.real(np.conj(lam[n]) * (Hc @ v[n - 1])))
        if entries is not None:
            _add_entries(gH, entries, lam[n], v[n - 1], f, 1.0 / energy_max)
    return gU / energy_max, gC / energy_max


def vac_gradient(H, V, phi, dts, energy_max, M, weights, Np=0, H_classes=(), V_classes=(), entries=None,
                 gH=None):
    """Gradient of L = sum_{k,n,b} w[k,n,b] C_n^VAC(t_k)[b] w.r.t. on-site energies and class scales,
    and (entries with dx, gH accumulated) w.r.t. each stored entry."""
    Ht = H / energy_max
    phi = _as_cols(phi)
    w = np.asarray(weights, dtype=np.float64)
    n_t = len(dts)
    psiL = [phi]
    psiR = [V @ phi]
    for k in range(n_t - 1):
        psiL.append(evolve(Ht, psiL[-1], -dts[k], energy_max, Np))
        psiR.append(evolve(Ht, psiR[-1], -dts[k], energy_max, Np))
    gU = np.zeros(H.shape[0])
    gC = np.zeros(len(H_classes))
    gL = np.zeros_like(phi)
    gR = np.zeros_like(phi)
    for k in range(n_t - 1, -1, -1):
        phiL = V @ psiL[k]
        u, c = moments_gradient(H, phiL, psiR[k], energy_max, w[k], H_classes, entries, gH)
        gU += u
        gC += c
        gR = gR + np.stack([chebyshev_series(Ht, w[k][:, b], phiL[:, b]) for b in range(phi.shape[1])], 1)
        gphiL = np.stack([chebyshev_series(Ht, w[k][:, b], psiR[k][:, b]) for b in range(phi.shape[1])], 1)
        gL = gL + V @ gphiL
        for q, Vc in enumerate(V_classes):
            gC[q] += np.sum(np.real(np.conj(gphiL) * (Vc @ psiL[k])))
        if entries is not None:
            _add_velocity_entries(gH, entries, gphiL, psiL[k])
        if k > 0:
            dt = -dts[k - 1]
            coef = evolution_coefficients(dt, energy_max, _np_for(dt, energy_max, Np))
            cw = np.repeat(coef[:, None], phi.shape[1], axis=1)
            for g_, psi_ in ((gL, psiL[k - 1]), (gR, psiR[k - 1])):
                u, c = moments_gradient(H, g_, psi_, energy_max, cw, H_classes, entries, gH)
                gU += u
                gC += c
            gL = evolve(Ht, gL, -dt, energy_max, len(coef))     # U(-dt)^+ = U(+dt)
            gR = evolve(Ht, gR, -dt, energy_max, len(coef))
    for q, Vc in enumerate(V_classes):
        gC[q] += np.sum(np.real(np.conj(gR) * (Vc @ phi)))
    if entries is not None:
        _add_velocity_entries(gH, entries, gR, phi)
    return gU, gC
