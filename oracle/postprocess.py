"""Oracle: running electrical conductivity from the reconstructed correlation rows
(test infrastructure only).

Section 2.2 (e = 1):
  sigma^VAC(E, t) = rho(E) int_0^t C_vv(E, t') dt'
  sigma^MSD(E, t) = rho(E) (1/2) d/dt DeltaX^2(E, t)
The library returns rho C_vv and rho DeltaX^2 on an energy grid at the row times
(gpuqt_vac / gpuqt_msd moments, then the KPM sum), so both are post-processing of
those rows over time.

Readings where the paper is silent (each listed in the design notes):
  * The VAC rows sit at t_k = dt_0 + ... + dt_{k-1} (row 0 at t = 0); the time
    integral is the trapezoid rule over consecutive rows, sigma^VAC(t_0) = 0.
  * The MSD rows sit at t_{k+1} = dt_0 + ... + dt_k with DeltaX^2 = 0 at t = 0;
    the derivative is that of the straight line between consecutive rows,
    (y_k - y_{k-1}) / dt_k (y_{-1} = 0), taken at the midpoint t_{k+1} - dt_k / 2.
    A zero time step has no derivative (NaN).
"""
from __future__ import annotations

import numpy as np


def sigma_vac(rows, dt):
    """rows [N_t, n_E] of rho C_vv at t_k; returns sigma^VAC [N_t, n_E] at the same times."""
    rows = np.asarray(rows, dtype=float)
    dt = np.asarray(dt, dtype=float)
    out = np.zeros_like(rows)
    for k in range(1, rows.shape[0]):
        out[k] = out[k - 1] + 0.5 * dt[k - 1] * (rows[k - 1] + rows[k])
    return out


def sigma_msd(rows, dt):
    """rows [N_t, n_E] of rho DeltaX^2 at t_{k+1}; returns (sigma^MSD [N_t, n_E], midpoint times)."""
    rows = np.asarray(rows, dtype=float)
    dt = np.asarray(dt, dtype=float)
    out = np.empty_like(rows)
    prev = np.zeros(rows.shape[1])
    for k in range(rows.shape[0]):
        with np.errstate(divide="ignore", invalid="ignore"):
            out[k] = (rows[k] - prev) / (2.0 * dt[k]) if dt[k] != 0 else np.nan
        prev = rows[k]
    t_mid = np.cumsum(dt) - 0.5 * dt
    return out, t_mid


def transport_lengths(rho, vac0=None, sigma=None, msd=None):
    """Transport regimes of Section 2.2 from reconstructed rows (e = hbar = 1).

    rho [n_E] the DOS; vac0 [n_E] rho C_vv at t = 0 (VAC row 0); sigma [N_t, n_E] a
    running conductivity (from sigma_vac or sigma_msd); msd [N_t, n_E] rho DeltaX^2.
    Returns a dict with whatever the inputs allow:
      sigma_sc = the maximum over the rows of sigma (the paper's choice of the semiclassical
                 conductivity; NaN rows skipped),
      v        = sqrt(C_vv(E, 0)), the group velocity (C_vv = rho C_vv / rho),
      tau      = sigma_sc / (rho v^2)      (equation sigma_sc solved for tau),
      mfp      = v tau                     (equation mfp),
      L        = 2 sqrt(DeltaX^2(E, t))    (equation L, per row),
      xi       = L(E, t_last) / (2 pi)     (equation xi, the last row standing for t -> inf).
    Readings: NaN where rho <= 0, where C_vv(E, 0) < 0 (v), where rho v^2 <= 0 (tau, mfp)
    and where DeltaX^2 < 0 (L, xi)."""
    rho = np.asarray(rho, dtype=float)
    ok = rho > 0
    out = {}
    if sigma is not None:
        s = np.asarray(sigma, dtype=float)
        sc = np.full(rho.shape, np.nan)
        for e in range(rho.shape[0]):
            col = s[:, e]
            col = col[~np.isnan(col)]
            if col.size:
                sc[e] = col.max()
        out["sigma_sc"] = sc
    if vac0 is not None:
        c0 = np.asarray(vac0, dtype=float)
        cvv = np.where(ok, c0 / np.where(ok, rho, 1.0), np.nan)
        v = np.where(cvv >= 0, np.sqrt(np.abs(cvv)), np.nan)
        out["v"] = v
        if sigma is not None:
            good = ok & (c0 > 0)
            tau = np.where(good, out["sigma_sc"] / np.where(good, c0, 1.0), np.nan)
            out["tau"] = tau
            out["mfp"] = v * tau
    if msd is not None:
        m = np.asarray(msd, dtype=float)
        dx2 = np.where(ok[None, :], m / np.where(ok, rho, 1.0)[None, :], np.nan)
        L = np.where(dx2 >= 0, 2.0 * np.sqrt(np.abs(dx2)), np.nan)
        out["L"] = L
        out["xi"] = L[-1] / (2.0 * np.pi)
    return out
