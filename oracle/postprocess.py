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
