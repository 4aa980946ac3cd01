"""Oracle: the tight-binding operators H, V = i[H, X] and [X, H] (test infrastructure only).

Section 4.2 defines H = sum_mn H_mn |m><n| + sum_m U_m |m><m| from a
neighbour list, hoppings and on-site potentials; X is diagonal with the site
coordinates along the transport direction; V = (i/hbar)[H, X] has elements
(i/hbar)(X_n - X_m) H_mn.  With hbar = 1 (Section 4.2.6) and X - X written as
the position difference dx_mn = X_n - X_m, [X, H] has elements -dx_mn H_mn.
Periodic boundaries: the paper gives the period along x (Section 4.2.4) so
that bonds across the boundary get the short difference; we take the minimum
image dx - L round(dx / L).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _bond_lists(nn, nbr, hop):
    n, k = nbr.shape
    slot = np.arange(k)[None, :]
    valid = slot < np.asarray(nn)[:, None]
    rows = np.broadcast_to(np.arange(n)[:, None], (n, k))[valid]
    cols = np.asarray(nbr)[valid].astype(np.int64)
    if hop is None:
        vals = np.full(rows.shape[0], -1.0 + 0j)   # paper's default hopping
    else:
        vals = np.asarray(hop)[valid].astype(np.complex128)
    return rows, cols, vals


def position_differences(x, rows, cols, length_x):
    """dx = X_col - X_row, minimum image when length_x > 0 (Section 4.2.4)."""
    d = np.asarray(x)[cols] - np.asarray(x)[rows]
    if length_x > 0:
        d = d - length_x * np.round(d / length_x)
    return d


def operators(nn, nbr, hop, onsite, x, length_x):
    """Return (H, V, XH) as complex128 CSR matrices.

    H  : hoppings plus on-site diagonal (Section 4.2, Hamiltonian).
    V  : i * dx * H_mn on bonds (Section 4.2, velocity operator, hbar = 1).
    XH : [X, H] = -dx * H_mn on bonds (zero diagonal).
    Duplicate bonds (a neighbour listed twice) are summed, as the paper's
    double sum over m, n does.
    """
    n = len(nn)
    rows, cols, vals = _bond_lists(nn, nbr, hop)
    dx = position_differences(x, rows, cols, length_x)
    U = np.zeros(n) if onsite is None else np.asarray(onsite, dtype=np.float64)
    H = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr() \
        + sp.diags(U.astype(np.complex128), 0, format="csr")
    V = sp.coo_matrix((1j * dx * vals, (rows, cols)), shape=(n, n)).tocsr()
    XH = sp.coo_matrix((-dx * vals, (rows, cols)), shape=(n, n)).tocsr()
    return H.tocsr(), V, XH


def gershgorin_bound(H):
    """max_i sum_j |H_ij| (diagonal included): every eigenvalue lies within it."""
    A = abs(H).tocsr()
    return float(np.max(np.asarray(A.sum(axis=1)).ravel())) if H.shape[0] else 0.0
