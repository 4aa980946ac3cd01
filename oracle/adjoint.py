"""Oracle: gradients of Chebyshev moments by the plain reverse of the recurrence (test infrastructure only).

The paper computes the moments mu_n = <phi_L|T_n(H~)|phi_R> by the forward
recurrence v_0 = phi_R, v_1 = H~ v_0, v_n = 2 H~ v_{n-1} - v_{n-2}
(Sections 3.2-3.3); it has no derivatives.  For a loss L = sum_n w_n Re mu_n
the reverse of that recurrence (every v_n stored, DeltaE held fixed) is

  lam_M = lam_{M+1} = 0,  lam_n = w_n phi_L + 2 H~ lam_{n+1} - lam_{n+2}   (n = M-1 .. 1)
  dL/dp = Re[ sum_{n>=2} 2 <lam_n| dH~/dp v_{n-1}> + <lam_1| dH~/dp v_0> ]

Parameters:
  * on-site U_i:  dH~/dU_i = e_i e_i^T / DeltaE;
  * hopping class c, as the relative change H_ij -> (1 + eps_c) H_ij on every
    bond of class c, at eps_c = 0:  dH~/deps_c = H_c / DeltaE, where H_c is the
    class-c part of the hopping matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def class_parts(nn, nbr, hop, hop_class, n_class):
    """H_c: the hoppings of class c as separate sparse matrices."""
    n, k = nbr.shape
    slot = np.arange(k)[None, :]
    valid = slot < np.asarray(nn)[:, None]
    rows = np.broadcast_to(np.arange(n)[:, None], (n, k))[valid]
    cols = np.asarray(nbr)[valid].astype(np.int64)
    vals = (np.full(rows.shape[0], -1.0 + 0j) if hop is None
            else np.asarray(hop)[valid].astype(np.complex128))
    cls = (np.zeros(rows.shape[0], dtype=np.int64) if hop_class is None
           else np.asarray(hop_class)[valid])
    return [sp.coo_matrix((np.where(cls == c, vals, 0), (rows, cols)), shape=(n, n)).tocsr()
            for c in range(n_class)]


def moments_gradient(H, phiL, phiR, energy_max, weights, H_classes=()):
    """Gradient of L = sum_{n,b} w[n,b] Re mu[n,b] w.r.t. on-site energies and class scales.

    Returns (grad_onsite [n], grad_class [len(H_classes)]).
    """
    Ht = H / energy_max
    phiL = np.asarray(phiL, dtype=np.complex128)
    phiR = np.asarray(phiR, dtype=np.complex128)
    if phiL.ndim == 1:
        phiL, phiR = phiL[:, None], phiR[:, None]
    w = np.asarray(weights, dtype=np.float64)
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
        lam[n] = w[n] * phiL + 2.0 * (Ht @ lam[n + 1]) - lam[n + 2]
    gU = np.zeros(H.shape[0])
    gC = np.zeros(len(H_classes))
    for n in range(1, M):
        f = 1.0 if n == 1 else 2.0
        gU += f * np.sum(np.real(np.conj(lam[n]) * v[n - 1]), axis=1)
        for c, Hc in enumerate(H_classes):
            gC[c] += f * np.sum(np.real(np.conj(lam[n]) * (Hc @ v[n - 1])))
    return gU / energy_max, gC / energy_max
