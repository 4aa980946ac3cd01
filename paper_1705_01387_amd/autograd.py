"""torch.autograd Functions over the library's forward and adjoint entry points.

Parameters are the on-site energies U (float64 CUDA tensor [n]) and the
hopping-class scales s (float64 tensor [n_class]; every hopping of class c
is s_c times the hopping given when the handle was built).  DeltaE stays fixed.
Forward and backward both set the handle to the given parameter values
(gpuqt_update_h_values) before running, so interleaved calls stay consistent.
The library's class gradients are dL/ds_c themselves (taken against the
build-time hoppings), so they are finite at every scale, s_c = 0 included.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as Bd


def _set(H, onsite, scales):
    Bd.gpuqt_update_h_values(H, onsite.detach().contiguous(), scales.detach().cpu().numpy())


class Moments(torch.autograd.Function):
    """Re <phi|T_n(H~)|phi>, shape [n_seg, B, M]."""

    @staticmethod
    def forward(ctx, onsite, scales, H, phi, M):
        _set(H, onsite, scales)
        mu = Bd.gpuqt_moments(H, phi, phi, M)
        ctx.H, ctx.M = H, M
        ctx.save_for_backward(onsite, scales, phi)
        return mu.real.contiguous()

    @staticmethod
    def backward(ctx, g):
        onsite, scales, phi = ctx.saved_tensors
        H = ctx.H
        _set(H, onsite, scales)
        gU = torch.zeros_like(onsite)
        gC = torch.zeros(scales.shape[0], dtype=torch.float64, device=onsite.device)
        Bd.gpuqt_moments_backward(H, phi, phi, g.contiguous(), gU, gC)
        return gU, gC.to(scales.device), None, None, None


class VAC(torch.autograd.Function):
    """C_n^VAC(t_k) rows, shape [n_t, n_seg, B, M].

    When a gradient is needed and the recorded forward (states, moment and evolution
    chains, gpuqt_vac_tape_size) fits in Bd.KEEP_ALL_FRACTION of the free device memory, the
    forward keeps it and the backward recomputes nothing; otherwise the backward
    re-evolves and recomputes as gpuqt_vac_backward does."""

    @staticmethod
    def forward(ctx, onsite, scales, H, phi, dt, M, Np):
        _set(H, onsite, scales)
        dtn = np.asarray(dt, dtype=np.float64)
        ctx.tape = None
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            need = Bd.gpuqt_vac_tape_size(H, Bd._cols(phi), dtn, M, Np)
            free, _ = torch.cuda.mem_get_info(phi.device)
            if need <= Bd.KEEP_ALL_FRACTION * free:
                out, ctx.tape = Bd.gpuqt_vac_record(H, phi, dtn, M, Np)
        if ctx.tape is None:
            out = Bd.gpuqt_vac(H, phi, dtn, M, Np)
        ctx.H, ctx.dt, ctx.Np = H, dtn, Np
        ctx.save_for_backward(onsite, scales, phi)
        return out

    @staticmethod
    def backward(ctx, g):
        onsite, scales, phi = ctx.saved_tensors
        H = ctx.H
        _set(H, onsite, scales)
        gU = torch.zeros_like(onsite)
        gC = torch.zeros(scales.shape[0], dtype=torch.float64, device=onsite.device)
        if ctx.tape is not None:
            Bd.gpuqt_vac_backward_tape(H, phi, ctx.dt, g.contiguous(), ctx.tape, gU, gC, Np=ctx.Np)
            ctx.tape = None
        else:
            Bd.gpuqt_vac_backward(H, phi, ctx.dt, g.contiguous(), gU, gC, Np=ctx.Np)
        return gU, gC.to(scales.device), None, None, None, None, None


class KPM(torch.autograd.Function):
    """Jackson-damped KPM sum of moment rows C [R, M] on an energy grid -> [R, n_E]."""

    @staticmethod
    def forward(ctx, C, energies, energy_max, volume):
        ctx.args = (np.asarray(energies, dtype=np.float64), int(C.shape[-1]), float(energy_max),
                    float(volume))
        return Bd.gpuqt_kpm_reconstruct(C.detach().contiguous(), energies, energy_max, volume)

    @staticmethod
    def backward(ctx, g):
        E, M, dE, vol = ctx.args
        return Bd.gpuqt_kpm_reconstruct_adjoint(g.contiguous(), E, M, dE, vol), None, None, None
