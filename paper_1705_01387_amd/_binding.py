"""ctypes binding of libgpuqt.so: the C entry points under the same names.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Vectors are torch complex128 tensors on the GPU in layout [n][B];
descriptor arrays are numpy arrays on the host.  The library is loaded from
the package directory; if it has not been built the binding raises instead
of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpuqt.so")

GPUQT_OK = 0
GPUQT_ERR_WORKSPACE = 4
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_LAYOUT", 3: "ERR_SPECTRUM", 4: "ERR_WORKSPACE",
                5: "ERR_HIP", 6: "ERR_NOMEM", 7: "ERR_UNSUPPORTED"}
OP_MOMENTS, OP_EVOLVE, OP_EVOLVE_COMMUTATOR, OP_VAC, OP_MSD, OP_MOMENTS_BACKWARD, OP_AUTOTUNE = range(7)
VELOCITY, COMMUTATOR_XH = 0, 1


class GpuqtError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("max_nn", ctypes.c_int32),
        ("nn", ctypes.c_void_p), ("nbr", ctypes.c_void_p), ("hop", ctypes.c_void_p),
        ("hop_is_complex", ctypes.c_int32), ("hop_class", ctypes.c_void_p),
        ("n_class", ctypes.c_int32), ("onsite", ctypes.c_void_p), ("x", ctypes.c_void_p),
        ("length_x", ctypes.c_double), ("volume", ctypes.c_double),
        ("energy_max", ctypes.c_double), ("n_segments", ctypes.c_int32),
        ("seg_offsets", ctypes.c_void_p), ("seg_energy_max", ctypes.c_void_p),
        ("seg_length_x", ctypes.c_void_p), ("check_hermitian", ctypes.c_int32),
        ("slice_height", ctypes.c_int32), ("band_rows", ctypes.c_int32), ("no_dictionary", ctypes.c_int32),
    ]


class HInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("n_segments", ctypes.c_int32), ("n_class", ctypes.c_int32),
        ("hop_mode", ctypes.c_int32), ("slice_height", ctypes.c_int32),
        ("n_slices", ctypes.c_int64), ("entries", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("max_width", ctypes.c_int32), ("uniform_width", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32), ("kernel_variant", ctypes.c_int32),
        ("device_bytes", ctypes.c_size_t), ("row_period", ctypes.c_int64),
        ("banded_mask", ctypes.c_int32), ("family_caps", ctypes.c_int32), ("max_nn", ctypes.c_int32),
        ("pencil_mask", ctypes.c_int32), ("box", ctypes.c_int32 * 3), ("box_msd", ctypes.c_int32),
        ("sheets", ctypes.c_int32),
    ]


class ModelParams(ctypes.Structure):
    _fields_ = [
        ("n_random_vectors", ctypes.c_int32), ("n_moments", ctypes.c_int32), ("energy_max", ctypes.c_double),
        ("calculate_vac", ctypes.c_int32), ("calculate_msd", ctypes.c_int32), ("n_energies", ctypes.c_int32),
        ("n_time_steps", ctypes.c_int32), ("energies", ctypes.c_void_p), ("time_steps", ctypes.c_void_p),
    ]


_lib = None

_SIGS = {
    "gpuqt_build_h": (ctypes.c_int32, [ctypes.POINTER(_Desc), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "gpuqt_destroy_h": (None, [ctypes.c_void_p]),
    "gpuqt_h_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(HInfo), ctypes.c_void_p, ctypes.c_void_p]),
    "gpuqt_workspace_size": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "gpuqt_moments": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p]),
    "gpuqt_moments_plain": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p]),
    "gpuqt_evolve": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gpuqt_apply_commutator": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gpuqt_vac": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gpuqt_msd": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gpuqt_kpm_reconstruct": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "gpuqt_jackson": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_void_p]),
    "gpuqt_bessel": (ctypes.c_int32, [ctypes.c_double, ctypes.c_int32, ctypes.c_void_p]),
    "gpuqt_auto_terms": (ctypes.c_int32, [ctypes.c_double]),
    "gpuqt_last_error": (ctypes.c_char_p, []),
    "gpuqt_moments_backward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                ctypes.c_size_t, ctypes.c_void_p]),
    "gpuqt_vac_backward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gpuqt_tie_entry_gradient": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p]),
    "gpuqt_vac_backward_workspace_size": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                           ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                           ctypes.c_int32, ctypes.c_int32,
                                                           ctypes.POINTER(ctypes.c_size_t)]),
    "gpuqt_transport_lengths": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32] + [ctypes.c_void_p] * 11),
    "gpuqt_vac_tape_size": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "gpuqt_vac_record": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p]),
    "gpuqt_vac_backward_tape": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                                 ctypes.c_size_t, ctypes.c_void_p]),
    "gpuqt_vac_backward_tape_workspace_size": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                                ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                                ctypes.POINTER(ctypes.c_size_t)]),
    "gpuqt_kpm_reconstruct_adjoint": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                                       ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                                                       ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                                       ctypes.c_void_p]),
    "gpuqt_set_timing": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "gpuqt_timing": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gpuqt_update_h_values": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "gpuqt_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "gpuqt_copy_probe": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gpuqt_set_variant": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "gpuqt_model_load": (ctypes.c_int32, [ctypes.c_char_p, ctypes.c_void_p]),
    "gpuqt_model_desc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "gpuqt_model_params": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "gpuqt_model_free": (None, [ctypes.c_void_p]),
    "gpuqt_running_conductivity": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gpuqt_schedule_rows": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "gpuqt_moments_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "gpuqt_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "gpuqt_tune_cache_key": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t]),
    "gpuqt_autotune_cached": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "gpuqt_tune_cache_load": (ctypes.c_int32, [ctypes.c_char_p]),
    "gpuqt_tune_cache_save": (ctypes.c_int32, [ctypes.c_char_p]),
    "gpuqt_tune_cache_clear": (None, []),
    "gpuqt_autotune_block": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                              ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "gpuqt_build_h_tuned": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
}

# kernel variants measured on the MI355X for the workloads of this package (see gpuqt_autotune_cached)
TUNE_CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.tsv")


def lib():
    """Load libgpuqt.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if os.path.exists(TUNE_CACHE_PATH) and L.gpuqt_tune_cache_load(os.fsencode(TUNE_CACHE_PATH)) != GPUQT_OK:
            raise RuntimeError(f"{TUNE_CACHE_PATH}: {L.gpuqt_last_error().decode()}")
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != GPUQT_OK:
        raise GpuqtError(st, where, lib().gpuqt_last_error().decode())


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stream(stream):
    """The raw hipStream_t of a torch stream, of a raw handle, or of torch's current stream."""
    if stream is not None:
        return getattr(stream, "cuda_stream", stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dev_vec(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _cols(t):
    return 1 if t.dim() == 1 else int(t.shape[1])


# --------------------------------------------------------------------------
# host helpers
# --------------------------------------------------------------------------

def gpuqt_last_error() -> str:
    return lib().gpuqt_last_error().decode()


def gpuqt_jackson(M: int) -> np.ndarray:
    g = np.zeros(max(M, 0))
    _check(lib().gpuqt_jackson(M, _ptr(g) if M > 0 else None), "gpuqt_jackson")
    return g


def gpuqt_bessel(tau: float, Np: int) -> np.ndarray:
    J = np.zeros(max(Np, 0))
    _check(lib().gpuqt_bessel(float(tau), Np, _ptr(J) if Np > 0 else None), "gpuqt_bessel")
    return J


def gpuqt_auto_terms(tau: float) -> int:
    return int(lib().gpuqt_auto_terms(float(tau)))


# --------------------------------------------------------------------------
# Hamiltonian handle
# --------------------------------------------------------------------------

class Hamiltonian:
    """Owner of a gpuqt_h handle (device layout of H on the current device)."""

    def __init__(self, handle: int, keep):
        self._h = ctypes.c_void_p(handle)
        self._keep = keep
        info = HInfo()
        _check(lib().gpuqt_h_info(self._h, ctypes.byref(info), None, None), "gpuqt_h_info")
        dE = np.zeros(info.n_segments)
        gb = np.zeros(info.n_segments)
        _check(lib().gpuqt_h_info(self._h, ctypes.byref(info), _ptr(dE), _ptr(gb)), "gpuqt_h_info")
        self.info = info
        self.energy_max = dE
        self.gershgorin = gb

    @property
    def handle(self):
        return self._h

    @property
    def n(self) -> int:
        return int(self.info.n)

    @property
    def n_segments(self) -> int:
        return int(self.info.n_segments)

    def close(self):
        if self._h is not None and self._h.value:
            lib().gpuqt_destroy_h(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gpuqt_build_h(nn, nbr, hop=None, onsite=None, x=None, length_x=0.0, volume=1.0,
                  energy_max=0.0, hop_class=None, n_class=1, seg_offsets=None,
                  seg_energy_max=None, seg_length_x=None, check_hermitian=False,
                  slice_height=0, band_rows=0, no_dictionary=False, tune_block=0,
                  stream=None) -> Hamiltonian:
    """Build the device layout of H from a neighbour list (the paper's input files).
    tune_block > 0: choose the slice height by measurement at that block width
    (gpuqt_build_h_tuned; the result's slice_tuning holds the height and the times)."""
    nn = np.ascontiguousarray(nn, dtype=np.int32)
    n = nn.shape[0]
    nbr = np.ascontiguousarray(nbr, dtype=np.int32).reshape(n, -1)
    max_nn = nbr.shape[1]
    keep = [nn, nbr]
    d = _Desc()
    d.n = n
    d.max_nn = max_nn
    d.nn = _ptr(nn)
    d.nbr = _ptr(nbr)
    if hop is not None:
        hop = np.asarray(hop)
        if np.iscomplexobj(hop):
            hop = np.ascontiguousarray(hop, dtype=np.complex128).reshape(n, max_nn)
            d.hop_is_complex = 1
        else:
            hop = np.ascontiguousarray(hop, dtype=np.float64).reshape(n, max_nn)
        keep.append(hop)
        d.hop = _ptr(hop)
    if hop_class is not None:
        hop_class = np.ascontiguousarray(hop_class, dtype=np.int32).reshape(n, max_nn)
        keep.append(hop_class)
        d.hop_class = _ptr(hop_class)
    d.n_class = int(n_class)
    if onsite is not None:
        onsite = np.ascontiguousarray(onsite, dtype=np.float64)
        keep.append(onsite)
        d.onsite = _ptr(onsite)
    if x is None:
        raise ValueError("positions x are required")
    x = np.ascontiguousarray(x, dtype=np.float64)
    keep.append(x)
    d.x = _ptr(x)
    d.length_x = float(length_x)
    d.volume = float(volume)
    d.energy_max = float(energy_max)
    if seg_offsets is not None:
        so = np.ascontiguousarray(seg_offsets, dtype=np.int64)
        keep.append(so)
        d.n_segments = so.shape[0] - 1
        d.seg_offsets = _ptr(so)
    if seg_energy_max is not None:
        se = np.ascontiguousarray(seg_energy_max, dtype=np.float64)
        keep.append(se)
        d.seg_energy_max = _ptr(se)
    if seg_length_x is not None:
        sl = np.ascontiguousarray(seg_length_x, dtype=np.float64)
        keep.append(sl)
        d.seg_length_x = _ptr(sl)
    d.check_hermitian = 1 if check_hermitian else 0
    d.slice_height = int(slice_height)
    d.band_rows = int(band_rows)
    d.no_dictionary = 1 if no_dictionary else 0
    out = ctypes.c_void_p()
    if tune_block:
        S = ctypes.c_int32()
        us = np.zeros(4)
        _check(lib().gpuqt_build_h_tuned(ctypes.byref(d), int(tune_block), _stream(stream) if stream else None,
                                         ctypes.byref(out), ctypes.byref(S), _ptr(us)), "gpuqt_build_h_tuned")
        H = Hamiltonian(out.value, None)
        H.slice_tuning = {"slice_height": int(S.value), "us_per_step": dict(zip((32, 64, 128, 256), us.tolist()))}
        return H
    _check(lib().gpuqt_build_h(ctypes.byref(d), stream, ctypes.byref(out)), "gpuqt_build_h")
    return Hamiltonian(out.value, None)


def gpuqt_build_h_tuned(*args, B: int = 1, **kw) -> Hamiltonian:
    """gpuqt_build_h with the slice height chosen by measurement at block width B."""
    kw["tune_block"] = int(B)
    return gpuqt_build_h(*args, **kw)


def gpuqt_build_h_from_model(m, energy_max=0.0, **kw) -> Hamiltonian:
    """gpuqt_build_h for an inputs.Model (neighbour list, hoppings, potentials, positions)."""
    return gpuqt_build_h(m.nn, m.nbr, m.hop, m.onsite, m.x, m.length_x, m.volume, energy_max,
                         hop_class=m.hop_class if m.n_class > 1 else None, n_class=m.n_class, **kw)


def gpuqt_workspace_size(H: Hamiltonian, op: int, B: int, M: int = 0, Np: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(lib().gpuqt_workspace_size(H.handle, op, B, M, Np, ctypes.byref(out)), "gpuqt_workspace_size")
    return int(out.value)


def _scratch(nbytes, like, stream):
    """A uint8 device buffer of nbytes on the device of `like`.  When the call runs on a stream
    other than torch's current one, the buffer is recorded on that stream, so the caching
    allocator does not hand its memory out again before the enqueued kernels have finished."""
    import torch
    ws = torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=like.device)
    if stream is not None:
        with torch.cuda.device(like.device):
            raw = _stream(stream)
            if raw != torch.cuda.current_stream().cuda_stream:
                ts = stream if isinstance(stream, torch.cuda.Stream) else \
                    torch.cuda.ExternalStream(raw, device=like.device)
                ws.record_stream(ts)
    return ws


def _workspace(H, op, B, M, Np, ws, like=None, stream=None):
    import torch
    need = gpuqt_workspace_size(H, op, B, M, Np)
    if ws is None:
        if like is None:
            like = torch.empty(0, device=torch.device("cuda", torch.cuda.current_device()))
        ws = _scratch(need, like, stream)
    return ws, int(ws.numel() * ws.element_size())


# --------------------------------------------------------------------------
# compute entry points
# --------------------------------------------------------------------------

def gpuqt_moments(H: Hamiltonian, phiL, phiR, M: int, mu=None, ws=None, stream=None):
    """mu[s, b, k] = <phiL_b|T_k(H/DeltaE_s)|phiR_b> (complex128 [n_seg, B, M] on the GPU)."""
    import torch
    _dev_vec(phiL, "phiL")
    _dev_vec(phiR, "phiR")
    B = _cols(phiR)
    if mu is None:
        mu = torch.empty((H.n_segments, B, M), dtype=torch.complex128, device=phiR.device)
    ws, nb = _workspace(H, OP_MOMENTS, B, M, 0, ws, phiR, stream)
    _check(lib().gpuqt_moments(H.handle, B, _ptr(phiL), _ptr(phiR), M, _ptr(mu), _ptr(ws), nb,
                               _stream(stream)), "gpuqt_moments")
    return mu


def gpuqt_moments_plain(H: Hamiltonian, phiL, phiR, M: int, mu=None, ws=None, stream=None):
    """gpuqt_moments by the one-moment-per-step recurrence (M - 1 sparse steps)."""
    import torch
    _dev_vec(phiL, "phiL")
    _dev_vec(phiR, "phiR")
    B = _cols(phiR)
    if mu is None:
        mu = torch.empty((H.n_segments, B, M), dtype=torch.complex128, device=phiR.device)
    ws, nb = _workspace(H, OP_MOMENTS, B, M, 0, ws, phiR, stream)
    _check(lib().gpuqt_moments_plain(H.handle, B, _ptr(phiL), _ptr(phiR), M, _ptr(mu), _ptr(ws), nb,
                                     _stream(stream)), "gpuqt_moments_plain")
    return mu


def gpuqt_moments_noalloc(H: Hamiltonian, phiL, phiR, M: int, mu, stream=None):
    """gpuqt_moments with the library's fixed per-GPU workspace: the C call allocates nothing
    (mu, complex128 [n_seg, B, M] on the GPU, must be given).  Calls that overlap on one GPU
    race; the workspace limit is gpuqt_noalloc_scratch_bytes()."""
    _dev_vec(phiL, "phiL")
    _dev_vec(phiR, "phiR")
    _check(lib().gpuqt_moments_noalloc(H.handle, _cols(phiR), _ptr(phiL), _ptr(phiR), int(M), _ptr(mu),
                                       _stream(stream)), "gpuqt_moments_noalloc")
    return mu


def gpuqt_noalloc_scratch_bytes() -> int:
    return int(lib().gpuqt_noalloc_scratch_bytes())


def gpuqt_evolve(H: Hamiltonian, psi, dt: float, Np: int = 0, psi_out=None, chi=None,
                 chi_out=None, with_commutator=False, ws=None, stream=None):
    """psi_out = U(dt) psi; with_commutator: also chi_out = [X,U(dt)] psi + U(dt) chi."""
    import torch
    _dev_vec(psi, "psi")
    B = _cols(psi)
    if psi_out is None:
        psi_out = torch.empty_like(psi)
    if with_commutator and chi_out is None:
        chi_out = torch.empty_like(psi)
    op = OP_EVOLVE_COMMUTATOR if chi_out is not None else OP_EVOLVE
    if Np == 0:
        Np_ws = max(gpuqt_auto_terms(e * abs(dt)) for e in H.energy_max)
    else:
        Np_ws = Np
    ws, nb = _workspace(H, op, B, 0, Np_ws, ws, psi, stream)
    _check(lib().gpuqt_evolve(H.handle, B, float(dt), Np, _ptr(psi), _ptr(psi_out), _ptr(chi),
                              _ptr(chi_out), _ptr(ws), nb, _stream(stream)), "gpuqt_evolve")
    return (psi_out, chi_out) if chi_out is not None else psi_out


def gpuqt_apply_commutator(H: Hamiltonian, psi, which: int = VELOCITY, out=None, stream=None):
    """out = V psi (which=VELOCITY) or [X,H] psi (which=COMMUTATOR_XH)."""
    import torch
    _dev_vec(psi, "psi")
    if out is None:
        out = torch.empty_like(psi)
    _check(lib().gpuqt_apply_commutator(H.handle, _cols(psi), which, _ptr(psi), _ptr(out),
                                        _stream(stream)), "gpuqt_apply_commutator")
    return out


def _series(fn, name, op, H, phi, dt, M, Np, out, ws, stream):
    import torch
    _dev_vec(phi, "phi")
    B = _cols(phi)
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    n_t = dt.shape[0]
    if out is None:
        out = torch.empty((n_t, H.n_segments, B, M), dtype=torch.float64, device=phi.device)
    if Np == 0:
        Np_ws = max([1] + [gpuqt_auto_terms(e * abs(t)) for e in H.energy_max for t in dt])
    else:
        Np_ws = Np
    ws, nb = _workspace(H, op, B, M, Np_ws, ws, phi, stream)
    _check(fn(H.handle, B, _ptr(phi), n_t, _ptr(dt), M, Np, _ptr(out), _ptr(ws), nb, _stream(stream)), name)
    return out


def gpuqt_vac(H: Hamiltonian, phi, dt: Sequence[float], M: int, Np: int = 0, out=None, ws=None,
              stream=None):
    """C^VAC rows [n_t, n_seg, B, M] (real, on the GPU); row k at t = dt[0] + ... + dt[k-1]."""
    return _series(lib().gpuqt_vac, "gpuqt_vac", OP_VAC, H, phi, dt, M, Np, out, ws, stream)


def gpuqt_msd(H: Hamiltonian, phi, dt: Sequence[float], M: int, Np: int = 0, out=None, ws=None,
              stream=None):
    """C^MSD rows [n_t, n_seg, B, M] (real, on the GPU); row k at t = dt[0] + ... + dt[k]."""
    return _series(lib().gpuqt_msd, "gpuqt_msd", OP_MSD, H, phi, dt, M, Np, out, ws, stream)


def gpuqt_kpm_reconstruct(C, energies, energy_max: float, volume: float, jackson=True,
                          out=None, stream=None):
    """KPM sum of the paper's Section 3.3 for moment rows C [R, M] (float64 on the GPU)."""
    import torch
    C = C.contiguous()
    if C.dim() == 1:
        C = C[None, :]
    R, M = int(C.shape[0]), int(C.shape[1])
    E = torch.as_tensor(np.asarray(energies, dtype=np.float64), device=C.device)
    if out is None:
        out = torch.empty((R, E.shape[0]), dtype=torch.float64, device=C.device)
    _check(lib().gpuqt_kpm_reconstruct(R, M, _ptr(C), int(E.shape[0]), _ptr(E), float(energy_max),
                                       float(volume), 1 if jackson else 0, _ptr(out), _stream(stream)),
           "gpuqt_kpm_reconstruct")
    return out


SIGMA_VAC, SIGMA_MSD = 0, 1


def gpuqt_transport_lengths(rho, vac0=None, sigma=None, msd=None, stream=None) -> dict:
    """Section 2.2 transport quantities per energy (float64 CUDA tensors): sigma_sc (max of the
    running conductivity rows), v = sqrt(C_vv(E, 0)), tau, mean free path, L(E, t) and xi(E),
    each returned when its inputs are given (rho [n_E]; vac0 [n_E] rho C_vv(t=0); sigma and msd
    [n_t, n_E])."""
    import torch
    rho = rho.contiguous()
    n_E = int(rho.shape[0])
    rows = sigma if sigma is not None else msd
    n_t = int(rows.shape[0]) if rows is not None else 0
    vac0 = None if vac0 is None else vac0.contiguous()
    sigma = None if sigma is None else sigma.contiguous()
    msd = None if msd is None else msd.contiguous()
    if sigma is not None and msd is not None and sigma.shape != msd.shape:
        raise ValueError("sigma and msd rows must have the same shape")
    new = lambda *shape: torch.empty(shape, dtype=torch.float64, device=rho.device)
    out = {}
    if sigma is not None:
        out["sigma_sc"] = new(n_E)
    if vac0 is not None:
        out["v"] = new(n_E)
        if sigma is not None:
            out["tau"], out["mfp"] = new(n_E), new(n_E)
    if msd is not None:
        out["L"], out["xi"] = new(n_t, n_E), new(n_E)
    g = lambda k: _ptr(out.get(k))
    _check(lib().gpuqt_transport_lengths(n_t, n_E, _ptr(rho), _ptr(vac0), _ptr(sigma), _ptr(msd),
                                         g("sigma_sc"), g("v"), g("tau"), g("mfp"), g("L"), g("xi"),
                                         _stream(stream)), "gpuqt_transport_lengths")
    return out


def gpuqt_running_conductivity(mode: int, rows, dt, out=None, stream=None):
    """Running conductivity over the time rows [N_t, n_E] (float64 on the GPU): SIGMA_VAC
    integrates rho C_vv rows, SIGMA_MSD differentiates rho DeltaX^2 rows (Section 2.2)."""
    import torch
    rows = rows.contiguous()
    n_t, n_E = int(rows.shape[0]), int(rows.shape[1])
    d = torch.as_tensor(np.asarray(dt, dtype=np.float64), device=rows.device)
    if d.shape[0] != n_t:
        raise ValueError("dt must have one entry per row")
    if out is None:
        out = torch.empty_like(rows)
    _check(lib().gpuqt_running_conductivity(int(mode), n_t, _ptr(d), n_E, _ptr(rows), _ptr(out),
                                            _stream(stream)), "gpuqt_running_conductivity")
    return out


KEEP_ALL_FRACTION = 0.25   # keep every forward vector when that needs at most this share of free memory


def gpuqt_moments_backward(H: Hamiltonian, phiL, phiR, w, grad_onsite=None, grad_class=None,
                           want_lam0=False, ckpt_stride=None, ws=None, stream=None, grad_hop=None):
    """Accumulate dL/dU (grad_onsite, float64 [n]), dL/ds_c (grad_class, float64 [n_class], s_c
    the class scales) and, with grad_hop (float64 [n, max_nn, 2]), (dL/dRe H_ij, dL/dIm H_ij) of
    every stored entry on its own, for L = sum w[s,b,k] Re mu[s,b,k]; returns
    (grad_onsite, grad_class, lam0 or None).

    ckpt_stride: 1 keeps every forward vector (no recomputation), >= 2 checkpoints every that
    many steps, 0 every ceil(sqrt(M)); None (default) takes 1 when its workspace fits in
    KEEP_ALL_FRACTION of the free device memory, else 0."""
    import torch
    _dev_vec(phiL, "phiL")
    _dev_vec(phiR, "phiR")
    B = _cols(phiR)
    w = w.contiguous()
    M = int(w.shape[-1])
    if ckpt_stride is None:
        if ws is not None:
            ckpt_stride = 0
        else:
            need = gpuqt_workspace_size(H, OP_MOMENTS_BACKWARD, B, M, 1)
            free, _ = torch.cuda.mem_get_info(phiR.device)
            ckpt_stride = 1 if need <= KEEP_ALL_FRACTION * free else 0
    if grad_onsite is None:
        grad_onsite = torch.zeros(H.n, dtype=torch.float64, device=phiR.device)
    lam0 = torch.empty_like(phiR) if want_lam0 else None
    ws, nb = _workspace(H, OP_MOMENTS_BACKWARD, B, M, ckpt_stride, ws, phiR, stream)
    _entry_grad_check(H, grad_hop)
    _check(lib().gpuqt_moments_backward(H.handle, B, _ptr(phiL), _ptr(phiR), M, _ptr(w),
                                        _ptr(grad_onsite), _ptr(grad_class), _ptr(grad_hop), _ptr(lam0),
                                        ckpt_stride, _ptr(ws), nb, _stream(stream)), "gpuqt_moments_backward")
    return grad_onsite, grad_class, lam0


def gpuqt_vac_backward_workspace_size(H: Hamiltonian, B: int, dt, M: int, Np: int = 0,
                                      ckpt_stride: int = 0, time_stride: int = 1) -> int:
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    out = ctypes.c_size_t()
    _check(lib().gpuqt_vac_backward_workspace_size(H.handle, B, dt.shape[0], _ptr(dt), M, Np, int(ckpt_stride),
                                                   int(time_stride), ctypes.byref(out)),
           "gpuqt_vac_backward_workspace_size")
    return int(out.value)


def gpuqt_vac_tape_size(H: Hamiltonian, B: int, dt, M: int, Np: int = 0) -> int:
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    out = ctypes.c_size_t()
    _check(lib().gpuqt_vac_tape_size(H.handle, B, dt.shape[0], _ptr(dt), int(M), int(Np), ctypes.byref(out)),
           "gpuqt_vac_tape_size")
    return int(out.value)


def gpuqt_vac_record(H: Hamiltonian, phi, dt: Sequence[float], M: int, Np: int = 0, tape=None, out=None,
                     ws=None, stream=None):
    """gpuqt_vac that also keeps the states and moment chains in `tape` (a uint8 CUDA tensor of
    at least gpuqt_vac_tape_size bytes; allocated when None).  Returns (rows, tape)."""
    import torch
    _dev_vec(phi, "phi")
    B = _cols(phi)
    dtn = np.ascontiguousarray(dt, dtype=np.float64)
    if tape is None:
        tape = torch.empty(max(gpuqt_vac_tape_size(H, B, dtn, M, Np), 16), dtype=torch.uint8,
                           device=phi.device)
    tb = int(tape.numel() * tape.element_size())
    fn = lambda h, b, p, n, d, m, npp, o, w_, nb, st: lib().gpuqt_vac_record(h, b, p, n, d, m, npp, o, w_, nb,
                                                                           _ptr(tape), tb, st)
    rows = _series(fn, "gpuqt_vac_record", OP_VAC, H, phi, dtn, M, Np, out, ws, stream)
    return rows, tape


def gpuqt_vac_backward_tape_workspace_size(H: Hamiltonian, B: int, dt, M: int, Np: int = 0) -> int:
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    out = ctypes.c_size_t()
    _check(lib().gpuqt_vac_backward_tape_workspace_size(H.handle, B, dt.shape[0], _ptr(dt), M, Np,
                                                        ctypes.byref(out)), "gpuqt_vac_backward_tape_workspace_size")
    return int(out.value)


def gpuqt_vac_backward_tape(H: Hamiltonian, phi, dt, w, tape, grad_onsite=None, grad_class=None, Np: int = 0,
                            ws=None, stream=None):
    """gpuqt_vac_backward from the tape of gpuqt_vac_record (same phi, dt, M, Np): no state
    re-evolution and no forward pass of the rows' moments."""
    import torch
    _dev_vec(phi, "phi")
    B = _cols(phi)
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    w = w.contiguous()
    M = int(w.shape[-1])
    if grad_onsite is None:
        grad_onsite = torch.zeros(H.n, dtype=torch.float64, device=phi.device)
    if ws is None:
        ws = _scratch(gpuqt_vac_backward_tape_workspace_size(H, B, dt, M, Np), phi, stream)
    nb = int(ws.numel() * ws.element_size())
    tb = int(tape.numel() * tape.element_size())
    _check(lib().gpuqt_vac_backward_tape(H.handle, B, _ptr(phi), dt.shape[0], _ptr(dt), M, Np, _ptr(w),
                                         _ptr(grad_onsite), _ptr(grad_class), _ptr(tape), tb, _ptr(ws), nb,
                                         _stream(stream)),
           "gpuqt_vac_backward_tape")
    return grad_onsite, grad_class


def gpuqt_vac_backward(H: Hamiltonian, phi, dt, w, grad_onsite=None, grad_class=None, Np: int = 0,
                       ckpt_stride=None, time_stride=None, ws=None, stream=None, grad_hop=None):
    """Accumulate dL/dU, dL/ds_c and (grad_hop, float64 [n, max_nn, 2]) the per-entry hopping
    gradients for L = sum w[k,s,b,n] C^VAC rows (w float64 [n_t,n_seg,B,M]).

    ckpt_stride: 1 keeps every forward vector (two-chain reverse of each row's moments), 0
    recomputes from checkpoints; None (default) takes 1 when its workspace fits in
    KEEP_ALL_FRACTION of the free device memory (or 0 when ws is given).
    time_stride: 1 keeps every state psi_{L,R}(t_k), s >= 2 only every s-th (segments are
    re-evolved in the reverse), 0 every ceil(sqrt(n_t))-th; None (default) takes 1 when the
    workspace with every state fits in KEEP_ALL_FRACTION of the free memory (or 1 when ws is
    given), else 0."""
    import torch
    _dev_vec(phi, "phi")
    B = _cols(phi)
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    w = w.contiguous()
    M = int(w.shape[-1])
    free = None
    if time_stride is None:
        if ws is not None:
            time_stride = 1
        else:
            need = gpuqt_vac_backward_workspace_size(H, B, dt, M, Np, 0, 1)
            free, _ = torch.cuda.mem_get_info(phi.device)
            time_stride = 1 if need <= KEEP_ALL_FRACTION * free else 0
    if ckpt_stride is None:
        if ws is not None:
            ckpt_stride = 0
        else:
            need = gpuqt_vac_backward_workspace_size(H, B, dt, M, Np, 1, time_stride)
            if free is None:
                free, _ = torch.cuda.mem_get_info(phi.device)
            ckpt_stride = 1 if need <= KEEP_ALL_FRACTION * free else 0
    if grad_onsite is None:
        grad_onsite = torch.zeros(H.n, dtype=torch.float64, device=phi.device)
    if ws is None:
        ws = _scratch(gpuqt_vac_backward_workspace_size(H, B, dt, M, Np, ckpt_stride, time_stride), phi, stream)
    nb = int(ws.numel() * ws.element_size())
    _entry_grad_check(H, grad_hop)
    _check(lib().gpuqt_vac_backward(H.handle, B, _ptr(phi), dt.shape[0], _ptr(dt), M, Np, _ptr(w),
                                    _ptr(grad_onsite), _ptr(grad_class), _ptr(grad_hop), int(ckpt_stride),
                                    int(time_stride), _ptr(ws), nb, _stream(stream)),
           "gpuqt_vac_backward")
    return grad_onsite, grad_class


def _entry_grad_check(H: Hamiltonian, g):
    if g is None:
        return
    import torch
    shape = (H.n, int(H.info.max_nn), 2)
    if not (isinstance(g, torch.Tensor) and g.is_cuda and g.dtype == torch.float64 and g.is_contiguous()
            and tuple(g.shape) == shape):
        raise ValueError(f"per-entry gradients must be a contiguous float64 CUDA tensor of shape {shape}")


def gpuqt_tie_entry_gradient(H: Hamiltonian, untied, out=None, stream=None):
    """Hermitian tie of per-entry gradients [n, max_nn, 2]: each bond's gradient with respect to
    (Re h, Im h), h = H_ij = conj(H_ji), stored at both of its entries (the partner as (re, -im))."""
    import torch
    _entry_grad_check(H, untied)
    if out is None:
        out = torch.empty_like(untied)
    _entry_grad_check(H, out)
    _check(lib().gpuqt_tie_entry_gradient(H.handle, _ptr(untied), _ptr(out), _stream(stream)),
           "gpuqt_tie_entry_gradient")
    return out


def gpuqt_kpm_reconstruct_adjoint(g, energies, M: int, energy_max: float, volume: float,
                                  jackson=True, out=None, stream=None):
    """Transpose of gpuqt_kpm_reconstruct: g [R, n_E] (float64 on the GPU) -> [R, M]."""
    import torch
    g = g.contiguous()
    if g.dim() == 1:
        g = g[None, :]
    R = int(g.shape[0])
    E = torch.as_tensor(np.asarray(energies, dtype=np.float64), device=g.device)
    if out is None:
        out = torch.empty((R, M), dtype=torch.float64, device=g.device)
    _check(lib().gpuqt_kpm_reconstruct_adjoint(R, M, _ptr(g), int(E.shape[0]), _ptr(E), float(energy_max),
                                               float(volume), 1 if jackson else 0, _ptr(out),
                                               _stream(stream)), "gpuqt_kpm_reconstruct_adjoint")
    return out


K_FAMILIES = ("moment", "moment_sym", "moment_pair", "evolve", "msd", "evolve_pair")


def gpuqt_set_timing(H: Hamiltonian, enable: bool = True):
    _check(lib().gpuqt_set_timing(H.handle, 1 if enable else 0), "gpuqt_set_timing")


def gpuqt_timing(H: Hamiltonian) -> dict:
    """{family: (total ms, launches)} of the runs recorded since the last call."""
    ms = np.zeros(len(K_FAMILIES))
    n = np.zeros(len(K_FAMILIES), dtype=np.int64)
    _check(lib().gpuqt_timing(H.handle, _ptr(ms), _ptr(n)), "gpuqt_timing")
    return {f: (float(ms[i]), int(n[i])) for i, f in enumerate(K_FAMILIES)}


def gpuqt_update_h_values(H: Hamiltonian, onsite=None, class_scale=None, stream=None):
    """New on-site energies (float64 CUDA tensor [n]) and/or hopping-class scales (host sequence)."""
    cs = None if class_scale is None else np.ascontiguousarray(class_scale, dtype=np.float64)
    if onsite is not None:
        import torch
        if onsite.dtype != torch.float64 or not onsite.is_cuda or not onsite.is_contiguous():
            raise TypeError("onsite must be a contiguous float64 CUDA tensor")
    _check(lib().gpuqt_update_h_values(H.handle, _ptr(onsite), _ptr(cs), _stream(stream)),
           "gpuqt_update_h_values")


def gpuqt_autotune(H: Hamiltonian, B: int = 1, ws=None, stream=None):
    """Time the kernel variants (plain / non-temporal loads, plain / banded / pencil row order,
    each uncapped and at per-CU workgroup caps below its occupancy limit), keep the fastest;
    returns us per moment step of load variants 0..3, of the pencil order with plain and
    non-temporal loads (entries 4, 5) at their best cap, and of the periodic-box stencil
    (entry 6, at the chosen cap; blocks of B >= 2 on a periodic box), 0 where a variant does
    not exist.
    H.info.kernel_variant: bits 0-1 the load variant, bits 2-5 the cap (0: none), bit 6 the
    pencil order, from bit 8 the two-chain moment, MSD and two-vector evolution families'
    own caps."""
    t = np.zeros(7)
    ws, nb = _workspace(H, OP_AUTOTUNE, B, 0, 0, ws)
    _check(lib().gpuqt_autotune(H.handle, B, _ptr(ws), nb, _stream(stream), _ptr(t)), "gpuqt_autotune")
    info = HInfo()
    _check(lib().gpuqt_h_info(H.handle, ctypes.byref(info), None, None), "gpuqt_h_info")
    H.info = info
    return t


def gpuqt_set_variant(H: Hamiltonian, variant: int):
    """Pin the kernel variant code (bit 0: non-temporal streams, bit 1: banded row order,
    bits 2-5: resident workgroups per CU at most, 0 = no cap; bit 6 (with bit 1): the pencil
    order instead of the banded one; bit 7: the evolution and MSD terms on the other load
    variant; bit 26: the periodic-box Hermitian step (blocks of B >= 2), bit 27: the
    periodic-box MSD term; from bit 8, 3 bits per kernel
    family: 0 = that cap, 1 + c = the family's own cap c).  H.info.kernel_variant after
    gpuqt_autotune is such a code."""
    _check(lib().gpuqt_set_variant(H.handle, int(variant)), "gpuqt_set_variant")
    info = HInfo()
    _check(lib().gpuqt_h_info(H.handle, ctypes.byref(info), None, None), "gpuqt_h_info")
    H.info = info


def _refresh_info(H: Hamiltonian):
    info = HInfo()
    _check(lib().gpuqt_h_info(H.handle, ctypes.byref(info), None, None), "gpuqt_h_info")
    H.info = info


def gpuqt_tune_cache_key(H: Hamiltonian, B: int) -> str:
    """The configuration key under which variants for H at block width B are cached."""
    buf = ctypes.create_string_buffer(256)
    _check(lib().gpuqt_tune_cache_key(H.handle, int(B), buf, 256), "gpuqt_tune_cache_key")
    return buf.value.decode()


def gpuqt_autotune_cached(H: Hamiltonian, B: int = 1, ws=None, stream=None):
    """The cached variant for H's configuration at B, or gpuqt_autotune (then cached).  The
    autotuning workspace is only allocated on a miss.  Returns (times per load variant,
    whether the choice came from the cache)."""
    t = np.zeros(7)
    hit = ctypes.c_int32()
    if ws is None:
        st = lib().gpuqt_autotune_cached(H.handle, int(B), None, 0, _stream(stream), _ptr(t), ctypes.byref(hit))
        if st == GPUQT_ERR_WORKSPACE:
            ws, _ = _workspace(H, OP_AUTOTUNE, B, 0, 0, None, None, stream)
        else:
            _check(st, "gpuqt_autotune_cached")
            _refresh_info(H)
            return t, bool(hit.value)
    nb = int(ws.numel() * ws.element_size())
    _check(lib().gpuqt_autotune_cached(H.handle, int(B), _ptr(ws), nb, _stream(stream), _ptr(t),
                                       ctypes.byref(hit)), "gpuqt_autotune_cached")
    _refresh_info(H)
    return t, bool(hit.value)


def gpuqt_tune_cache_load(path):
    _check(lib().gpuqt_tune_cache_load(os.fsencode(str(path))), "gpuqt_tune_cache_load")


def gpuqt_tune_cache_save(path):
    _check(lib().gpuqt_tune_cache_save(os.fsencode(str(path))), "gpuqt_tune_cache_save")


def gpuqt_tune_cache_clear():
    lib().gpuqt_tune_cache_clear()


def gpuqt_autotune_block(H: Hamiltonian, n_vectors: int, max_B: int = 16, ws=None, stream=None):
    """Block width for n_vectors random vectors by measurement: (best B, microseconds per vector
    and Hermitian moment step for B = 1, 2, 4, 8, 16; 0 where not tried).  The workspace (the
    autotuning workspace of the widest block tried, max_B) bounds the widths tried."""
    B = 1
    while B * 2 <= min(max_B, n_vectors, 16):
        B *= 2
    ws, nb = _workspace(H, OP_AUTOTUNE, B, 0, 0, ws, None, stream)
    best = ctypes.c_int32()
    us = np.zeros(5)
    _check(lib().gpuqt_autotune_block(H.handle, int(n_vectors), _ptr(ws), nb, _stream(stream), ctypes.byref(best),
                                      _ptr(us)), "gpuqt_autotune_block")
    _refresh_info(H)
    return int(best.value), us


def gpuqt_schedule_rows(seg_offsets, period=None, band_rows=0, cus=256, B=1, pencil=False):
    """Host-only: (workgroup, iteration) visiting each row under the library's row schedule
    (pencil: the pencil order of band width band_rows for segments with a period >= 128)."""
    off = np.ascontiguousarray(seg_offsets, dtype=np.int64)
    per = None if period is None else np.ascontiguousarray(period, dtype=np.int64)
    n = int(off[-1])
    blk = np.empty(n, dtype=np.int32)
    it = np.empty(n, dtype=np.int32)
    _check(lib().gpuqt_schedule_rows(len(off) - 1, _ptr(off), _ptr(per), int(band_rows), 1 if pencil else 0,
                                     int(cus), int(B), _ptr(blk), _ptr(it)), "gpuqt_schedule_rows")
    return blk, it


class InputFolder:
    """An input folder of the paper's program (Section 4.2), read by the library's reader:
    the model arrays (nn, nbr, hop, onsite, x, length_x, volume) and the run parameters."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def gpuqt_model_load(path) -> InputFolder:
    """Read neighbour.in, hopping.in, potential.in, position.in, energy.in, time_step.in and
    para.in from a folder (host only); returns copies of the arrays."""
    h = ctypes.c_void_p()
    _check(lib().gpuqt_model_load(os.fsencode(str(path)), ctypes.byref(h)), "gpuqt_model_load")
    try:
        d = _Desc()
        _check(lib().gpuqt_model_desc(h, ctypes.byref(d)), "gpuqt_model_desc")
        p = ModelParams()
        _check(lib().gpuqt_model_params(h, ctypes.byref(p)), "gpuqt_model_params")
        n, k = int(d.n), int(d.max_nn)

        def arr(ptr, count, ctype):
            if not ptr or count == 0:
                return None
            return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctype)), shape=(count,)).copy()

        hop = None
        if d.hop:
            raw = arr(d.hop, n * k * (2 if d.hop_is_complex else 1), ctypes.c_double)
            hop = raw.view(np.complex128).reshape(n, k) if d.hop_is_complex else raw.reshape(n, k)
        nbr = arr(d.nbr, n * k, ctypes.c_int32)
        return InputFolder(
            n=n, max_nn=k, nn=arr(d.nn, n, ctypes.c_int32),
            nbr=nbr.reshape(n, k) if nbr is not None else np.zeros((n, 0), np.int32), hop=hop,
            onsite=arr(d.onsite, n, ctypes.c_double), x=arr(d.x, n, ctypes.c_double),
            length_x=float(d.length_x), volume=float(d.volume), energy_max=float(p.energy_max),
            n_random_vectors=int(p.n_random_vectors), n_moments=int(p.n_moments),
            calculate_vac=bool(p.calculate_vac), calculate_msd=bool(p.calculate_msd),
            energies=arr(p.energies, p.n_energies, ctypes.c_double),
            time_steps=arr(p.time_steps, p.n_time_steps, ctypes.c_double))
    finally:
        lib().gpuqt_model_free(h)


def gpuqt_copy_probe(src, dst, stream=None):
    nbytes = src.numel() * src.element_size()
    _check(lib().gpuqt_copy_probe(_ptr(src), _ptr(dst), nbytes, _stream(stream)), "gpuqt_copy_probe")
    return dst
