"""CPU tests of the C ABI: the library loads, exports every declared symbol,
its host helpers agree with independent routines, and descriptor validation
rejects malformed models before touching any device."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.special

import paper_1705_01387_amd as P
from paper_1705_01387_amd import inputs as I
from paper_1705_01387_amd import _binding as Bd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "gpuqt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gpuqt_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(P.LIB_PATH)
    syms = declared_symbols()
    assert "gpuqt_moments" in syms and "gpuqt_msd" in syms and "gpuqt_build_h" in syms
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    # every declared symbol has a binding of the same name (handle lifetime and the model
    # accessors are used inside Hamiltonian and gpuqt_model_load)
    inside = ("gpuqt_destroy_h", "gpuqt_h_info", "gpuqt_model_desc", "gpuqt_model_params", "gpuqt_model_free")
    for s in syms:
        assert hasattr(P, s) or s in inside, s


def test_bessel_matches_high_precision():
    """Miller recurrence vs 40-digit mpmath (scipy's jv itself errs by ~1e-14 at tau = 1000)."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    for tau in (0.0, 1e-3, 0.5, 3.7, 36.36, 209.46, 1000.0):
        Np = max(P.gpuqt_auto_terms(tau) + 5, 8)
        J = P.gpuqt_bessel(tau, Np)
        ref = np.array([float(mp.besselj(m, tau)) for m in range(Np)])
        assert np.max(np.abs(J - ref)) < 1e-15, tau
        if tau < 300:
            assert np.max(np.abs(J - scipy.special.jv(np.arange(Np), tau))) < 5e-15


def test_auto_terms_rule():
    for tau in (0.0, 0.3, 4.5, 22.0, 209.46, 1500.0):
        Np = P.gpuqt_auto_terms(tau)
        assert Np > tau
        assert abs(scipy.special.jv(Np, tau)) < 1.2e-16
        if Np - 1 > tau:
            assert abs(scipy.special.jv(Np - 1, tau)) >= 0.8e-16
    assert P.gpuqt_auto_terms(-1.0) == -1


def test_jackson_matches_definition_values():
    g = P.gpuqt_jackson(1000)
    assert abs(g[0] - 1) < 1e-15
    a = 1 / 1001
    n = np.arange(1000)
    ref = (1 - n * a) * np.cos(np.pi * n * a) + a * np.sin(np.pi * n * a) / np.tan(np.pi * a)
    assert np.max(np.abs(g - ref)) < 1e-14


def _desc_call(**kw):
    m = I.square(6, 5, W=1.0, seed=1)
    args = dict(nn=m.nn, nbr=m.nbr, hop=m.hop, onsite=m.onsite, x=m.x, length_x=m.length_x,
                volume=m.volume, energy_max=0.0)
    args.update(kw)
    return P.gpuqt_build_h(**args)


def _status(fn):
    with pytest.raises(P.GpuqtError) as e:
        fn()
    return e.value.status


def test_validation_errors_before_device():
    m = I.square(6, 5, W=1.0, seed=1)
    bad = m.nbr.copy()
    bad[3, 1] = 30
    assert _status(lambda: _desc_call(nbr=bad)) == 2                       # index out of range
    nn = m.nn.copy()
    nn[0] = 9
    assert _status(lambda: _desc_call(nn=nn)) == 2                         # count > max_nn
    assert _status(lambda: _desc_call(energy_max=2.0)) == 3                # below Gershgorin
    h = np.full(m.nbr.shape, -1.0 + 0j)
    h[0, 0] = -1.0 + 0.5j                                                  # no conjugate partner
    assert _status(lambda: _desc_call(hop=h, check_hermitian=True)) == 2
    m2 = I.chain(4)                                                        # |dx| = L/2
    assert _status(lambda: P.gpuqt_build_h(m2.nn, I.chain(4).nbr, None, None,
                                           np.array([0., 1., 2., 3.]), 2.0, 4.0)) == 2
    seg = np.array([0, 15, 30])                                            # bond across segments
    assert _status(lambda: _desc_call(seg_offsets=seg)) == 2
    assert _status(lambda: _desc_call(slice_height=48)) == 1


def test_ctypes_mirrors_match_the_header(tmp_path):
    """Field offsets of the binding's struct mirrors equal what a C compiler gives for the header."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gpuqt.h"', 'int main(void){']
    for cname, mirror in (("gpuqt_h_desc", Bd._Desc), ("gpuqt_h_info_t", Bd.HInfo),
                          ("gpuqt_model_params_t", Bd.ModelParams)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in mirror._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "abi"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for ln in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, f, v = ln.split()
        got[(cname, f)] = int(v)
    for cname, mirror in (("gpuqt_h_desc", Bd._Desc), ("gpuqt_h_info_t", Bd.HInfo),
                          ("gpuqt_model_params_t", Bd.ModelParams)):
        assert got[(cname, "size")] == ctypes.sizeof(mirror)
        for f, _ in mirror._fields_:
            assert got[(cname, f)] == getattr(mirror, f).offset, (cname, f)


def test_tune_cache_file_format(tmp_path):
    """The tuning cache file: '<key>TAB<code>' lines and '#' comments; a missing file is an
    argument error, a malformed line a layout error naming file:line with nothing merged,
    and a saved cache reloads to the same entries."""
    P.lib()
    try:
        P.gpuqt_tune_cache_clear()
        with pytest.raises(P.GpuqtError) as e:
            P.gpuqt_tune_cache_load(tmp_path / "missing.tsv")
        assert e.value.status == 1
        bad = tmp_path / "bad.tsv"
        bad.write_text("# comment\ngfx950 n10 K4 B1\t12\ngfx950 n11 K4 B1 no-code\n")
        with pytest.raises(P.GpuqtError) as e:
            P.gpuqt_tune_cache_load(bad)
        assert e.value.status == 2 and "bad.tsv:3" in str(e.value)
        empty = tmp_path / "empty.tsv"
        P.gpuqt_tune_cache_save(empty)
        assert [ln for ln in empty.read_text().splitlines() if not ln.startswith("#")] == []
        good = tmp_path / "good.tsv"
        good.write_text("# comment\ngfx950 n10 K4 w4 S64 h0 s1 p5 m0 B1\t12\ngfx950 n11 K4 w4 S64 h0 s1 p5 m0 B2\t77\n")
        P.gpuqt_tune_cache_load(good)
        out = tmp_path / "out.tsv"
        P.gpuqt_tune_cache_save(out)
        lines = [ln for ln in out.read_text().splitlines() if not ln.startswith("#")]
        assert lines == ["gfx950 n10 K4 w4 S64 h0 s1 p5 m0 B1\t12", "gfx950 n11 K4 w4 S64 h0 s1 p5 m0 B2\t77"]
    finally:
        P.gpuqt_tune_cache_clear()
        P.gpuqt_tune_cache_load(P.TUNE_CACHE_PATH)


def test_committed_tune_cache_is_well_formed():
    """The package's cache of MI355X choices: every line a gfx950 key and a variant code that
    gpuqt_set_variant accepts (load variant, a per-CU cap of at most 8, the pencil bit, family
    caps)."""
    lines = [ln for ln in open(P.TUNE_CACHE_PATH).read().splitlines() if ln and not ln.startswith("#")]
    assert lines
    for ln in lines:
        key, code = ln.split("\t")
        code = int(code)
        assert key.startswith("gfx950 ") and key.split()[-1].startswith("B")
        assert ((code >> 2) & 15) <= 8 and code >> 28 == 0
        assert not (code >> 6) & 1 or (code >> 1) & 1          # the pencil bit only with the banded bit
