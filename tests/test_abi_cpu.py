"""The C-ABI library loads, exports every declared symbol and rejects bad
arguments on the host (no compute call, no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1708_07045_amd as fd
from paper_1708_07045_amd._lib import GridDesc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fftdg.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fftdg_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = fd.load()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(fd.EXPORTS) <= set(names)


def test_version_and_status_strings():
    L = fd.load()
    assert L.fftdg_version() == 10000
    for code in (0, -1, -2, -3, -4, -5):
        assert L.fftdg_status_string(code)
    assert L.fftdg_status_string(-99) == b"unknown status"


def _desc(**kw):
    d = dict(n_rec=96, n_fft=128, h=0.25, origin=(0.0, 0.0, 0.0), precision=fd.F32, clash_mode=fd.OCC,
             ljr_cap=10.0, occ_f=0.5)
    d.update(kw)
    return GridDesc(d["n_rec"], d["n_fft"], d["h"], (ctypes.c_double * 3)(*d["origin"]), d["precision"],
                    d["clash_mode"], d["ljr_cap"], d["occ_f"])


@pytest.mark.parametrize("kw", [
    dict(n_fft=96),                      # unsupported FFT edge
    dict(n_fft=512),                     # beyond the largest built size
    dict(precision=fd.F64, n_fft=256),   # 256 is FP32 only
    dict(n_rec=300, n_fft=256),          # n_rec > n_fft
    dict(precision=fd.F64, n_fft=128),   # FP64 limited to 32/64
    dict(n_rec=200),                     # n_rec > n_fft
    dict(n_rec=2),
    dict(h=0.0),
    dict(h=float("nan")),
    dict(origin=(0.0, float("inf"), 0.0)),
    dict(precision=7),
    dict(clash_mode=9),
    dict(clash_mode=fd.CAP, ljr_cap=-1.0),
    dict(occ_f=0.0),
])
def test_create_rejects_bad_descriptions(kw):
    L = fd.load()
    h = ctypes.c_void_p()
    g = _desc(**kw)
    assert L.fftdg_create(ctypes.byref(h), ctypes.byref(g), 0, None) == fd._lib.E_INVALID
    assert not h.value


def test_grid_tools_reject_bad_arguments_without_a_device():
    L = fd.load()
    g = _desc(n_rec=1)
    assert L.fftdg_grids_build(0, None, ctypes.byref(g), 10, None, None, None, None, None, None) == fd._lib.E_INVALID
    assert L.fftdg_grid_energies(0, None, None, None, 1, 1, None, None, None, None, None) == fd._lib.E_INVALID
    assert L.fftdg_pair_energies(0, None, 0, None, None, None, None, 1, 1, None, None, None, None, 0,
                                 None) == fd._lib.E_INVALID


def test_create_null_arguments():
    L = fd.load()
    h = ctypes.c_void_p()
    assert L.fftdg_create(None, ctypes.byref(_desc()), 0, None) == fd._lib.E_INVALID
    assert L.fftdg_create(ctypes.byref(h), None, 0, None) == fd._lib.E_INVALID


def test_create_without_device_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    L = fd.load()
    h = ctypes.c_void_p()
    assert L.fftdg_create(ctypes.byref(h), ctypes.byref(_desc()), 0, None) == fd._lib.E_DEVICE


def test_calls_with_null_context():
    L = fd.load()
    assert L.fftdg_scan(None, None, 300.0, None) == fd._lib.E_INVALID
    assert L.fftdg_reduce(None, None, None, None, 300.0, None, None) == fd._lib.E_INVALID
    assert L.fftdg_set_receptors(None, 1, None, None, None) == fd._lib.E_INVALID
    assert L.fftdg_last_error(None) == b"context is NULL"
    L.fftdg_destroy(None)


def test_batch_offsets_and_select_length():
    """The binding lays a batch out as CSR offsets over ligands and takes a
    selection only with one byte per configuration (the library reads that
    many)."""
    import numpy as np
    import paper_1708_07045_amd as fd
    from workload import synth
    rng = np.random.default_rng(3)
    ligs = [synth.make_ligand(rng, rng, na, nc, nr) for na, nc, nr in ((3, 2, 4), (5, 1, 0), (2, 3, 1))]
    b = fd.Batch(ligs)
    np.testing.assert_array_equal(b.atom_off, [0, 3, 8, 10])
    np.testing.assert_array_equal(b.conf_off, [0, 2, 3, 6])
    np.testing.assert_array_equal(b.cfg_off, [0, 8, 8, 11])
    assert b.n_cfg == 11 and b.conf_xyz.shape == (3 * 2 + 5 + 2 * 3, 3)
    assert b.with_select(np.ones(11, np.uint8)).select.size == 11
    for bad in (np.ones(10, np.uint8), np.ones(12, np.uint8)):
        with pytest.raises(ValueError):
            fd.Batch(ligs, bad)
        with pytest.raises(ValueError):
            b.with_select(bad)


def test_partials_buffer_check():
    """Calls that hand partials to the library first check that the buffer
    is a contiguous tensor on the context's device holding n_snap * n_cfg
    records (checked here with a stand-in context on the CPU device)."""
    import types
    import numpy as np
    import torch
    import paper_1708_07045_amd as fd
    from workload import synth
    rng = np.random.default_rng(4)
    b = fd.Batch([synth.make_ligand(rng, rng, 3, 2, 5)])             # 10 configurations
    ctx = types.SimpleNamespace(torch=torch, n_snap=3, device=torch.device("cpu"))
    need = 3 * 10 * fd.PARTIAL_DTYPE.itemsize
    ok = torch.empty(need, dtype=torch.uint8)
    assert fd.FFTDG._partials_ok(ctx, ok, b) is ok
    assert fd.FFTDG._partials_ok(ctx, torch.empty(need // 8, dtype=torch.float64), b) is not None
    for bad in (torch.empty(need - 1, dtype=torch.uint8), np.zeros(need, np.uint8),
                torch.empty(2 * need, dtype=torch.uint8)[::2]):
        with pytest.raises(ValueError):
            fd.FFTDG._partials_ok(ctx, bad, b)
