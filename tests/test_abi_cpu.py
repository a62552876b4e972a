"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments on the host before any device
work (these run without a GPU)."""
import ctypes as C
import dataclasses
import os
import re

import numpy as np
import pytest

from paper_2307_08006_amd import labf, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    from paper_2307_08006_amd import build
    if build.is_stale():
        build.build(force=True)


def _declared():
    txt = open(os.path.join(ROOT, "include", "labf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(labf_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = labf.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(labf.EXPORTS) == names


def _pme_dims(spec, dims, order=4, beta=0.3):
    """Smooth PME on with the given grid (rejected before any device work
    when the grid, the order or beta is out of range)."""
    spec.pme_order, spec.ewald_beta = order, beta
    spec.pme_dims = np.array([dims], np.int32)


def _spec():
    spec, lam = synth.lj_reduced(n_atoms=125, density=0.5, r_cut=2.0, r_skin=0.2)
    return spec, lam


@pytest.mark.parametrize("mutate,msg", [
    (lambda s: setattr(s, "r_cut", 10.0), "L/2"),
    (lambda s: setattr(s, "dt", 0.0), "out of range"),
    (lambda s: s.mass.__setitem__(3, 0.0), "mass"),
    (lambda s: s.epsilon.__setitem__(3, -1.0), "epsilon"),
    (lambda s: s.pos.__setitem__((2, 1), np.nan), "position"),
    (lambda s: setattr(s, "atom_offset", np.array([0, 0, 125], np.int64)), "at least one atom"),
    (lambda s: setattr(s, "anchor", np.zeros((125, 3))), "together"),
    (lambda s: setattr(s, "rebuild_interval", 0), "rebuild_interval"),
    (lambda s: setattr(s, "r_skin_alch", 0.1), "r_skin_alch"),
    (lambda s: setattr(s, "r_skin_alch", 1.5), "L/2"),
    (lambda s: setattr(s, "column_width", np.array([0.3])), "column_width"),
    (lambda s: setattr(s, "precision", "fp16"), None),
    (lambda s: _pme_dims(s, [0, 16, 16]), "pme_dims"),
    (lambda s: _pme_dims(s, [16, 28, 16]), "pme_dims"),
    (lambda s: _pme_dims(s, [16, 16, 20]), "pme_dims"),
    (lambda s: _pme_dims(s, [264, 16, 16]), "pme_dims"),
    (lambda s: _pme_dims(s, [16, 16, 8]), "pme_dims"),
    (lambda s: _pme_dims(s, [16, 16, 16], order=5), "pme_order"),
    (lambda s: _pme_dims(s, [16, 16, 16], beta=0.0), "ewald_beta"),
])
def test_invalid_descriptor_is_rejected_on_host(mutate, msg):
    _ensure_built()
    spec, lam = _spec()
    if mutate is not None:
        mutate(spec)
    if spec.precision == "fp16":
        # the binding maps unknown precisions to FP32; check the raw ABI instead
        d = labf.SystemDesc()
        d.n_walkers, d.precision = 1, 7
        h = C.c_void_p()
        assert labf.lib().labf_create_system(C.byref(d), None, C.byref(h)) == -1
        assert h.value is None
        return
    with pytest.raises(labf.LabfError) as ei:
        labf.System(spec)
    assert ei.value.code == -1
    assert msg in str(ei.value)


def test_null_arguments_are_rejected():
    _ensure_built()
    L = labf.lib()
    assert L.labf_create_system(None, None, None) == -1
    h = C.c_void_p()
    assert L.labf_create_system(None, None, C.byref(h)) == -1
    assert L.labf_step_walkers(None, 1, 0, None) == -1
    assert L.labf_energy_forward(None, None, None, None, None, None, None) == -1
    assert L.labf_workspace_size(None, None) == -1
    assert L.labf_energy_backward(None, None, None, None, None, None, None, None, None) == -1
    assert L.labf_read_atoms(None, None, None, None) == -1
    assert L.labf_philox(-1, None, None, None, None) == -1
    assert L.labf_philox(0, None, None, None, None) == 0
    L.labf_destroy_system(None)
    assert b"NULL" in L.labf_last_error(None) or L.labf_last_error(None) is not None


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(labf, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(labf, "_lib", None)
    with pytest.raises(labf.LabfError):
        labf.lib()


def test_probe_rejects_bad_arguments_without_a_gpu():
    _ensure_built()
    L = labf.lib()
    rate = np.zeros(1)
    p = rate.ctypes.data
    assert L.labf_probe(7, 16, p, None) == -1              # unknown kind
    assert L.labf_probe(0, 0, p, None) == -1               # no iterations
    assert L.labf_probe(3, 6, p, None) == -1               # triad size not a multiple of 4
    assert L.labf_probe(3, (1 << 30) + 4, p, None) == -1   # triad too large
    assert L.labf_probe(0, 16, None, None) == -1           # no output


def _raw_desc(spec, **over):
    d, keep = labf._desc(spec)
    for k, v in over.items():
        setattr(d, k, v)
    return d, keep


def test_workspace_size_is_host_arithmetic():
    """labf_workspace_size runs without a GPU: it plans the layout on the
    host; the size grows with the walkers, the ABF bin capacity and the list
    capacity, and is a multiple of 256 bytes."""
    _ensure_built()
    spec, lam = _spec()
    n1 = labf.workspace_size(spec)
    assert n1 > 0 and n1 % 256 == 0
    b2, _ = synth.batch(spec, lam, 3, seed=5)
    assert labf.workspace_size(b2) > 2 * n1
    assert labf.workspace_size(spec, max_bins=4096) > labf.workspace_size(spec, max_bins=64)
    assert labf.workspace_size(spec, list_capacity=4096) > labf.workspace_size(spec, list_capacity=256)
    # the pruned lists hold up to every atom of a cluster list's entries
    assert (labf.workspace_size(spec, list_capacity=512) - labf.workspace_size(spec, list_capacity=256)
            >= 256 * 4 * (1 + 8) * int(np.ceil(spec.n_atoms / 8)))
    # PME grids (complex FP64) live in the workspace too
    sp = synth.with_pme(dataclasses.replace(spec), dims=(16, 16, 32))
    sp2 = synth.with_pme(dataclasses.replace(spec), dims=(16, 16, 16))
    assert labf.workspace_size(sp) - labf.workspace_size(sp2) >= 16 * 16 * 16 * 16


@pytest.mark.parametrize("field,value,msg", [
    ("max_bins", -1, "max_bins"), ("max_bins", 5000, "max_bins"),
    ("list_capacity", 3, "list_capacity"), ("list_capacity", (1 << 20) + 1, "list_capacity"),
    ("prune_buffer", np.array([-0.1]), "prune_buffer"), ("prune_buffer", np.array([5.0]), "prune_buffer"),
    ("prune_buffer", np.array([np.nan]), "prune_buffer"),
])
def test_workspace_size_validates_the_descriptor(field, value, msg):
    _ensure_built()
    spec, _ = _spec()
    if isinstance(value, np.ndarray):
        value = np.ascontiguousarray(value, np.float64)
        d, keep = _raw_desc(spec, **{field: value.ctypes.data})
        keep["_value"] = value
    else:
        d, keep = _raw_desc(spec, **{field: value})
    n = C.c_size_t(7)
    assert labf.lib().labf_workspace_size(C.byref(d), C.byref(n)) == -1
    assert n.value == 0
    assert msg in labf.lib().labf_last_error(None).decode()


@pytest.mark.parametrize("ws,nbytes,msg", [
    (None, 0, "workspace is NULL"),
    (256, 1024, "too small"),
    (0x1000 + 8, 1 << 40, "aligned"),
])
def test_create_rejects_a_missing_or_short_workspace_before_device_work(ws, nbytes, msg):
    """The workspace checks come before any device call (the pointer is
    never touched), so they run without a GPU."""
    _ensure_built()
    spec, _ = _spec()
    d, keep = _raw_desc(spec, workspace=ws, workspace_bytes=nbytes)
    h = C.c_void_p()
    assert labf.lib().labf_create_system(C.byref(d), None, C.byref(h)) == -1
    assert h.value is None
    assert msg in labf.lib().labf_last_error(None).decode()
