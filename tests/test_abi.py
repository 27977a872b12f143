"""The C-ABI library without a GPU: it loads, exports every entry point
the header declares, parses atoms on the host, and rejects bad arguments
before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1411_1079_amd import rh15d, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rh15d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rh15d_\w+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert set(declared_functions()) == set(rh15d.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = rh15d.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_atom_setup_on_host_matches_oracle_grid(atom_dir):
    for key in ("two_level", "h6", "tiny"):
        a = rh15d.Atom(atom_dir[key])
        o = O.Atom(atom_dir[key])
        assert (a.n_levels, a.n_lines, a.n_continua, a.n_lambda) == (o.n_levels, o.n_lines, o.n_cont, o.n_lambda)
        np.testing.assert_array_equal(a.lam, o.lam)


def test_bad_atom_file(tmp_path):
    p = tmp_path / "bad.atom"
    p.write_text("RH15D-ATOM 1\nNAME X\nMASS_AMU 1\nABUNDANCE 1\nLEVELS 1\n0 1 0\n")
    with pytest.raises(rh15d.RH15DError) as e:
        rh15d.Atom(str(p))
    assert e.value.code == -2
    with pytest.raises(rh15d.RH15DError):
        rh15d.Atom(str(tmp_path / "missing.atom"))


class _FakeTensor:
    """Host arrays standing in for device buffers: validation rejects
    these calls before any pointer is dereferenced or any HIP call."""

    def __init__(self, a):
        self.a = np.ascontiguousarray(a, dtype=np.float64)
        self.dtype = type("d", (), {"is_floating_point": True})()

    def element_size(self):
        return 8

    def is_contiguous(self):
        return True

    def data_ptr(self):
        return self.a.ctypes.data


def _fake_columns(nd):
    off = np.concatenate([[0], np.cumsum(nd)]).astype(np.int64)
    n = int(off[-1])
    f = lambda: _FakeTensor(np.ones(n))
    return rh15d.DeviceColumns(offset=off, z=f(), T=f(), n_e=f(), n_H=f(), v_z=f(), v_turb=f())


@pytest.mark.parametrize("bad", [
    dict(n_mu=0), dict(n_mu=17), dict(ng_order=3), dict(max_iter=-1), dict(precision=5), dict(start=7),
    dict(tol=-1.0), dict(start=2),
])
def test_invalid_options_rejected(atom_dir, bad):
    a = rh15d.Atom(atom_dir["h6"])
    dc = _fake_columns([5, 6])
    with pytest.raises(rh15d.RH15DError) as e:
        rh15d.workspace_size(a, dc, rh15d.default_options(**bad))
    assert e.value.code == -1


@pytest.mark.parametrize("nd", [[1], [5, 1], [2000]])
def test_invalid_depths_rejected(atom_dir, nd):
    a = rh15d.Atom(atom_dir["h6"])
    with pytest.raises(rh15d.RH15DError) as e:
        rh15d.workspace_size(a, _fake_columns(nd), rh15d.default_options())
    assert "depth points" in str(e.value)


def _grid_call(atom, nd_in, nd_out, **weights):
    """rh15d_optimize_grid on host arrays standing in for device buffers
    (every case here fails validation before any HIP call)."""
    dc = _fake_columns(nd_in)
    off = np.concatenate([[0], np.cumsum(nd_out)]).astype(np.int64)
    bufs = [np.zeros(max(int(off[-1]), 1)) for _ in range(6)] + [np.zeros(len(nd_out), dtype=np.int32)]
    o = rh15d.GridOutput()
    o.depth_offset = off.ctypes.data_as(C.POINTER(C.c_int64))
    for name, b in zip(("z", "T", "n_e", "n_H", "v_z", "v_turb", "status"), bufs):
        setattr(o, name, b.ctypes.data)
    opts = rh15d.default_grid_options(**weights)
    return rh15d.lib().rh15d_optimize_grid(atom._h, C.byref(rh15d._cols_struct(dc)), C.byref(opts), C.byref(o), None)


@pytest.mark.parametrize("case", [
    dict(w_T=-1.0), dict(w_z=0.0, w_T=0.0, w_v=0.0, w_tau=0.0), dict(w_v=float("nan")), dict(w_tau=float("inf")),
    dict(nd_out=[1, 5]), dict(nd_out=[5, 1025]), dict(nd_in=[8193, 4]),
])
def test_grid_optimisation_rejects_bad_arguments(atom_dir, case):
    a = rh15d.Atom(atom_dir["h6"])
    case = dict(case)
    nd_in, nd_out = case.pop("nd_in", [6, 4]), case.pop("nd_out", [5, 5])
    assert _grid_call(a, nd_in, nd_out, **case) == -1
    assert rh15d.lib().rh15d_last_error()


def test_grid_defaults_and_empty_call(atom_dir):
    o = rh15d.default_grid_options()
    assert (o.w_z, o.w_T, o.w_v, o.w_tau) == (1.0, 2.0, 2.0e-4, 0.2)
    a = rh15d.Atom(atom_dir["h6"])
    assert _grid_call(a, [], []) == 0   # nothing to do, nothing launched


def test_partial_magnetic_field_rejected(atom_dir):
    a = rh15d.Atom(atom_dir["zeeman_tiny"])
    dc = _fake_columns([5, 6])
    dc.B = _FakeTensor(np.ones(11))
    with pytest.raises(rh15d.RH15DError) as e:
        rh15d.workspace_size(a, dc, rh15d.default_options())
    assert e.value.code == -1 and "B_incl" in str(e.value)


def test_zeeman_atoms_load_on_host(atom_dir):
    for key in ("zeeman_tiny", "zeeman_tiny_prd", "ca2", "ca2_crd"):
        a = rh15d.Atom(atom_dir[key])
        o = O.Atom(atom_dir[key])
        assert (a.n_levels, a.n_lines, a.n_continua, a.n_lambda) == (o.n_levels, o.n_lines, o.n_cont, o.n_lambda)


def test_network_training_entries_reject_bad_arguments():
    """The training entry points check their arguments before any HIP call:
    a missing handle or buffer, a batch outside 1..262144, a negative batch
    count."""
    lib = rh15d.lib()
    buf = np.zeros(64, dtype=np.float32)
    p = buf.ctypes.data
    lr = (C.c_float * 2)(1e-3, 1e-3)
    assert lib.rh15d_mlp_train_batches(None, p, p, 4, 2, lr, None, None) == -1
    assert lib.rh15d_mlp_train_step(None, p, p, 4, C.c_float(1e-3), None, None) == -1
    assert lib.rh15d_mlp_gradients(None, p, p, 4, None, None) == -1
    assert lib.rh15d_mlp_forward(None, p, 4, p, None) == -1
    assert "argument" in lib.rh15d_last_error().decode()
