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
