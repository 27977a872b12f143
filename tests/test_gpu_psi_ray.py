"""Psi* of every ray (the full diagonal of the local operator, for small
problems) through the C ABI against the oracle: FP64 lock-step on ragged
columns of the tiny atom (blends, a line inside a continuum, overlapping
continua), the same with a PRD line and its final rho, the FP32 form
within 1e-3, consistency with the per-transition average, and NaN rows of
an unusable column."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1411_1079_amd import synth

import conftest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rh():
    from paper_1411_1079_amd import rh15d
    return rh15d


def _solve(atom_path, cols, **opts):
    rh = _rh()
    print(f"[gpu] psi_ray {atom_path.split('/')[-1]} columns={cols.n_columns} depth={int(cols.offset[-1])} {opts}",
          flush=True)
    atom = rh.Atom(atom_path)
    dc = rh.DeviceColumns.from_host(cols)
    s = rh.Solver(atom, dc, rh.default_options(**opts), want_psi=True, want_psi_ray=True)
    s.run()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in s.result().items()}


def _columns():
    return synth.Columns.from_list([conftest.tiny_column(8), conftest.tiny_column(13, vz=-4e3),
                                    conftest.tiny_column(5, vz=1e3)])


@pytest.mark.parametrize("scheduler", [0, 1])
def test_tiny_atom_lockstep(atom_dir, scheduler):
    cols = _columns()
    kw = dict(n_mu=3, tol=1e-10, max_iter=300)
    r = _solve(atom_dir["tiny"], cols, precision=0, scheduler=scheduler, **kw)
    a = O.Atom(atom_dir["tiny"])
    for c in range(cols.n_columns):
        col = cols.column(c)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        ref, rtol = conftest.oracle_lockstep_rtol(a, col, **kw)
        pr = O.column_psi_ray(a, col, ref["pops"], 3)
        got = r["psi_ray"][lo:hi]
        np.testing.assert_allclose(got, pr, rtol=max(rtol, 1e-10) * 10, atol=1e-12 * np.abs(pr).max())
        assert np.all(got[0, :, :, 0] == 0.0) and np.all(got[-1, :, :, 1] == 0.0)


def test_prd_line(atom_dir):
    """The PRD atom on the stable ragged columns of the PRD lock-step tests,
    40 iterations: Psi* with the emission profile of the final rho."""
    cols = synth.Columns.from_list([conftest.tiny_column(10, vz=2e3), conftest.tiny_column(7, vz=5e3),
                                    conftest.tiny_column(2)])
    kw = dict(n_mu=3, tol=0.0, max_iter=40, coll_scale=1e-2, prd=1)
    r = _solve(atom_dir["prd_tiny"], cols, precision=0, scheduler=1, **kw)
    a = O.Atom(atom_dir["prd_tiny"])
    for c in range(cols.n_columns):
        col = cols.column(c)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        ref, rtol = conftest.oracle_lockstep_rtol(a, col, prd_lines=(0,), **kw)
        pr = O.column_psi_ray(a, col, ref["pops"], 3, prd_rho=ref["rho"])
        np.testing.assert_allclose(r["psi_ray"][lo:hi], pr, rtol=max(rtol, 1e-10) * 10, atol=1e-12 * np.abs(pr).max())


def test_fp32_form(atom_dir):
    cols = _columns()
    r = _solve(atom_dir["tiny"], cols, precision=1, scheduler=1, n_mu=3, tol=1e-6, max_iter=300)
    assert np.all(r["status"] == 0)
    a = O.Atom(atom_dir["tiny"])
    for c in range(cols.n_columns):
        col = cols.column(c)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        ref = O.solve_column(a, col, n_mu=3, tol=1e-10, max_iter=300)
        pr = O.column_psi_ray(a, col, ref["pops"], 3)
        np.testing.assert_allclose(r["psi_ray"][lo:hi], pr, rtol=1e-3, atol=1e-9 * np.abs(pr).max())


def test_unusable_column_rows_are_nan(atom_dir):
    rh = _rh()
    cols = _columns()
    T = cols.T.copy()
    T[cols.offset[1] + 2] = -1.0
    bad = synth.Columns(offset=cols.offset, z=cols.z, T=T, n_e=cols.n_e, n_H=cols.n_H, v_z=cols.v_z,
                        v_turb=cols.v_turb)
    r = _solve(atom_dir["tiny"], bad, precision=0, n_mu=3, tol=1e-8, max_iter=300)
    assert r["status"][1] == rh.BAD_INPUT
    lo, hi = int(cols.offset[1]), int(cols.offset[2])
    assert np.all(np.isnan(r["psi_ray"][lo:hi]))
    assert np.all(np.isfinite(r["psi_ray"][:lo])) and np.all(np.isfinite(r["psi_ray"][hi:]))
