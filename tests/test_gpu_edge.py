"""Edge cases of the solve through the C ABI: no columns, the shortest and
the longest allowed columns, a batch larger than the resident slots with a
single slot, an iteration limit reached, a provided start on the slot
scheduler, and a workspace that is too small."""
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


def _solve(atom_path, cols, init_pops=None, **opts):
    rh = _rh()
    print(f"[gpu] {atom_path.split('/')[-1]} columns={cols.n_columns} depth={int(cols.offset[-1])} {opts}", flush=True)
    atom = rh.Atom(atom_path)
    dc = rh.DeviceColumns.from_host(cols, init_pops=init_pops)
    out = rh.solve(atom, dc, want_psi=True, **opts)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check(g, cols, atom_path, rtol=1e-10, **kw):
    a = O.Atom(atom_path)
    for c in range(cols.n_columns):
        r, tol = conftest.oracle_lockstep_rtol(a, cols.column(c), floor=rtol, **kw)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        assert g["n_iter"][c] == r["n_iter"] and g["status"][c] == r["status"], c
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=tol)
        np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=tol)


def test_no_columns(atom_dir):
    rh = _rh()
    atom = rh.Atom(atom_dir["h6"])
    empty = synth.Columns.from_list([])
    dc = rh.DeviceColumns.from_host(empty)
    for sched in (0, 1):
        out = rh.solve(atom, dc, scheduler=sched)
        torch.cuda.synchronize()
        assert out["pops"].numel() == 0 and out["n_iter"].numel() == 0


@pytest.mark.parametrize("scheduler,precision", [(0, 0), (1, 0), (1, 1)])
def test_two_point_and_longest_columns(atom_dir, scheduler, precision):
    """Columns of the minimum (2) and maximum (1024) depth counts together,
    the longest one a resampled cube column."""
    base = synth.cube_columns(1, 64, 64).column(7)
    n = len(base["T"])
    zf = np.linspace(0.0, n - 1.0, 1024)
    longest = {k: np.interp(zf, np.arange(n), np.asarray(v, dtype=np.float64)) for k, v in base.items()}
    longest["n_H"] = np.exp(np.interp(zf, np.arange(n), np.log(base["n_H"])))
    longest["n_e"] = np.exp(np.interp(zf, np.arange(n), np.log(base["n_e"])))
    two = {k: np.asarray(v)[[0, -1]] for k, v in base.items()}
    cols = synth.Columns.from_list([two, longest, two])
    assert list(np.diff(cols.offset)) == [2, 1024, 2]
    kw = dict(n_mu=3, tol=1e-4, max_iter=40)
    g = _solve(atom_dir["h6"], cols, scheduler=scheduler, precision=precision, **kw)
    if precision == 0:
        _check(g, cols, atom_dir["h6"], **kw)
    else:
        a = O.Atom(atom_dir["h6"])
        for c in range(cols.n_columns):
            r = O.solve_column(a, cols.column(c), **kw)
            lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
            np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=1e-3)
            np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=1e-3)


def test_depth_beyond_limit_rejected(atom_dir):
    rh = _rh()
    base = synth.cfg2_columns(seed=1, n_columns=1).column(0)
    zf = np.linspace(0.0, 81.0, 1025)
    col = {k: np.interp(zf, np.arange(82), np.asarray(v, dtype=np.float64)) for k, v in base.items()}
    cols = synth.Columns.from_list([col])
    atom = rh.Atom(atom_dir["h6"])
    dc = rh.DeviceColumns.from_host(cols)
    with pytest.raises(rh.RH15DError):
        rh.solve(atom, dc)


def test_one_slot_many_columns_and_iteration_limit(atom_dir):
    """A single resident slot cycling through every column, and columns
    stopped by the iteration limit (status 1) next to converged ones."""
    cols = synth.cfg2_columns(seed=8, n_columns=5)
    kw = dict(n_mu=3, tol=1e-8, max_iter=6, coll_scale=0.05)
    g = _solve(atom_dir["h6"], cols, scheduler=1, batch_columns=1, **kw)
    assert np.any(g["status"] == 1) and np.all(g["n_iter"][g["status"] == 1] == 6)
    _check(g, cols, atom_dir["h6"], **kw)
    h = _solve(atom_dir["h6"], cols, scheduler=0, batch_columns=2, **kw)
    for k in ("pops", "spectrum", "n_iter", "status"):
        np.testing.assert_array_equal(g[k], h[k])


def test_provided_start_on_slots(atom_dir):
    cols = synth.cfg2_columns(seed=3, n_columns=4)
    a = O.Atom(atom_dir["h6"])
    first = [O.solve_column(a, cols.column(c), n_mu=5, tol=0.0, max_iter=3) for c in range(cols.n_columns)]
    init = np.concatenate([r["pops"] for r in first])
    kw = dict(n_mu=5, tol=0.0, max_iter=2, start=O.START_PROVIDED)
    g = _solve(atom_dir["h6"], cols, init_pops=init, scheduler=1, batch_columns=3, **kw)
    for c in range(cols.n_columns):
        r = O.solve_column(a, cols.column(c), init_pops=first[c]["pops"], **kw)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=1e-10)


def test_workspace_too_small_is_an_error(atom_dir):
    rh = _rh()
    atom = rh.Atom(atom_dir["h6"])
    dc = rh.DeviceColumns.from_host(synth.cfg2_columns(seed=2, n_columns=3))
    opts = rh.default_options(n_mu=3)
    need = rh.workspace_size(atom, dc, opts)
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        rh.Solver(atom, dc, opts, workspace=small)
    s = rh.Solver(atom, dc, opts)
    s.ws_bytes = need // 2          # bypass the binding's own check: the library must refuse
    with pytest.raises(rh.RH15DError, match="workspace too small"):
        s.run()
