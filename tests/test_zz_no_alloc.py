"""rh15d_solve_columns_static (the solve in the library's fixed device
region, nothing allocated) against rh15d_solve_columns through the C ABI:
two calls in a row, the second with fewer columns, bit for bit equal; sizes
beyond the region and profiling are rejected."""
import numpy as np
import pytest

from paper_1411_1079_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("pops", "spectrum", "n_iter", "status", "history", "psi_star")


def _pair(rh, atom, cols, **kw):
    """The same solve through both entry points (the normal one first, which
    also builds the atom's device tables)."""
    dc = rh.DeviceColumns.from_host(cols)
    ref = rh.Solver(atom, dc, rh.default_options(**kw), want_psi=True).run()
    torch.cuda.synchronize()
    fixed = rh.Solver(atom, dc, rh.default_options(**kw), want_psi=True)
    for t in (fixed.pops, fixed.spectrum, fixed.history, fixed.psi_star):
        t.fill_(-1.0)                      # nothing left over from an earlier call
    fixed.run_static()
    torch.cuda.synchronize()
    a = {k: v.cpu().numpy() for k, v in ref.result().items()}
    b = {k: v.cpu().numpy() for k, v in fixed.result().items()}
    return a, b


@pytest.mark.parametrize("precision,scheduler", [(0, 0), (1, 1)])
def test_static_workspace_matches_solve(atom_dir, precision, scheduler):
    from paper_1411_1079_amd import rh15d as rh
    atom = rh.Atom(atom_dir["h6"])
    print(f"[gpu] static workspace {rh.static_workspace_bytes()} bytes", flush=True)
    big = synth.cfg2_columns(seed=5, n_columns=6)
    small = synth.cfg2_columns(seed=6, n_columns=3)
    for cols, batch in ((big, 0), (small, 2)):
        kw = dict(n_mu=5, tol=1e-4, max_iter=60, precision=precision, scheduler=scheduler, batch_columns=batch)
        print(f"[gpu] columns={cols.n_columns} {kw}", flush=True)
        a, b = _pair(rh, atom, cols, **kw)
        assert np.all(a["status"] == 0)
        for k in KEYS:
            np.testing.assert_array_equal(b[k], a[k], err_msg=k)


def test_static_workspace_limits(atom_dir):
    from paper_1411_1079_amd import rh15d as rh
    atom = rh.Atom(atom_dir["h6"])
    cols = synth.cfg2_columns(seed=2, n_columns=64)
    dc = rh.DeviceColumns.from_host(cols)
    s = rh.Solver(atom, dc, rh.default_options(n_mu=5, batch_columns=64), want_psi=False)
    with pytest.raises(rh.RH15DError, match="more than"):
        s.run_static()
    s = rh.Solver(atom, dc, rh.default_options(n_mu=5, profile=1), want_psi=False)
    with pytest.raises(rh.RH15DError, match="profiling"):
        s.run_static()
