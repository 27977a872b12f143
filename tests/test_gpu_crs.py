"""Convergence aids (Sec. 2.3) through the C ABI.  Collisional-radiative
switching: the GPU path against the oracle with the switched collisions, in
lock-step for FP64 (same iteration counts, same Ng decisions) and within
1e-3 for the FP32 form; switching off reproduces the default bit for bit;
invalid factors are rejected.  Failed columns solved again with another
option set."""
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
    print(f"[gpu] {atom_path.split('/')[-1]} columns={cols.n_columns} depth={int(cols.offset[-1])} {opts}", flush=True)
    atom = rh.Atom(atom_path)
    dc = rh.DeviceColumns.from_host(cols)
    out = rh.solve(atom, dc, want_psi=True, **opts)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _columns():
    cube = synth.cube_columns(1, 64, 64)
    parts = [cube.column(c) for c in (33, 177)]
    parts += [synth.cfg2_columns(seed=9, n_columns=3).column(c) for c in range(3)]
    return synth.Columns.from_list(parts)


@pytest.mark.parametrize("scheduler", [0, 1])
def test_fp64_lockstep_with_switching(atom_dir, scheduler):
    cols = _columns()
    kw = dict(n_mu=3, tol=1e-6, max_iter=120, coll_scale=0.3, crs_f0=1e4)
    g = _solve(atom_dir["h6"], cols, scheduler=scheduler, **kw)
    a = O.Atom(atom_dir["h6"])
    for c in range(cols.n_columns):
        r, rtol = conftest.oracle_lockstep_rtol(a, cols.column(c), **kw)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        assert g["status"][c] == r["status"] == 0 and g["n_iter"][c] == r["n_iter"], (c, g["n_iter"][c], r["n_iter"])
        assert r["n_iter"] >= 5
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=rtol)
        np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=rtol)
        n = r["n_iter"]
        np.testing.assert_allclose(g["history"][c, :n], r["history"][:n], rtol=1e-6, atol=4 * rtol)


def test_fp32_with_switching(atom_dir):
    cols = _columns()
    kw = dict(n_mu=5, tol=1e-4, max_iter=120, crs_f0=1e3)
    g = _solve(atom_dir["h6"], cols, precision=1, scheduler=1, **kw)
    a = O.Atom(atom_dir["h6"])
    for c in range(cols.n_columns):
        r = O.solve_column(a, cols.column(c), **kw)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        assert g["status"][c] == 0 and r["status"] == 0
        assert g["n_iter"][c] >= 4
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=1e-3)
        np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=1e-3)


def test_switching_off_is_the_default(atom_dir):
    cols = _columns().select([0, 2])
    kw = dict(n_mu=3, tol=1e-6, max_iter=60, scheduler=1)
    ref = _solve(atom_dir["h6"], cols, **kw)
    off = _solve(atom_dir["h6"], cols, crs_f0=0.5, **kw)
    for k in ("pops", "spectrum", "n_iter", "status", "history", "psi_star"):
        np.testing.assert_array_equal(ref[k], off[k], err_msg=k)


@pytest.mark.parametrize("bad", [float("nan"), -1.0, float("inf")])
def test_invalid_factor_rejected(atom_dir, bad):
    rh = _rh()
    atom = rh.Atom(atom_dir["h6"])
    dc = rh.DeviceColumns.from_host(_columns().select([0]))
    with pytest.raises(rh.RH15DError, match="crs_f0"):
        rh.solve(atom, dc, crs_f0=bad)


def test_failed_columns_solved_again_with_other_options(atom_dir):
    """Columns stopped by a small iteration limit are solved again with
    another option set (switched collisions, a larger limit): every column
    then converges, the re-solved ones match the oracle run with the second
    option set (their iteration counts adding both attempts, their history
    rows holding both attempts' changes in order), and the columns that had
    converged keep their results bit for bit."""
    rh = _rh()
    cols = _columns()
    atom = rh.Atom(atom_dir["h6"])
    dc = rh.DeviceColumns.from_host(cols)
    first = dict(n_mu=3, tol=1e-6, max_iter=6, coll_scale=0.3)
    print(f"[gpu] first attempt {first}", flush=True)
    out = rh.solve(atom, dc, want_psi=True, **first)
    torch.cuda.synchronize()
    g0 = {k: v.cpu().numpy().copy() for k, v in out.items()}
    failed = g0["status"] != 0
    assert failed.any() and (~failed).any()
    again = dict(n_mu=3, tol=1e-6, max_iter=120, coll_scale=0.3, crs_f0=1e3)
    print(f"[gpu] second attempt {again}", flush=True)
    n = rh.resolve_failed(atom, dc, out, rh.default_options(**again))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    assert n == int(failed.sum()) and np.all(g["status"] == 0)
    a = O.Atom(atom_dir["h6"])
    for c in range(cols.n_columns):
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        if not failed[c]:
            for k in ("n_iter", "status"):
                assert g[k][c] == g0[k][c]
            np.testing.assert_array_equal(g["pops"][lo:hi], g0["pops"][lo:hi])
            np.testing.assert_array_equal(g["spectrum"][c], g0["spectrum"][c])
            continue
        r, rtol = conftest.oracle_lockstep_rtol(a, cols.column(c), **again)
        assert g["n_iter"][c] == first["max_iter"] + r["n_iter"]
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=rtol)
        np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=rtol)
        np.testing.assert_allclose(g["psi_star"][lo:hi].T, r["psi_star"], rtol=rtol, atol=1e-300)
        # the history row: the first attempt's changes, then the second's
        n1 = first["max_iter"]
        np.testing.assert_array_equal(g["history"][c, :n1], g0["history"][c, :n1])
        m = min(g["history"].shape[1] - n1, r["n_iter"])
        np.testing.assert_allclose(g["history"][c, n1:n1 + m], r["history"][:m], rtol=1e-6, atol=4 * rtol)
