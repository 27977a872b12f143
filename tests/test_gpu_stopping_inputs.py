"""Through the C ABI: the fixed-point bound of the stopping rule, the
escape-probability start, per-column handling of unusable inputs and
singular rate matrices, the graph path, and re-solving failed columns.
FP64 results are in lock-step with the oracle (same iteration counts, same
Ng decisions), element by element."""
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


def _solve(atom_path, cols, stream=None, **opts):
    rh = _rh()
    print(f"[gpu] {atom_path.split('/')[-1]} columns={cols.n_columns} depth={int(cols.offset[-1])} {opts}", flush=True)
    atom = rh.Atom(atom_path)
    dc = rh.DeviceColumns.from_host(cols)
    o = rh.default_options(**opts)
    s = rh.Solver(atom, dc, o, want_psi=True)
    if stream is not None:
        with torch.cuda.stream(stream):
            s.run(stream)
    else:
        s.run()
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in s.result().items()}
    out["stats"] = rh.last_stats()
    return out


def _lockstep(g, cols, atom_path, **kw):
    a = O.Atom(atom_path)
    for c in range(cols.n_columns):
        r, rtol = conftest.oracle_lockstep_rtol(a, cols.column(c), **kw)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        assert g["n_iter"][c] == r["n_iter"] and g["status"][c] == r["status"], (c, g["n_iter"][c], r["n_iter"])
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=rtol, err_msg=f"pops {c}")
        np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=rtol, err_msg=f"spectrum {c}")
        np.testing.assert_allclose(g["psi_star"][lo:hi].T, r["psi_star"], rtol=rtol, atol=1e-300, err_msg=f"psi {c}")
        n = r["n_iter"]
        if n > 0:
            np.testing.assert_allclose(g["history"][c, :n], r["history"][:n], rtol=1e-6, atol=4 * rtol)


def _slow_columns():
    cube = synth.cube_columns(1, 64, 64)
    parts = [cube.column(c) for c in (686, 818, 9)]
    parts += [synth.cfg2_columns(seed=4, n_columns=2).column(c) for c in range(2)]
    return synth.Columns.from_list(parts)


@pytest.mark.parametrize("scheduler", [0, 1])
def test_fixed_point_bound_lockstep(atom_dir, scheduler):
    """Change test 1e-4 plus the fixed-point bound 2e-4 (Ng on): the GPU
    stops at the oracle's iteration on every column."""
    cols = _slow_columns()
    kw = dict(n_mu=3, tol=1e-4, tol_fp=2e-4, max_iter=200)
    g = _solve(atom_dir["h6"], cols, scheduler=scheduler, batch_columns=2, **kw)
    _lockstep(g, cols, atom_dir["h6"], **kw)
    plain = _solve(atom_dir["h6"], cols, scheduler=scheduler, batch_columns=2, n_mu=3, tol=1e-4, max_iter=200)
    assert np.all(g["n_iter"] >= plain["n_iter"]) and np.any(g["n_iter"] > plain["n_iter"])


@pytest.mark.parametrize("scheduler", [0, 1])
def test_escape_start_lockstep(atom_dir, scheduler):
    """Escape-probability start (Sec. 2.3): after 1 or 3 escape iterations,
    with 0 or 2 MALI iterations, on the tiny atom (blends, a line inside a
    continuum, overlapping continua) and on the six-level atom."""
    tiny = synth.Columns.from_list([conftest.tiny_column(8), conftest.tiny_column(12, vz=-5e3),
                                    conftest.tiny_column(2)])
    h6 = synth.cfg2_columns(seed=3, n_columns=3)
    for atom, cols, extra in (("tiny", tiny, dict(coll_scale=1e-3)), ("h6", h6, {})):
        for esc, it in ((1, 0), (3, 0), (3, 2)):
            kw = dict(n_mu=3, tol=0.0, max_iter=it, start=O.START_ESCAPE, esc_iter=esc, **extra)
            g = _solve(atom_dir[atom], cols, scheduler=scheduler, batch_columns=2, **kw)
            _lockstep(g, cols, atom_dir[atom], **kw)


def test_escape_start_converges_in_fp32(atom_dir):
    cols = synth.cfg2_columns(seed=3, n_columns=4)
    kw = dict(n_mu=5, tol=1e-4, tol_fp=2e-4, max_iter=200, start=O.START_ESCAPE)
    g = _solve(atom_dir["h6"], cols, scheduler=1, precision=1, **kw)
    a = O.Atom(atom_dir["h6"])
    for c in range(cols.n_columns):
        r = O.solve_column(a, cols.column(c), n_mu=5, tol=1e-10, max_iter=400)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        assert g["status"][c] == 0
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=1e-3)
        np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=1e-3)


def _with_bad_columns():
    """Good columns with three unusable ones between them: a NaN
    temperature, a zero electron density, a height that does not
    decrease."""
    good = synth.cfg2_columns(seed=0, n_columns=5)
    parts = [good.column(c) for c in range(5)]
    bad = []
    for field, k, v in (("T", 10, np.nan), ("n_e", 40, 0.0), ("z", 7, None)):
        col = {key: np.array(val, dtype=np.float64) for key, val in parts[1].items()}
        if field == "z":
            col["z"][k] = col["z"][k - 1]
        else:
            col[field][k] = v
        bad.append(col)
    mixed = [parts[0], bad[0], parts[1], parts[2], bad[1], parts[3], bad[2], parts[4]]
    is_bad = np.array([False, True, False, False, True, False, True, False])
    return good, synth.Columns.from_list(mixed), is_bad


@pytest.mark.parametrize("scheduler,precision", [(0, 0), (1, 0), (1, 1)])
def test_unusable_columns_are_isolated(atom_dir, scheduler, precision):
    """Sec. 2.2: a problematic column is handled on its own.  Columns whose
    data fail the input checks get status BAD_INPUT, no iterations and NaN
    outputs; every other column's results are bit for bit those of a solve
    without them (the oracle reports the same status)."""
    good, mixed, is_bad = _with_bad_columns()
    kw = dict(n_mu=3, tol=1e-4, max_iter=40, scheduler=scheduler, precision=precision, batch_columns=3)
    g = _solve(atom_dir["h6"], mixed, **kw)
    ref = _solve(atom_dir["h6"], good, **kw)
    a = O.Atom(atom_dir["h6"])
    j = 0
    for c in range(mixed.n_columns):
        lo, hi = int(mixed.offset[c]), int(mixed.offset[c + 1])
        if is_bad[c]:
            assert g["status"][c] == O.BAD_INPUT and g["n_iter"][c] == 0
            assert O.solve_column(a, mixed.column(c), n_mu=3)["status"] == O.BAD_INPUT
            for k in ("spectrum", "history"):
                assert np.all(np.isnan(g[k][c])), k
            assert np.all(np.isnan(g["pops"][lo:hi])) and np.all(np.isnan(g["psi_star"][lo:hi]))
            continue
        glo, ghi = int(good.offset[j]), int(good.offset[j + 1])
        np.testing.assert_array_equal(g["pops"][lo:hi], ref["pops"][glo:ghi])
        np.testing.assert_array_equal(g["spectrum"][c], ref["spectrum"][j])
        np.testing.assert_array_equal(g["psi_star"][lo:hi], ref["psi_star"][glo:ghi])
        np.testing.assert_array_equal(g["history"][c], ref["history"][j])
        assert g["n_iter"][c] == ref["n_iter"][j] and g["status"][c] == ref["status"][j] == 0
        j += 1


def _write_isolated_level_atom(path):
    """Three bound levels; level 2 has no radiative (f = 0) and no
    collisional (Omega = 0) link to the others, so the rate matrix has a
    zero row (level 2 is never the most populated one, whose row the
    particle conservation replaces)."""
    lam01 = synth._H * synth._C / (2.0 * synth._EV) * 1e9
    lam12 = synth._H * synth._C / (6.0 * synth._EV) * 1e9
    levels = [(0.0, 2.0, 0), (2.0, 4.0, 0), (8.0, 1.0, 0)]
    lines = [dict(l=0, u=1, f=0.1, profile="GAUSS", coll="OMEGA", cval=1.0, lam=synth.line_grid_nm(lam01, n=9, x_max=4)),
             dict(l=1, u=2, f=0.0, profile="GAUSS", coll="OMEGA", cval=0.0, lam=synth.line_grid_nm(lam12, n=9, x_max=4))]
    return synth.write_atom(path, "ISOLATED", 1.00794, 1.0, levels, lines, [], 1.0e-38)


@pytest.mark.parametrize("scheduler", [0, 1])
def test_singular_rate_matrix_status(atom_dir, tmp_path, scheduler):
    """A singular rate matrix gives status SINGULAR after the first
    iteration, as in the oracle; the columns of another atom are not
    affected (per-column status, no error)."""
    path = _write_isolated_level_atom(str(tmp_path / "isolated.atom"))
    cols = synth.cfg2_columns(seed=1, n_columns=3)
    kw = dict(n_mu=3, tol=1e-4, max_iter=10, scheduler=scheduler)
    g = _solve(path, cols, **kw)
    a = O.Atom(path)
    for c in range(cols.n_columns):
        r = O.solve_column(a, cols.column(c), n_mu=3, tol=1e-4, max_iter=10)
        assert r["status"] == 3 and r["n_iter"] == 1
        assert g["status"][c] == 3 and g["n_iter"][c] == 1


def test_graph_path_is_used_and_matches_eager(atom_dir):
    """On a non-default stream with profiling off the slot scheduler replays
    a captured graph (graph_launches > 0); with profiling on it launches
    every kernel itself; the results are identical."""
    cols = _slow_columns()
    kw = dict(n_mu=3, tol=1e-4, tol_fp=2e-4, max_iter=200, scheduler=1, batch_columns=2)
    st = torch.cuda.Stream()
    g = _solve(atom_dir["h6"], cols, stream=st, **kw)
    e = _solve(atom_dir["h6"], cols, profile=1, **kw)
    print(f"graph launches {g['stats']['graph_launches']}, eager {e['stats']['graph_launches']}", flush=True)
    assert g["stats"]["graph_launches"] > 0 and e["stats"]["graph_launches"] == 0
    for k in ("pops", "spectrum", "n_iter", "status", "history", "psi_star"):
        np.testing.assert_array_equal(g[k], e[k], err_msg=k)


def test_resolve_failed_appends_history(atom_dir):
    """Columns stopped by a 6-iteration limit are solved again from LTE on
    a side stream; their history rows hold the first attempt's 6 changes
    followed by the second attempt's, and n_iter counts both."""
    rh = _rh()
    cols = _slow_columns()
    atom = rh.Atom(atom_dir["h6"])
    dc = rh.DeviceColumns.from_host(cols)
    first = dict(n_mu=3, tol=1e-6, max_iter=6)
    out = rh.solve(atom, dc, **first)
    torch.cuda.synchronize()
    h0 = out["history"].cpu().numpy().copy()
    failed = out["status"].cpu().numpy() != 0
    assert failed.any()
    again = rh.default_options(n_mu=3, tol=1e-6, max_iter=40)
    st = torch.cuda.Stream()
    n = rh.resolve_failed(atom, dc, out, again, stream=st)
    torch.cuda.synchronize()
    assert n == int(failed.sum())
    g = {k: v.cpu().numpy() for k, v in out.items()}
    a = O.Atom(atom_dir["h6"])
    for c in np.nonzero(failed)[0]:
        r = O.solve_column(a, cols.column(int(c)), n_mu=3, tol=1e-6, max_iter=40)
        assert g["n_iter"][c] == 6 + r["n_iter"] and g["status"][c] == r["status"]
        np.testing.assert_array_equal(g["history"][c, :6], h0[c, :6])
        m = min(r["n_iter"], g["history"].shape[1] - 6)
        np.testing.assert_allclose(g["history"][c, 6:6 + m], r["history"][:m], rtol=1e-6, atol=4e-10)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=1e-9)
