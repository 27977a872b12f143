"""The slot scheduler (resident slots, converged columns retired and slots
refilled from a device-side queue, each iteration replayed as a hipGraph)
against the plain chunked scheduler and the oracle.  Columns are
independent, so every result must be bitwise identical whatever the slot
count, the scheduler, or graph versus eager launches."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1411_1079_amd import synth

import conftest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solve(atom_path, cols, stream=None, **opts):
    from paper_1411_1079_amd import rh15d as rh
    print(f"[gpu] {atom_path.split('/')[-1]} columns={cols.n_columns} opts={opts} stream={stream is not None}",
          flush=True)
    atom = rh.Atom(atom_path)
    dc = rh.DeviceColumns.from_host(cols)
    o = rh.default_options(**opts)
    s = rh.Solver(atom, dc, o, want_spectrum=True, want_psi=True)
    if stream is not None:
        with torch.cuda.stream(stream):
            s.run(stream)
        stream.synchronize()
    else:
        s.run()
        torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in s.result().items()}


def _mixed_columns():
    """Ragged columns that converge after different numbers of iterations."""
    cube = synth.cube_columns(1, 64, 64)
    parts = [cube.column(c) for c in (0, 9, 33, 64, 101, 150, 177, 200, 230, 255)]
    parts += [synth.cfg2_columns(seed=6, n_columns=4).column(c) for c in range(4)]
    return synth.Columns.from_list(parts)


def _same(a, b):
    for k in ("pops", "spectrum", "n_iter", "status", "history", "psi_star"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_slots_match_chunked_bitwise(atom_dir):
    cols = _mixed_columns()
    kw = dict(n_mu=5, tol=1e-5, max_iter=60, coll_scale=0.1)
    ref = _solve(atom_dir["h6"], cols, scheduler=0, **kw)
    assert len(set(ref["n_iter"].tolist())) > 2          # columns finish at different iterations
    for S in (1, 3, 5, 14):
        _same(_solve(atom_dir["h6"], cols, scheduler=1, batch_columns=S, **kw), ref)
    _same(_solve(atom_dir["h6"], cols, scheduler=0, batch_columns=4, **kw), ref)


def test_slots_graph_replay_matches_eager(atom_dir):
    """On a non-default stream the slot scheduler replays a captured graph;
    run it several times with eager work in between and compare every
    replay with the eager result."""
    cols = _mixed_columns()
    kw = dict(n_mu=5, tol=1e-5, max_iter=60, scheduler=1, batch_columns=4)
    eager = _solve(atom_dir["h6"], cols, **kw)
    st = torch.cuda.Stream()
    for rep in range(3):
        g = _solve(atom_dir["h6"], cols, stream=st, **kw)
        _same(g, eager)
        torch.ones(1000, device="cuda").sum().item()    # eager work between replays
    g32 = _solve(atom_dir["h6"], cols, stream=st, precision=1, **kw)
    e32 = _solve(atom_dir["h6"], cols, precision=1, **kw)
    _same(g32, e32)


def test_slots_against_oracle(atom_dir):
    cols = _mixed_columns()
    kw = dict(n_mu=5, tol=1e-5, max_iter=60, coll_scale=0.1)
    g = _solve(atom_dir["h6"], cols, scheduler=1, batch_columns=3, **kw)
    a = O.Atom(atom_dir["h6"])
    for c in range(cols.n_columns):
        r, rtol = conftest.oracle_lockstep_rtol(a, cols.column(c), **kw)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        assert g["n_iter"][c] == r["n_iter"] and g["status"][c] == r["status"]
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=rtol)
        np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=rtol)
        np.testing.assert_allclose(g["psi_star"][lo:hi].T, r["psi_star"], rtol=rtol, atol=1e-300)


def test_slots_zero_iterations_and_zero_radiation(atom_dir):
    cols = synth.cfg2_columns(seed=2, n_columns=5)
    a = O.Atom(atom_dir["h6"])
    for start, it in ((O.START_LTE, 0), (O.START_ZERO_RADIATION, 0), (O.START_ZERO_RADIATION, 3)):
        kw = dict(n_mu=3, tol=0.0, max_iter=it, start=start)
        g = _solve(atom_dir["h6"], cols, scheduler=1, batch_columns=2, **kw)
        for c in range(cols.n_columns):
            r = O.solve_column(a, cols.column(c), **kw)
            lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
            assert g["n_iter"][c] == r["n_iter"] == it and g["status"][c] == r["status"]
            np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=1e-10)
            np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=1e-10)


@pytest.mark.parametrize("mc,pack", [(1, 1), (1, 2), (5, 1), (5, 2)])
def test_every_sweep_shape_matches_oracle(atom_dir, mc, pack):
    """Angles per lane and the packing of wavelengths into wavefronts change
    only the order of the sums: every shape agrees with the oracle."""
    cols = _mixed_columns().select([0, 3, 7, 11])
    kw = dict(n_mu=5, tol=1e-5, max_iter=60, coll_scale=0.1)
    g = _solve(atom_dir["h6"], cols, scheduler=1, sweep_mc=mc, sweep_pack=pack, **kw)
    a = O.Atom(atom_dir["h6"])
    for c in range(cols.n_columns):
        r, rtol = conftest.oracle_lockstep_rtol(a, cols.column(c), **kw)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        assert g["n_iter"][c] == r["n_iter"] and g["status"][c] == r["status"]
        np.testing.assert_allclose(g["pops"][lo:hi], r["pops"], rtol=rtol)
        np.testing.assert_allclose(g["spectrum"][c], r["spectrum"], rtol=rtol)
        np.testing.assert_allclose(g["psi_star"][lo:hi].T, r["psi_star"], rtol=rtol, atol=1e-300)


def test_autotune_picks_a_shape_used_by_automatic_solves(atom_dir):
    """The autotuner times every shape, keeps the fastest, and a later
    solve with the automatic shape gives exactly the chosen shape's
    results."""
    from paper_1411_1079_amd import rh15d as rh
    cols = _mixed_columns()
    kw = dict(n_mu=5, tol=1e-5, max_iter=60, scheduler=1, precision=1)
    atom = rh.Atom(atom_dir["h6"])
    dc = rh.DeviceColumns.from_host(cols)
    print(f"[gpu] autotune on {cols.n_columns} columns", flush=True)
    r = rh.autotune(atom, dc, **kw)
    print(r, flush=True)
    assert len(r["candidates"]) == 4            # mc 1 and 5 (3 does not divide n_mu = 5) x two packings
    assert min(c["ms"] for c in r["candidates"]) == next(
        c["ms"] for c in r["candidates"] if (c["sweep_mc"], c["sweep_pack"]) == (r["sweep_mc"], r["sweep_pack"]))
    auto = rh.Solver(atom, dc, rh.default_options(**kw), want_spectrum=True).run().result()
    chosen = rh.Solver(atom, dc, rh.default_options(sweep_mc=r["sweep_mc"], sweep_pack=r["sweep_pack"], **kw),
                       want_spectrum=True).run().result()
    torch.cuda.synchronize()
    for k in ("pops", "spectrum", "n_iter", "status"):
        np.testing.assert_array_equal(auto[k].cpu().numpy(), chosen[k].cpu().numpy())
