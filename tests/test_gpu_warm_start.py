"""The learned start solution end to end: train the network on columns the
GPU path converged (one synthetic cube), start MALI on another cube from
its prediction, and check what it gains and that MALI still decides the
answer.  The size of the gain is an empirical property of the synthetic
atmospheres (not pinned by the paper); the test requires a reduction of
the mean iteration count by at least 5 % and of the 99th percentile, and
answers within 1e-3 of the oracle converged to 1e-10 from either start
(both stop by the change test of 1e-4 and the fixed-point bound of
2e-4)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1411_1079_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KW = dict(n_mu=5, tol=1e-4, tol_fp=2e-4, max_iter=200)


@pytest.fixture(scope="module")
def cubes():
    """Training columns: every 4th column of one 256 x 256 cube; held-out
    columns: every 16th column of another."""
    a = synth.cube_columns(7, 256, 256).select(list(range(0, 65536, 4)))
    b = synth.cube_columns(1, 256, 256).select(list(range(0, 65536, 16)))
    return a, b


@pytest.fixture(scope="module")
def trained(atom_dir, cubes):
    from paper_1411_1079_amd import rh15d as rh
    from paper_1411_1079_amd import warmstart
    atom = rh.Atom(atom_dir["h6"])
    train_cols = cubes[0]
    print(f"[gpu] converge training columns: {train_cols.n_columns}", flush=True)
    dc = rh.DeviceColumns.from_host(train_cols)
    # targets: the FP64 form converged well below the iteration's own stopping rule
    res = rh.solve(atom, dc, precision=0, scheduler=1, n_mu=5, tol=1e-6, max_iter=300)
    assert int((res["status"] != 0).sum()) <= train_cols.n_columns // 100
    print("[gpu] train network", flush=True)
    net, rep = warmstart.train(atom, dc, res["pops"], steps=6000, batch=8192, lr=2e-3, seed=1)
    print(f"trained on {rep.points} points: loss {rep.loss_first:.4g} -> {rep.loss_last:.4g} in {rep.seconds:.2f} s",
          flush=True)
    assert rep.loss_last < 0.01 * rep.loss_first
    return atom, net


def _errors(atom_path, cols, out, picks):
    """Largest relative difference of populations and emergent intensity
    from the oracle converged to 1e-10, per picked column."""
    a = O.Atom(atom_path)
    errs = []
    for c in picks:
        r = O.solve_column(a, cols.column(c), n_mu=5, tol=1e-10, max_iter=400)
        lo, hi = int(cols.offset[c]), int(cols.offset[c + 1])
        errs.append(max(np.max(np.abs(out["pops"][lo:hi] / r["pops"] - 1)),
                        np.max(np.abs(out["spectrum"][c] / r["spectrum"] - 1))))
    return np.array(errs)


def _accuracy_unchanged(atom_path, cols, out, cold, picks):
    """Both the learned start and the LTE start end within 1e-3 of the
    oracle converged to 1e-10."""
    ew, ec = _errors(atom_path, cols, out, picks), _errors(atom_path, cols, cold, picks)
    print(f"errors vs converged oracle: learned start {ew}, LTE start {ec}", flush=True)
    assert np.all(ew <= 1e-3) and np.all(ec <= 1e-3), (ew, ec)


def test_warm_start_reduces_iterations(trained, cubes, atom_dir):
    """Fewer iterations on average and in the slow tail, every column
    converged, accuracy against the oracle unchanged."""
    from paper_1411_1079_amd import rh15d as rh
    from paper_1411_1079_amd import warmstart
    atom, net = trained
    cols = cubes[1]
    dc = rh.DeviceColumns.from_host(cols)
    print(f"[gpu] cold and warm solves of {cols.n_columns} held-out columns", flush=True)
    cold = {k: v.cpu().numpy() for k, v in rh.solve(atom, dc, precision=1, scheduler=1, **KW).items()}
    ws = warmstart.WarmStartSolver(atom, dc, net, rh.default_options(precision=1, scheduler=1, **KW))
    ws.run()
    assert ws.refine_failed() == 0
    warm = {k: v.cpu().numpy() for k, v in ws.result().items()}
    assert np.all(cold["status"] == 0) and np.all(warm["status"] == 0)
    ic, iw = cold["n_iter"], warm["n_iter"]
    print(f"mean iterations cold {ic.mean():.3f} warm {iw.mean():.3f}; p90 {np.percentile(ic, 90)} -> "
          f"{np.percentile(iw, 90)}; p99 {np.percentile(ic, 99)} -> {np.percentile(iw, 99)}; "
          f"max {ic.max()} -> {iw.max()}", flush=True)
    assert iw.mean() <= 0.95 * ic.mean()
    assert np.percentile(iw, 99) < np.percentile(ic, 99)
    picks = [int(np.argmax(ic)), int(np.argmax(iw)), 0, 1000, cols.n_columns - 1]
    _accuracy_unchanged(atom_dir["h6"], cols, warm, cold, picks)


def test_bad_network_still_converges(trained, cubes, atom_dir):
    """Garbage weights (huge outputs, clamped) or non-finite weights (LTE
    start): MALI still converges every column to the oracle's answer, with
    columns that fail from the learned start redone from LTE."""
    from paper_1411_1079_amd import rh15d as rh
    from paper_1411_1079_amd import warmstart
    atom, _ = trained
    cols = cubes[1].select(list(range(0, 4096, 256)))
    dc = rh.DeviceColumns.from_host(cols)
    cold = {k: v.cpu().numpy() for k, v in rh.solve(atom, dc, precision=1, scheduler=1, **KW).items()}
    for kind in ("huge", "nan"):
        print(f"[gpu] {kind} network warm start, {cols.n_columns} columns", flush=True)
        net = rh.MLP(64, 2, atom.n_levels, seed=4)
        p = synth.mlp_params([36, 64, 64, atom.n_levels], seed=4, weight_scale=300.0, bias_std=30.0)
        if kind == "nan":
            p[:] = np.nan
        net.set_params(p)
        ws = warmstart.WarmStartSolver(atom, dc, net, rh.default_options(precision=1, scheduler=1, **KW))
        ws.run()
        redone = ws.refine_failed()
        out = {k: v.cpu().numpy() for k, v in ws.result().items()}
        print(f"{kind}: redone {redone}, iterations mean {out['n_iter'].mean():.2f} max {out['n_iter'].max()}",
              flush=True)
        assert np.all(out["status"] == 0)
        _accuracy_unchanged(atom_dir["h6"], cols, out, cold, [0, 7, 15])
