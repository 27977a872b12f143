"""The polarised emergent spectrum (Zeeman effect, full Stokes vector)
through the C ABI, against the oracle: the Zeeman test atom (J 1/2 -> 1/2,
1/2 -> 3/2 and 3/2 -> 1/2 lines) with a field that varies with depth, in
FP64 lock-step; with a PRD line; the FP32 form (Stokes in FP64 from its
populations) within 1e-3; zero field against the Stokes-I spectrum;
unusable columns and non-finite fields; the Ca II-like atom on synthetic
cube columns with a field of 0-2 kG and isotropic direction."""
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


def zeeman_columns(n_cols=3, n=40):
    parts, fields = [], []
    for c in range(n_cols):
        z = np.linspace(1.5e6, 0.0, n)
        s = np.linspace(0.0, 1.0, n)
        T = 4300.0 + 300.0 * c + 2500.0 * s ** 2
        T[-1] = T[-2]
        nH = 1.0e21 * np.exp(-z / 1.5e5)
        vz = 2.0e3 * (c - 1) * np.cos(3.0 * s)
        parts.append(dict(z=z, T=T, n_e=1.0e-3 * nH, n_H=nH, v_z=vz, v_turb=np.full(n, 1.5e3)))
        fields.append((0.05 + 0.1 * s + 0.02 * c, 0.3 + 1.5 * s + 0.2 * c, 0.7 - 2.0 * s + 0.5 * c))
    return synth.Columns.from_list(parts), fields


def _field_arrays(fields):
    return tuple(np.concatenate([f[i] for f in fields]) for i in range(3))


def _solve(atom_path, cols, field, **opts):
    rh = _rh()
    print(f"[gpu] stokes {atom_path.split('/')[-1]} columns={cols.n_columns} depth={int(cols.offset[-1])} "
          f"field={'yes' if field is not None else 'no'} {opts}", flush=True)
    atom = rh.Atom(atom_path)
    dc = rh.DeviceColumns.from_host(cols, field=field)
    s = rh.Solver(atom, dc, rh.default_options(**opts), want_stokes=True)
    s.run()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in s.result().items()}


def _compare(st_gpu, st_ref, rtol, what):
    scale = np.max(np.abs(st_ref[:, 0]))
    np.testing.assert_allclose(st_gpu[:, 0], st_ref[:, 0], rtol=rtol, atol=0, err_msg=f"{what} I")
    np.testing.assert_allclose(st_gpu[:, 1:], st_ref[:, 1:], rtol=0, atol=rtol * scale, err_msg=f"{what} QUV")


def test_zeeman_atom_lockstep_fp64(atom_dir):
    cols, fields = zeeman_columns()
    kw = dict(n_mu=3, tol=1e-10, max_iter=400)
    r = _solve(atom_dir["zeeman_tiny"], cols, _field_arrays(fields), precision=0, **kw)
    assert np.all(r["status"] == 0)
    a = O.Atom(atom_dir["zeeman_tiny"])
    for c in range(cols.n_columns):
        col = cols.column(c)
        ref, rtol = conftest.oracle_lockstep_rtol(a, col, **kw)
        st = O.stokes_column(a, col, ref["pops"], 3, *fields[c])
        assert np.max(np.abs(st[:, 3])) > 1e-3 * np.max(st[:, 0])   # the field matters
        _compare(r["stokes"][c], st, max(rtol, 1e-10) * 10, f"column {c}")


def test_zero_field_is_the_spectrum(atom_dir):
    cols, _ = zeeman_columns(2)
    for prec in (0, 1):
        r = _solve(atom_dir["zeeman_tiny"], cols, None, precision=prec, n_mu=3, tol=1e-6, max_iter=200)
        # FP64 Stokes from the final populations against the sweep precision's spectrum
        rtol = 1e-12 if prec == 0 else 1e-4
        np.testing.assert_allclose(r["stokes"][:, :, 0], r["spectrum"], rtol=rtol)
        assert np.max(np.abs(r["stokes"][:, :, 1:])) <= 1e-13 * np.max(r["stokes"][:, :, 0])


def test_prd_line_uses_the_final_rho(atom_dir):
    cols, fields = zeeman_columns(2, n=24)
    kw = dict(n_mu=3, tol=1e-9, max_iter=3000)
    r = _solve(atom_dir["zeeman_tiny_prd"], cols, _field_arrays(fields), precision=0, prd=1, **kw)
    assert np.all(r["status"] == 0)
    a = O.Atom(atom_dir["zeeman_tiny_prd"])
    for c in range(cols.n_columns):
        col = cols.column(c)
        ref = O.solve_column(a, col, prd=1, prd_lines=(1,), **kw)
        assert ref["n_iter"] == r["n_iter"][c]
        st = O.stokes_column(a, col, ref["pops"], 3, *fields[c], prd_rho=ref["rho"])
        _compare(r["stokes"][c], st, 1e-7, f"PRD column {c}")


def test_fp32_form_within_1e3(atom_dir):
    """The precision error alone: the FP32 form and the oracle both run 80
    iterations (no change test), and the Stokes vector of the FP32 form's
    populations (computed in FP64) is within 1e-3 of the oracle's.  The two
    columns converge by then (the oracle's change is below 3e-6 and its
    populations within 1e-5 of its 1e-10 answer); the third column of
    zeeman_columns still changes by 3e-4 per iteration at 80 iterations and
    is 0.8 % from its fixed point, where a comparison at a fixed count
    measures the trajectory rather than the precision."""
    cols, fields = zeeman_columns()
    cols, fields = cols.select([0, 1]), fields[:2]
    kw = dict(n_mu=3, tol=0.0, max_iter=80)
    r = _solve(atom_dir["zeeman_tiny"], cols, _field_arrays(fields), precision=1, scheduler=1, **kw)
    assert np.all(r["status"] == 1) and np.all(r["n_iter"] == 80)
    a = O.Atom(atom_dir["zeeman_tiny"])
    for c in range(cols.n_columns):
        col = cols.column(c)
        ref = O.solve_column(a, col, **kw)
        st = O.stokes_column(a, col, ref["pops"], 3, *fields[c])
        _compare(r["stokes"][c], st, 1e-3, f"FP32 column {c}")


def test_unusable_column_and_field(atom_dir):
    """A column with a NaN temperature: NaN Stokes (status BAD_INPUT); a
    column with a NaN field value: NaN Stokes but a converged solve; the
    columns between them as with no such neighbours."""
    rh = _rh()
    cols, fields = zeeman_columns(4)
    T = cols.T.copy()
    T[cols.offset[1] + 5] = np.nan
    cols_bad = synth.Columns(offset=cols.offset, z=cols.z, T=T, n_e=cols.n_e, n_H=cols.n_H, v_z=cols.v_z,
                             v_turb=cols.v_turb)
    B, inc, az = (x.copy() for x in _field_arrays(fields))
    inc[cols.offset[2] + 7] = np.inf
    kw = dict(precision=0, n_mu=3, tol=1e-8, max_iter=400)
    r = _solve(atom_dir["zeeman_tiny"], cols_bad, (B, inc, az), **kw)
    assert r["status"][1] == rh.BAD_INPUT and np.all(np.isnan(r["stokes"][1]))
    assert r["status"][2] == 0 and np.all(np.isnan(r["stokes"][2]))
    good = cols.select([0, 3])
    rg = _solve(atom_dir["zeeman_tiny"], good, _field_arrays([fields[0], fields[3]]), **kw)
    np.testing.assert_array_equal(r["stokes"][[0, 3]], rg["stokes"])


def cube_field(cols, seed=11):
    """Config-5 field: per column a strength uniform in 0-2 kG and an
    isotropic direction (cos of the inclination uniform in [-1, 1], azimuth
    uniform), constant along the column."""
    rng = np.random.default_rng(seed)
    n = cols.n_columns
    B = rng.uniform(0.0, 0.2, n)
    inc = np.arccos(rng.uniform(-1.0, 1.0, n))
    az = rng.uniform(0.0, 2.0 * np.pi, n)
    nd = np.diff(cols.offset)
    return tuple(np.repeat(x, nd) for x in (B, inc, az)), (B, inc, az)


def test_ca_like_atom_cube_columns(atom_dir):
    """Two synthetic-cube columns (their lowest 120 points) with the Ca
    II-like atom in complete redistribution: the split resonance lines in
    FP64 lock-step with the oracle."""
    base = synth.cube_columns(seed=4, nx=2, ny=2)
    parts = [{k: v[-120:] for k, v in base.column(c).items()} for c in (0, 3)]
    cols = synth.Columns.from_list(parts)
    field, per_col = cube_field(cols)
    kw = dict(n_mu=5, tol=1e-9, max_iter=300)
    r = _solve(atom_dir["ca2_crd"], cols, field, precision=0, **kw)
    assert np.all(r["status"] == 0)
    a = O.Atom(atom_dir["ca2_crd"])
    for c in range(cols.n_columns):
        col = cols.column(c)
        ref, rtol = conftest.oracle_lockstep_rtol(a, col, **kw)
        st = O.stokes_column(a, col, ref["pops"], 5, per_col[0][c], per_col[1][c], per_col[2][c])
        _compare(r["stokes"][c], st, max(rtol, 1e-10) * 10, f"Ca column {c}")
