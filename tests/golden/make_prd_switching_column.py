"""Writes prd_switching_column.json: the oracle's solve of one column of the
64 x 64 synthetic cube (seed 1, column 1959, 200 depth points) with the
Ca II-like atom, both resonance lines in angle-averaged partial frequency
redistribution (Sec. 2.1), 5 angles, the change test 1e-4 with the
fixed-point bound 1e-4: without PRD switching the iteration breaks down
(non-finite rates, status 2) at iteration 41; with the switching of
Sec. 2.3, Eq. 1 (eps0 = 0.01) it converges.

Run from the repository root:  python3 tests/golden/make_prd_switching_column.py
It calls only the oracle and the input generator."""
import json
import os
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_1411_1079_amd import synth  # noqa: E402

COLUMN = 1959
OPTS = dict(n_mu=5, tol=1e-4, tol_fp=1e-4, prd=1, prd_lines=(0, 1))
EPS0 = 0.01


def column():
    return synth.cube_columns(1, 64, 64).column(COLUMN)


def main():
    atoms = synth.write_atoms(tempfile.mkdtemp())
    a = O.Atom(atoms["ca2"])
    col = column()
    plain = O.solve_column(a, col, max_iter=60, **OPTS)
    sw = O.solve_column(a, col, max_iter=400, prd_eps0=EPS0, **OPTS)
    out = dict(column=COLUMN, options={k: list(v) if isinstance(v, tuple) else v for k, v in OPTS.items()},
               eps0=EPS0,
               plain=dict(n_iter=plain["n_iter"], status=plain["status"],
                          history=[float(x) for x in plain["history"][:plain["n_iter"] - 1]]),
               switching=dict(n_iter=sw["n_iter"], status=sw["status"], pops=sw["pops"].tolist(),
                              spectrum=sw["spectrum"].tolist()))
    with open(os.path.join(HERE, "prd_switching_column.json"), "w") as f:
        json.dump(out, f)
    print("plain", plain["n_iter"], plain["status"], "switching", sw["n_iter"], sw["status"])


if __name__ == "__main__":
    main()
