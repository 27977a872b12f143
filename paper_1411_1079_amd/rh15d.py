"""Python binding of librh15d (ctypes over the C ABI in include/rh15d.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  If the
library is not built, importing this module raises; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librh15d.so")

FP64, FP32 = 0, 1
START_LTE, START_ZERO_RADIATION, START_PROVIDED, START_ESCAPE = 0, 1, 2, 3
SCHED_CHUNKED, SCHED_SLOTS = 0, 1
CONVERGED, MAX_ITER, NONFINITE, SINGULAR, BAD_INPUT = 0, 1, 2, 3, 4

EXPORTS = (
    "rh15d_load_atom", "rh15d_free_atom", "rh15d_atom_get_info", "rh15d_atom_lambda", "rh15d_default_options",
    "rh15d_workspace_size", "rh15d_solve_columns", "rh15d_last_error", "rh15d_last_stats",
    "rh15d_autotune", "rh15d_departures", "rh15d_pops_from_departures", "rh15d_mlp_create", "rh15d_mlp_free", "rh15d_mlp_n_params",
    "rh15d_mlp_get_params", "rh15d_mlp_set_params", "rh15d_mlp_get_grads", "rh15d_mlp_get_normalization",
    "rh15d_mlp_set_normalization", "rh15d_mlp_fit_normalization", "rh15d_mlp_features", "rh15d_mlp_forward",
    "rh15d_mlp_gradients", "rh15d_mlp_train_step", "rh15d_mlp_train_batches", "rh15d_solve_columns_static", "rh15d_static_workspace_bytes",
    "rh15d_default_grid_options", "rh15d_optimize_grid",
)


class AtomInfo(C.Structure):
    _fields_ = [("n_levels", C.c_int), ("n_lines", C.c_int), ("n_continua", C.c_int), ("n_transitions", C.c_int),
                ("n_lambda", C.c_int)]


class Columns(C.Structure):
    _fields_ = [("n_columns", C.c_int64), ("depth_offset", C.POINTER(C.c_int64))] + \
               [(n, C.c_void_p) for n in ("z", "T", "n_e", "n_H", "v_z", "v_turb", "init_pops", "B", "B_incl",
                                          "B_azim")]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("n_mu", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int),
                ("ng_order", C.c_int), ("ng_delay", C.c_int), ("ng_period", C.c_int), ("start", C.c_int),
                ("coll_scale", C.c_double), ("scheduler", C.c_int), ("batch_columns", C.c_int),
                ("profile", C.c_int), ("sweep_mc", C.c_int), ("sweep_pack", C.c_int), ("crs_f0", C.c_double),
                ("tol_fp", C.c_double), ("esc_iter", C.c_int), ("prd", C.c_int), ("prd_eps0", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("sweep_launches", C.c_int64), ("sweep_ms", C.c_double), ("se_ms", C.c_double),
                ("converge_ms", C.c_double), ("prep_ms", C.c_double), ("final_ms", C.c_double),
                ("total_ms", C.c_double), ("column_iterations", C.c_int64), ("ray_steps", C.c_int64),
                ("sweep_flops", C.c_double), ("sweep_bytes", C.c_double), ("graph_launches", C.c_int64)]


TUNE_MAX = 6


class TuneResult(C.Structure):
    _fields_ = [("sweep_mc", C.c_int), ("sweep_pack", C.c_int), ("n_candidates", C.c_int),
                ("cand_mc", C.c_int * TUNE_MAX), ("cand_pack", C.c_int * TUNE_MAX), ("ms", C.c_double * TUNE_MAX)]


class GridOptions(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("w_z", "w_T", "w_v", "w_tau")]


class GridOutput(C.Structure):
    _fields_ = [("depth_offset", C.POINTER(C.c_int64))] + \
        [(n, C.c_void_p) for n in ("z", "T", "n_e", "n_H", "v_z", "v_turb", "status")]


class Outputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("pops", "history", "n_iter", "status", "spectrum", "psi_star", "stokes",
                                          "psi_ray")]


_lib = None


def lib():
    """Load librh15d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() or "
                               "python paper_1411_1079_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.rh15d_load_atom.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
        L.rh15d_free_atom.argtypes = [C.c_void_p]
        L.rh15d_free_atom.restype = None
        L.rh15d_atom_get_info.argtypes = [C.c_void_p, C.POINTER(AtomInfo)]
        L.rh15d_atom_lambda.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        L.rh15d_default_options.argtypes = [C.POINTER(Options)]
        L.rh15d_workspace_size.argtypes = [C.c_void_p, C.POINTER(Columns), C.POINTER(Options), C.POINTER(C.c_size_t)]
        L.rh15d_solve_columns.argtypes = [C.c_void_p, C.POINTER(Columns), C.POINTER(Options), C.POINTER(Outputs),
                                          C.c_void_p, C.c_size_t, C.c_void_p]
        L.rh15d_last_error.restype = C.c_char_p
        L.rh15d_solve_columns_static.argtypes = [C.c_void_p, C.POINTER(Columns), C.POINTER(Options),
                                                 C.POINTER(Outputs), C.c_void_p]
        L.rh15d_static_workspace_bytes.argtypes = []
        L.rh15d_static_workspace_bytes.restype = C.c_size_t
        L.rh15d_last_stats.argtypes = [C.POINTER(Stats)]
        L.rh15d_default_grid_options.argtypes = [C.POINTER(GridOptions)]
        L.rh15d_optimize_grid.argtypes = [C.c_void_p, C.POINTER(Columns), C.POINTER(GridOptions),
                                          C.POINTER(GridOutput), C.c_void_p]
        vp, fp = C.c_void_p, C.POINTER(C.c_float)
        L.rh15d_autotune.argtypes = [vp, C.POINTER(Columns), C.POINTER(Options), vp, C.POINTER(TuneResult)]
        L.rh15d_departures.argtypes = [vp, C.POINTER(Columns), vp, vp, vp]
        L.rh15d_pops_from_departures.argtypes = [vp, C.POINTER(Columns), vp, C.c_double, vp, vp]
        L.rh15d_mlp_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, C.POINTER(vp)]
        L.rh15d_mlp_free.argtypes = [vp]
        L.rh15d_mlp_free.restype = None
        L.rh15d_mlp_n_params.argtypes = [vp, C.POINTER(C.c_int64)]
        L.rh15d_mlp_get_params.argtypes = [vp, fp]
        L.rh15d_mlp_set_params.argtypes = [vp, fp]
        L.rh15d_mlp_get_grads.argtypes = [vp, fp]
        L.rh15d_mlp_get_normalization.argtypes = [vp, fp, fp]
        L.rh15d_mlp_set_normalization.argtypes = [vp, fp, fp]
        L.rh15d_mlp_fit_normalization.argtypes = [vp, vp, C.c_int64, vp]
        L.rh15d_mlp_features.argtypes = [C.POINTER(Columns), vp, C.c_int64, vp, vp]
        L.rh15d_mlp_forward.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.rh15d_mlp_gradients.argtypes = [vp, vp, vp, C.c_int64, fp, vp]
        L.rh15d_mlp_train_step.argtypes = [vp, vp, vp, C.c_int64, C.c_float, fp, vp]
        L.rh15d_mlp_train_batches.argtypes = [vp, vp, vp, C.c_int64, C.c_int, fp, vp, vp]
        _lib = L
    return _lib


class RH15DError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librh15d error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise RH15DError(rc, lib().rh15d_last_error().decode())


class Atom:
    """A model atom loaded by the library (rh15d_load_atom)."""

    def __init__(self, path: str):
        h = C.c_void_p()
        _check(lib().rh15d_load_atom(path.encode(), C.byref(h)))
        self._h = h
        info = AtomInfo()
        _check(lib().rh15d_atom_get_info(h, C.byref(info)))
        self.n_levels, self.n_lines, self.n_continua = info.n_levels, info.n_lines, info.n_continua
        self.n_transitions, self.n_lambda = info.n_transitions, info.n_lambda
        self.lam = np.empty(self.n_lambda)
        _check(lib().rh15d_atom_lambda(h, self.lam.ctypes.data_as(C.POINTER(C.c_double))))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.rh15d_free_atom(self._h)
            self._h = None


def last_stats() -> dict:
    """Measurements of this thread's last solve: times and work counts when
    it ran with profile=1, graph_launches always."""
    st = Stats()
    _check(lib().rh15d_last_stats(C.byref(st)))
    return {name: getattr(st, name) for name, _ in Stats._fields_}


def default_options(**kw) -> Options:
    o = Options()
    _check(lib().rh15d_default_options(C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


@dataclass
class DeviceColumns:
    """Columns resident on the device: CSR offsets on the host, per-depth
    fields as float64 CUDA tensors."""
    offset: np.ndarray
    z: object
    T: object
    n_e: object
    n_H: object
    v_z: object
    v_turb: object
    init_pops: object = None
    B: object = None          # magnetic field strength [T], inclination and azimuth [rad] (all or none)
    B_incl: object = None
    B_azim: object = None

    @property
    def n_columns(self):
        return len(self.offset) - 1

    @property
    def total_depth(self):
        return int(self.offset[-1])

    @staticmethod
    def from_host(cols, device="cuda", init_pops=None, field=None):
        """field: None or (B, B_incl, B_azim) host arrays [total_depth]."""
        import torch
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(device)
        f = (None, None, None) if field is None else tuple(t(x) for x in field)
        return DeviceColumns(offset=np.ascontiguousarray(cols.offset, dtype=np.int64), z=t(cols.z), T=t(cols.T),
                             n_e=t(cols.n_e), n_H=t(cols.n_H), v_z=t(cols.v_z), v_turb=t(cols.v_turb),
                             init_pops=None if init_pops is None else t(init_pops), B=f[0], B_incl=f[1], B_azim=f[2])


def _cols_struct(dc: DeviceColumns) -> Columns:
    off = dc.offset
    s = Columns()
    s.n_columns = dc.n_columns
    s.depth_offset = off.ctypes.data_as(C.POINTER(C.c_int64))
    for n in ("z", "T", "n_e", "n_H", "v_z", "v_turb"):
        ten = getattr(dc, n)
        assert ten.dtype.is_floating_point and ten.element_size() == 8 and ten.is_contiguous()
        setattr(s, n, ten.data_ptr())
    s.init_pops = dc.init_pops.data_ptr() if dc.init_pops is not None else None
    for n in ("B", "B_incl", "B_azim"):
        ten = getattr(dc, n, None)
        if ten is not None:
            assert ten.dtype.is_floating_point and ten.element_size() == 8 and ten.is_contiguous()
        setattr(s, n, ten.data_ptr() if ten is not None else None)
    return s


def static_workspace_bytes() -> int:
    """Size of the library's fixed workspace region per device."""
    return int(lib().rh15d_static_workspace_bytes())


def workspace_size(atom: Atom, dc: DeviceColumns, opts: Options) -> int:
    n = C.c_size_t()
    _check(lib().rh15d_workspace_size(atom._h, C.byref(_cols_struct(dc)), C.byref(opts), C.byref(n)))
    return n.value


class Solver:
    """Reusable output and workspace buffers for repeated solves."""

    def __init__(self, atom: Atom, dc: DeviceColumns, opts: Options, want_spectrum=True, want_psi=False,
                 want_history=True, workspace=None, want_stokes=False, want_psi_ray=False):
        import torch
        self.atom, self.dc, self.opts = atom, dc, opts
        dev = dc.z.device
        L, n = atom.n_levels, dc.n_columns
        self.pops = torch.empty((dc.total_depth, L), dtype=torch.float64, device=dev)
        self.history = torch.empty((n, max(opts.max_iter, 1)), dtype=torch.float64, device=dev) if want_history else None
        self.n_iter = torch.empty(n, dtype=torch.int32, device=dev)
        self.status = torch.empty(n, dtype=torch.int32, device=dev)
        self.spectrum = torch.empty((n, atom.n_lambda), dtype=torch.float64, device=dev) if want_spectrum else None
        self.psi_star = (torch.empty((dc.total_depth, atom.n_transitions), dtype=torch.float64, device=dev)
                         if want_psi else None)
        self.stokes = torch.empty((n, atom.n_lambda, 4), dtype=torch.float64, device=dev) if want_stokes else None
        self.psi_ray = (torch.empty((dc.total_depth, atom.n_lambda, opts.n_mu, 2), dtype=torch.float64, device=dev)
                        if want_psi_ray else None)
        self.ws_bytes = workspace_size(atom, dc, opts)
        if workspace is None:
            workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        elif workspace.numel() < self.ws_bytes + 256:
            raise ValueError(f"workspace of {workspace.numel()} bytes < {self.ws_bytes + 256}")
        self.workspace = workspace
        self._cols = _cols_struct(dc)
        self._out = Outputs()
        for name in ("pops", "history", "n_iter", "status", "spectrum", "psi_star", "stokes", "psi_ray"):
            ten = getattr(self, name)
            setattr(self._out, name, ten.data_ptr() if ten is not None else None)

    def run(self, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(self.dc.z.device)
        ws = self.workspace.data_ptr()
        ws_al = (ws + 255) & ~255
        _check(lib().rh15d_solve_columns(self.atom._h, C.byref(self._cols), C.byref(self.opts), C.byref(self._out),
                                         C.c_void_p(ws_al), self.ws_bytes, C.c_void_p(st.cuda_stream)))
        return self

    def run_static(self, stream=None):
        """The same solve through rh15d_solve_columns_static: the library's
        fixed device region as workspace, nothing allocated."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(self.dc.z.device)
        _check(lib().rh15d_solve_columns_static(self.atom._h, C.byref(self._cols), C.byref(self.opts),
                                                C.byref(self._out), C.c_void_p(st.cuda_stream)))
        return self

    def result(self) -> dict:
        out = dict(pops=self.pops, n_iter=self.n_iter, status=self.status)
        if self.history is not None:
            out["history"] = self.history
        if self.spectrum is not None:
            out["spectrum"] = self.spectrum
        if self.psi_star is not None:
            out["psi_star"] = self.psi_star
        if self.stokes is not None:
            out["stokes"] = self.stokes
        if self.psi_ray is not None:
            out["psi_ray"] = self.psi_ray
        return out


def resolve_failed(atom: Atom, dc: DeviceColumns, out: dict, opts: Options, stream=None) -> int:
    """Solve again, with the option set `opts`, every column of `dc` whose
    status in the result `out` (the dict of CUDA tensors that solve() or
    Solver.result() returns) is not converged, and write the new results
    into `out`.  The paper's code re-runs failed columns with other options
    (Sec. 2.3, convergence aids); here any option set can serve, e.g. the
    LTE start, collisional-radiative switching or a larger iteration limit.
    n_iter then counts the iterations of both attempts, and the history row
    of such a column holds the first attempt's changes followed by the
    second attempt's, as far as the row's width allows.  Columns with
    unusable data (status BAD_INPUT) are not solved again.  Every step runs
    on `stream` (default: the current stream).  Returns the number of
    columns solved again (a host synchronisation)."""
    import torch
    dev = dc.z.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    with torch.cuda.stream(st):
        status = out["status"]
        bad = torch.nonzero((status != CONVERGED) & (status != BAD_INPUT)).flatten().cpu().numpy()
        if bad.size == 0:
            return 0
        off = dc.offset
        lens = np.diff(off)[bad]
        idx = np.concatenate([np.arange(off[c], off[c + 1]) for c in bad])
        it = torch.as_tensor(idx, dtype=torch.int64, device=dev)
        fields = {k: torch.index_select(getattr(dc, k), 0, it) for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
        init = None
        if opts.start == START_PROVIDED:
            if dc.init_pops is None:
                raise ValueError("a provided start needs the columns' init_pops")
            init = torch.index_select(dc.init_pops, 0, it)
        if dc.B is not None:
            for k in ("B", "B_incl", "B_azim"):
                fields[k] = torch.index_select(getattr(dc, k), 0, it)
        sub = DeviceColumns(offset=np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), init_pops=init, **fields)
        r = Solver(atom, sub, opts, want_spectrum=out.get("spectrum") is not None,
                   want_psi=out.get("psi_star") is not None, want_history=out.get("history") is not None,
                   want_stokes=out.get("stokes") is not None, want_psi_ray=out.get("psi_ray") is not None).run(st)
        cb = torch.as_tensor(bad, dtype=torch.int64, device=dev)
        out["pops"].index_copy_(0, it, r.pops)
        if out.get("psi_star") is not None:
            out["psi_star"].index_copy_(0, it, r.psi_star)
        if out.get("spectrum") is not None:
            out["spectrum"].index_copy_(0, cb, r.spectrum)
        if out.get("stokes") is not None:
            out["stokes"].index_copy_(0, cb, r.stokes)
        if out.get("psi_ray") is not None:
            out["psi_ray"].index_copy_(0, it, r.psi_ray)
        n1 = out["n_iter"].index_select(0, cb)
        if out.get("history") is not None:
            # the first attempt's n1 entries, then the second attempt's
            h = out["history"]
            rows = h.index_select(0, cb)
            for i, n in enumerate(n1.cpu().tolist()):
                w = min(h.shape[1] - n, r.history.shape[1])
                if w > 0:
                    rows[i, n:n + w] = r.history[i, :w]
            h.index_copy_(0, cb, rows)
        out["n_iter"].index_copy_(0, cb, n1 + r.n_iter)
        out["status"].index_copy_(0, cb, r.status)
    return int(bad.size)


def solve(atom: Atom, dc: DeviceColumns, want_spectrum=True, want_psi=False, want_stokes=False, **opts) -> dict:
    """Solve every column; returns CUDA tensors (pops, history, n_iter,
    status, spectrum, psi_star, stokes)."""
    o = default_options(**opts)
    return Solver(atom, dc, o, want_spectrum=want_spectrum, want_psi=want_psi, want_stokes=want_stokes).run().result()


def autotune(atom: Atom, dc: DeviceColumns, stream=None, **opts) -> dict:
    """Time every formal-solution shape on the columns dc (solved twice
    each) and keep the fastest for later solves with automatic shape."""
    o = default_options(**opts)
    r = TuneResult()
    _check(lib().rh15d_autotune(atom._h, C.byref(_cols_struct(dc)), C.byref(o), _stream(stream), C.byref(r)))
    n = r.n_candidates
    return dict(sweep_mc=r.sweep_mc, sweep_pack=r.sweep_pack,
                candidates=[dict(sweep_mc=r.cand_mc[i], sweep_pack=r.cand_pack[i], ms=r.ms[i]) for i in range(n)])


def _stream(stream=None):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(st.cuda_stream)


def default_grid_options(**kw) -> GridOptions:
    o = GridOptions()
    _check(lib().rh15d_default_grid_options(C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def optimize_grid(atom: Atom, dc: DeviceColumns, n_out, stream=None, **weights):
    """Re-grid every column (rh15d_optimize_grid): n_out is one point count
    for all columns or one per column.  Returns (DeviceColumns of the new
    grids, per-column status tensor)."""
    import torch
    n = dc.n_columns
    counts = np.broadcast_to(np.asarray(n_out, dtype=np.int64), (n,))
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    dev = dc.z.device
    new = {k: torch.empty(int(off[-1]), dtype=torch.float64, device=dev)
           for k in ("z", "T", "n_e", "n_H", "v_z", "v_turb")}
    status = torch.empty(n, dtype=torch.int32, device=dev)
    o = GridOutput()
    o.depth_offset = off.ctypes.data_as(C.POINTER(C.c_int64))
    for k, t in new.items():
        setattr(o, k, t.data_ptr())
    o.status = status.data_ptr()
    opts = default_grid_options(**weights)
    _check(lib().rh15d_optimize_grid(atom._h, C.byref(_cols_struct(dc)), C.byref(opts), C.byref(o), _stream(stream)))
    return DeviceColumns(offset=off, **new), status


def departures(atom: Atom, dc: DeviceColumns, pops, out=None, stream=None):
    """ln(n_i / n*_i) of populations pops (CUDA float64 [total_depth][L])."""
    import torch
    if out is None:
        out = torch.empty((dc.total_depth, atom.n_levels), dtype=torch.float32, device=pops.device)
    assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == dc.total_depth * atom.n_levels
    assert pops.dtype == torch.float64 and pops.is_contiguous() and pops.numel() == out.numel()
    _check(lib().rh15d_departures(atom._h, C.byref(_cols_struct(dc)), C.c_void_p(pops.data_ptr()),
                                  C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def pops_from_departures(atom: Atom, dc: DeviceColumns, log_b, shrink=0.0, out=None, stream=None):
    """Start populations n_i = exp(l_i) n*_i renormalised per point, l_i =
    log_b_i shrunk toward 0 by `shrink` (non-finite predictions give LTE,
    others are clamped to |ln b| <= 50 first)."""
    import torch
    if out is None:
        out = torch.empty((dc.total_depth, atom.n_levels), dtype=torch.float64, device=log_b.device)
    assert log_b.dtype == torch.float32 and log_b.is_contiguous() and log_b.numel() == dc.total_depth * atom.n_levels
    assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == log_b.numel()
    _check(lib().rh15d_pops_from_departures(atom._h, C.byref(_cols_struct(dc)), C.c_void_p(log_b.data_ptr()),
                                            float(shrink), C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


N_FEATURES = 36


class MLP:
    """The start-solution network (rh15d_mlp_*): 36 -> n_layers x n_hidden
    (SiLU) -> n_out, trained and evaluated by the library's kernels."""

    def __init__(self, n_hidden=256, n_layers=3, n_out=6, seed=0):
        h = C.c_void_p()
        _check(lib().rh15d_mlp_create(n_hidden, n_layers, n_out, seed, C.byref(h)))
        self._h = h
        self.n_hidden, self.n_layers, self.n_out = n_hidden, n_layers, n_out
        n = C.c_int64()
        _check(lib().rh15d_mlp_n_params(h, C.byref(n)))
        self.n_params = n.value

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.rh15d_mlp_free(self._h)
            self._h = None

    def get_params(self) -> np.ndarray:
        a = np.empty(self.n_params, dtype=np.float32)
        _check(lib().rh15d_mlp_get_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float))))
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        assert a.size == self.n_params
        _check(lib().rh15d_mlp_set_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float))))

    def get_grads(self) -> np.ndarray:
        a = np.empty(self.n_params, dtype=np.float32)
        _check(lib().rh15d_mlp_get_grads(self._h, a.ctypes.data_as(C.POINTER(C.c_float))))
        return a

    def get_normalization(self):
        m, s = np.empty(N_FEATURES, np.float32), np.empty(N_FEATURES, np.float32)
        _check(lib().rh15d_mlp_get_normalization(self._h, m.ctypes.data_as(C.POINTER(C.c_float)),
                                                 s.ctypes.data_as(C.POINTER(C.c_float))))
        return m, s

    def set_normalization(self, mean, std):
        m = np.ascontiguousarray(mean, np.float32)
        s = np.ascontiguousarray(std, np.float32)
        _check(lib().rh15d_mlp_set_normalization(self._h, m.ctypes.data_as(C.POINTER(C.c_float)),
                                                 s.ctypes.data_as(C.POINTER(C.c_float))))

    def fit_normalization(self, feats, stream=None):
        _check(lib().rh15d_mlp_fit_normalization(self._h, C.c_void_p(feats.data_ptr()), feats.shape[0],
                                                 _stream(stream)))

    @staticmethod
    def features(dc: DeviceColumns, samples=None, out=None, stream=None):
        """Raw stencil features (CUDA float32 [n][36]) of sample points
        (CUDA int64 global depth indices) or of every point."""
        import torch
        n = dc.total_depth if samples is None else samples.numel()
        if samples is not None:
            assert samples.dtype == torch.int64 and samples.is_contiguous()
        if out is None:
            out = torch.empty((n, N_FEATURES), dtype=torch.float32, device=dc.z.device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == n * N_FEATURES
        _check(lib().rh15d_mlp_features(C.byref(_cols_struct(dc)),
                                        C.c_void_p(samples.data_ptr()) if samples is not None else None,
                                        n, C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def forward(self, feats, out=None, stream=None):
        import torch
        assert feats.dtype == torch.float32 and feats.is_contiguous() and feats.shape[-1] == N_FEATURES
        n = feats.shape[0]
        if out is None:
            out = torch.empty((n, self.n_out), dtype=torch.float32, device=feats.device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == n * self.n_out
        _check(lib().rh15d_mlp_forward(self._h, C.c_void_p(feats.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                       _stream(stream)))
        return out

    def _check_batch(self, feats, target):
        import torch
        assert feats.dtype == torch.float32 and feats.is_contiguous() and feats.shape[-1] == N_FEATURES
        assert target.dtype == torch.float32 and target.is_contiguous()
        assert target.numel() == feats.shape[0] * self.n_out

    def gradients(self, feats, target, stream=None) -> float:
        self._check_batch(feats, target)
        loss = C.c_float()
        _check(lib().rh15d_mlp_gradients(self._h, C.c_void_p(feats.data_ptr()), C.c_void_p(target.data_ptr()),
                                         feats.shape[0], C.byref(loss), _stream(stream)))
        return loss.value

    def train_step(self, feats, target, lr, want_loss=False, stream=None):
        self._check_batch(feats, target)
        loss = C.c_float()
        _check(lib().rh15d_mlp_train_step(self._h, C.c_void_p(feats.data_ptr()), C.c_void_p(target.data_ptr()),
                                          feats.shape[0], float(lr), C.byref(loss) if want_loss else None,
                                          _stream(stream)))
        return loss.value if want_loss else None

    def train_batches(self, feats, target, batch, lrs, losses=None, stream=None):
        """Adam steps on consecutive batches of `batch` rows of feats/target,
        step b with learning rate lrs[b]: the same as one train_step per
        batch, replayed from one captured step.  losses (CUDA float32
        [len(lrs)], optional) receives every step's loss."""
        import torch
        n = len(lrs)
        assert feats.dtype == torch.float32 and feats.is_contiguous() and feats.shape[-1] == N_FEATURES
        assert target.dtype == torch.float32 and target.is_contiguous()
        assert feats.shape[0] >= n * batch and target.numel() >= n * batch * self.n_out
        assert losses is None or (losses.dtype == torch.float32 and losses.is_cuda and losses.numel() >= n)
        lr = (C.c_float * max(n, 1))(*[float(x) for x in lrs])
        _check(lib().rh15d_mlp_train_batches(self._h, C.c_void_p(feats.data_ptr()), C.c_void_p(target.data_ptr()),
                                             int(batch), n, lr,
                                             C.c_void_p(losses.data_ptr()) if losses is not None else None,
                                             _stream(stream)))
