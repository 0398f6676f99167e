"""Python binding of libmpr (include/mpr.h): argument marshalling only.

Every computation runs in the library's HIP kernels (or, for mpr_match_T,
its native host code).  PyTorch provides device memory and the stream.
Importing this module loads libmpr.so built in place by
``python -m paper_1710_03038_amd.build``; it raises if the library is
missing: there is no fallback.
"""
import ctypes
import math
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MPR_LIB") or os.path.join(HERE, "libmpr.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mpr.h")

MPR_OK, MPR_E_ARG, MPR_E_SHAPE, MPR_E_DEGENERATE, MPR_E_NOPAIRS, MPR_E_RANGE, \
    MPR_E_WORKSPACE, MPR_E_HIP, MPR_E_STATE = range(9)
STATUS_NAMES = ["MPR_OK", "MPR_E_ARG", "MPR_E_SHAPE", "MPR_E_DEGENERATE", "MPR_E_NOPAIRS",
                "MPR_E_RANGE", "MPR_E_WORKSPACE", "MPR_E_HIP", "MPR_E_STATE"]
FP32, FP64 = 0, 1
MODEL_MPR, MODEL_GMRF = 0, 1
BC_OPEN, BC_REPLICATE = 0, 1
ADAPT, TRACE_E, NO_OR = 1, 2, 4
SAMPLE_PAIRS, STATE = 0, 1


class MPRError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 9 else status}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("a_targ", ctypes.c_double), ("k_a", ctypes.c_double),
                ("adapt_every", ctypes.c_int32), ("a_sample_keep", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("sweeps_per_pass", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("model", ctypes.c_int32), ("boundary", ctypes.c_int32)]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("chains", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("z", ctypes.c_void_p), ("known", ctypes.c_void_p)]


class FillReport(ctypes.Structure):
    _fields_ = [("records", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("a_eq", ctypes.c_void_p), ("acc_eq", ctypes.c_void_p), ("acc_samp", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libmpr.so (ctypes.CDLL).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch first: libmpr.so then binds to the HIP runtime torch has
        # loaded, so both share one runtime, device list and streams.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1710_03038_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        L.mpr_default_params.argtypes = [ctypes.POINTER(Params)]
        L.mpr_default_params.restype = None
        L.mpr_init_field.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Grid), i32, ctypes.POINTER(Params), vp,
                                     ctypes.POINTER(ctypes.c_size_t), vp]
        L.mpr_sweep.argtypes = [vp, i32, dp, u32, vp]
        L.mpr_specific_energy.argtypes = [vp, i32, dp, ctypes.POINTER(i64)]
        L.mpr_match_T.argtypes = [dp, i32, dp, dp, i32, dp, ctypes.POINTER(i32)]
        L.mpr_fill.argtypes = [vp, dp, i32, i32, i32, vp, vp, ctypes.POINTER(FillReport)]
        L.mpr_get_phi.argtypes = [vp, i32, i32, vp]
        L.mpr_set_phi.argtypes = [vp, i32, i32, vp]
        L.mpr_get_chain_state.argtypes = [vp, ctypes.POINTER(i64), dp]
        L.mpr_set_chain_state.argtypes = [vp, i64, dp]
        L.mpr_autotune.argtypes = [vp, dp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32)]
        L.mpr_reinit.argtypes = [vp]
        L.mpr_set_launch_shape.argtypes = [vp, i32, i32, i32, i32]
        L.mpr_validation_measures.argtypes = [vp, i32, vp, vp, dp]
        L.mpr_validation_measures_static.argtypes = [vp, vp, vp, i64, ctypes.c_double, vp, vp]
        L.mpr_equilibrate.argtypes = [vp, dp, i32, i32, i32, u32, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.mpr_set_graph.argtypes = [vp, i32]
        L.mpr_set_grid_q.argtypes = [vp, dp]
        L.mpr_cv_select_q.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Params), vp, i32, dp, i32,
                                      ctypes.POINTER(dp), ctypes.POINTER(dp), ctypes.POINTER(i32), i32, i32, i32,
                                      vp, ctypes.POINTER(ctypes.c_size_t), vp, dp, ctypes.POINTER(i32)]
        L.mpr_autotune_tile.argtypes = [ctypes.POINTER(Grid), i32, ctypes.POINTER(Params), dp, i32, i32, i32, vp,
                                        ctypes.POINTER(ctypes.c_size_t), vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i32)]
        L.mpr_set_timing.argtypes = [vp, i32]
        L.mpr_get_timing.argtypes = [vp, dp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.mpr_destroy.argtypes = [vp]
        L.mpr_destroy.restype = None
        L.mpr_last_error.argtypes = [vp]
        L.mpr_last_error.restype = ctypes.c_char_p
        for name in ("mpr_init_field", "mpr_sweep", "mpr_specific_energy", "mpr_match_T", "mpr_fill",
                     "mpr_get_phi", "mpr_set_phi", "mpr_get_chain_state", "mpr_set_chain_state",
                     "mpr_set_timing", "mpr_get_timing", "mpr_autotune", "mpr_autotune_tile"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions(path=HEADER):
    """Names of the functions declared in include/mpr.h."""
    with open(path) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:mpr_status|void|const char \*)\s*(mpr_\w+)\s*\(", text, re.M)))


def _check(status, ctx=None):
    if status != MPR_OK:
        msg = lib().mpr_last_error(ctx).decode()
        raise MPRError(status, msg)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default_params(**overrides):
    p = Params()
    lib().mpr_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if k == "dtype" and isinstance(v, str):
            v = {"fp32": FP32, "fp64": FP64}[v]
        if k == "model" and isinstance(v, str):
            v = {"mpr": MODEL_MPR, "gmrf": MODEL_GMRF}[v]
        if k == "boundary" and isinstance(v, str):
            v = {"open": BC_OPEN, "replicate": BC_REPLICATE}[v]
        setattr(p, k, v)
    return p


STATIC_MAX_SITES = 26214 * 4096


def validation_measures_static(z_true, zhat, known, shift, out, stream=None):
    """mpr_validation_measures_static: the eight validation measures of
    z_true, zhat (device float64) over the sites where known (device uint8)
    is 0, written asynchronously into the device tensor out (8 float64s)
    on the library's static scratch; nothing is allocated."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    n = z_true.numel()
    if zhat.numel() != n or known.numel() != n or out.numel() < 8:
        raise ValueError("z_true, zhat and known need one value per site; out needs 8")
    if z_true.dtype != torch.float64 or zhat.dtype != torch.float64 or out.dtype != torch.float64 \
            or known.dtype != torch.uint8:
        raise ValueError("z_true, zhat, out must be float64 and known uint8")
    _check(lib().mpr_validation_measures_static(ctypes.c_void_p(z_true.data_ptr()), ctypes.c_void_p(zhat.data_ptr()),
                                                ctypes.c_void_p(known.data_ptr()), n, float(shift),
                                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))
    return out


def match_T(e_s, tab_T, tab_e, raise_on_range=False):
    """Specific energy matching on a table (mpr_match_T).  Returns (T, status)."""
    e_s = np.ascontiguousarray(np.atleast_1d(e_s), dtype=np.float64)
    tab_T = np.ascontiguousarray(tab_T, dtype=np.float64)
    tab_e = np.ascontiguousarray(tab_e, dtype=np.float64)
    T = np.empty_like(e_s)
    st = np.zeros(e_s.shape, dtype=np.int32)
    rc = lib().mpr_match_T(_dptr(e_s), len(e_s), _dptr(tab_T), _dptr(tab_e), len(tab_T), _dptr(T),
                           st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc not in (MPR_OK, MPR_E_RANGE) or (rc == MPR_E_RANGE and raise_on_range):
        _check(rc)
    return T, st


def workspace_bytes(shapes, params):
    """Workspace needed for grids given as (ny, nx, chains) tuples."""
    gs = (Grid * len(shapes))()
    for g, (ny, nx, ch) in zip(gs, shapes):
        g.nx, g.ny, g.chains, g.reserved = nx, ny, ch, 0
    n = ctypes.c_size_t(0)
    _check(lib().mpr_init_field(None, gs, len(shapes), ctypes.byref(params), None, ctypes.byref(n), None))
    return n.value


def cv_select_q(z, known, fold, n_folds, qs, tables, n_eq, n_samp, stride, params=None, chains=1, stream=None):
    """mpr_cv_select_q: choose q by K-fold cross-validation.

    z (float64), known (uint8), fold (uint8): CUDA tensors (ny, nx); fold
    holds each sample site's fold id.  qs: candidates in (0, 0.5]; tables:
    per candidate (tab_T, tab_e).  Returns dict(aae, rase, T_mean (arrays
    per candidate), best (index), q (the chosen q))."""
    import torch

    params = params if params is not None else default_params()
    z = z.contiguous().to(torch.float64)
    known = known.contiguous().to(torch.uint8)
    fold = fold.contiguous().to(torch.uint8)
    if not (z.is_cuda and known.is_cuda and fold.is_cuda):
        raise ValueError("z, known and fold must be CUDA tensors")
    if z.shape != known.shape or z.shape != fold.shape or z.dim() != 2:
        raise ValueError("z, known and fold must be 2-D tensors of one shape")
    g = Grid()
    g.ny, g.nx = z.shape
    g.chains, g.reserved = int(chains), 0
    g.z, g.known = z.data_ptr(), known.data_ptr()
    nq = len(qs)
    q = np.ascontiguousarray(qs, dtype=np.float64)
    tabs = [(np.ascontiguousarray(t, dtype=np.float64), np.ascontiguousarray(e, dtype=np.float64)) for t, e in tables]
    if len(tabs) != nq:
        raise ValueError("one table per candidate")
    dp = ctypes.POINTER(ctypes.c_double)
    tT = (dp * nq)(*[_dptr(t) for t, _ in tabs])
    tE = (dp * nq)(*[_dptr(e) for _, e in tabs])
    nT = (ctypes.c_int32 * nq)(*[len(t) for t, _ in tabs])
    stream = stream if stream is not None else torch.cuda.current_stream(z.device)
    L = lib()
    n = ctypes.c_size_t(0)
    best = ctypes.c_int32(-1)
    args = (tT, tE, nT, int(n_eq), int(n_samp), int(stride))
    _check(L.mpr_cv_select_q(ctypes.byref(g), ctypes.byref(params), ctypes.c_void_p(fold.data_ptr()), int(n_folds),
                             _dptr(q), nq, *args, None, ctypes.byref(n), None, None, ctypes.byref(best)))
    ws = torch.empty(n.value + 256, dtype=torch.uint8, device=z.device)
    aligned = (ws.data_ptr() + 255) // 256 * 256
    score = np.empty(3 * nq)
    _check(L.mpr_cv_select_q(ctypes.byref(g), ctypes.byref(params), ctypes.c_void_p(fold.data_ptr()), int(n_folds),
                             _dptr(q), nq, *args, ctypes.c_void_p(aligned), ctypes.byref(n),
                             ctypes.c_void_p(stream.cuda_stream), _dptr(score), ctypes.byref(best)))
    sc = score.reshape(nq, 3)
    return dict(aae=sc[:, 0].copy(), rase=sc[:, 1].copy(), T_mean=sc[:, 2].copy(), best=int(best.value),
                q=float(q[best.value]))


def _grid_array(grids):
    """ctypes mpr_grid[] for (z, known, chains) CUDA tensors, and the
    converted tensors to keep alive while it is used."""
    import torch

    gs = (Grid * len(grids))()
    keep = []
    for g, (z, known, chains) in zip(gs, grids):
        if not (z.is_cuda and known.is_cuda):
            raise ValueError("z and known must be CUDA tensors")
        z = z.contiguous().to(torch.float64)
        known = known.contiguous().to(torch.uint8)
        if z.shape != known.shape or z.dim() != 2:
            raise ValueError("z and known must be 2-D tensors of one shape")
        ny, nx = z.shape
        g.nx, g.ny, g.chains, g.reserved = nx, ny, int(chains), 0
        g.z, g.known = z.data_ptr(), known.data_ptr()
        keep += [z, known]
    return gs, keep


def autotune_tile(grids, T, n_eq, n_samp, params=None, trial_sweeps=16, stream=None):
    """mpr_autotune_tile: the tile shape and sweeps per pass to build a
    Field of these grids with.  grids as for Field; T: per-grid
    temperatures.  Returns (tile_x, tile_y, sweeps_per_pass)."""
    import torch

    params = params if params is not None else default_params()
    if not grids:
        raise ValueError("need at least one grid")
    gs, keep = _grid_array(grids)
    dev = keep[0].device
    T = np.ascontiguousarray(np.broadcast_to(np.asarray(T, dtype=np.float64), (len(grids),)))
    stream = stream if stream is not None else torch.cuda.current_stream(dev)
    L = lib()
    n = ctypes.c_size_t(0)
    args = (gs, len(grids), ctypes.byref(params), _dptr(T), int(n_eq), int(n_samp), int(trial_sweeps))
    _check(L.mpr_autotune_tile(*args, None, ctypes.byref(n), None, None, None, None))
    ws = torch.empty(n.value + 256, dtype=torch.uint8, device=dev)
    aligned = (ws.data_ptr() + 255) // 256 * 256
    tx, ty, nsw = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(L.mpr_autotune_tile(*args, ctypes.c_void_p(aligned), ctypes.byref(n), ctypes.c_void_p(stream.cuda_stream),
                               ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(nsw)))
    del ws, keep
    return tx.value, ty.value, nsw.value


class Field:
    """A batch of gappy grids under simulation: one mpr_ctx and its workspace.

    grids: list of (z, known, chains) with z a CUDA float64 tensor (ny, nx)
    and known a CUDA uint8 tensor (ny, nx).  The tensors are kept alive
    with the context.
    """

    def __init__(self, grids, params=None, stream=None):
        import torch

        self._torch = torch
        self.params = params if params is not None else default_params()
        if not grids:
            raise ValueError("need at least one grid")
        gs, self._keep = _grid_array(grids)
        self.shapes = [(g.ny, g.nx, g.chains) for g in gs]
        dev = self._keep[0].device
        self.device = dev
        self.n_grids = len(grids)
        self.total_chains = sum(s[2] for s in self.shapes)
        # runs of consecutive grids of one shape: (offset, count, ny, nx),
        # so that per-grid result views are cut run by run
        self._runs, off = [], 0
        for ny, nx, _ in self.shapes:
            if self._runs and self._runs[-1][2:] == (ny, nx):
                o, n, _, _ = self._runs[-1]
                self._runs[-1] = (o, n + 1, ny, nx)
            else:
                self._runs.append((off, 1, ny, nx))
            off += ny * nx
        self._sites = off
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        n = ctypes.c_size_t(0)
        _check(lib().mpr_init_field(None, gs, len(grids), ctypes.byref(self.params), None, ctypes.byref(n), None))
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        size = ctypes.c_size_t(n.value)
        ctx = ctypes.c_void_p()
        _check(lib().mpr_init_field(ctypes.byref(ctx), gs, len(grids), ctypes.byref(self.params),
                                    ctypes.c_void_p(aligned), ctypes.byref(size),
                                    ctypes.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx

    # -- lifetime
    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            lib().mpr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _T(self, T):
        T = np.broadcast_to(np.asarray(T, dtype=np.float64), (self.n_grids,))
        return np.ascontiguousarray(T)

    # -- Algorithm 1
    def sweep(self, n_sweeps, T, adapt=False, trace_energy=False, trace=False, over_relax=True):
        """Run n hybrid sweeps (Metropolis only when not ``over_relax``).
        Returns a (n, chains, 2) tensor of (A, e) per sweep when ``trace`` (e
        is NaN unless ``trace_energy``)."""
        torch = self._torch
        T = self._T(T)
        tr = torch.empty((n_sweeps, self.total_chains, 2), dtype=torch.float64, device=self.device) if trace else None
        flags = (ADAPT if adapt else 0) | (TRACE_E if trace_energy else 0) | (0 if over_relax else NO_OR)
        _check(lib().mpr_sweep(self.ctx, n_sweeps, _dptr(T), flags,
                               ctypes.c_void_p(tr.data_ptr() if tr is not None else 0)), self.ctx)
        return tr

    def equilibrate(self, T, n_f=5, n_fit=20, i_max=1000, adapt=True, over_relax=True):
        """mpr_equilibrate (Algorithm 2, step 4, stopped by the Savitzky-Golay
        slope test).  Returns (sweeps run, per-chain sweeps at which the
        slope was first >= 0 or -1, (n, chains, 2) tensor of (A, e))."""
        torch = self._torch
        T = self._T(T)
        tr = torch.empty((i_max + 1, self.total_chains, 2), dtype=torch.float64, device=self.device)
        n = ctypes.c_int32(0)
        at = np.empty(self.total_chains, dtype=np.int32)
        flags = (ADAPT if adapt else 0) | (0 if over_relax else NO_OR)
        _check(lib().mpr_equilibrate(self.ctx, _dptr(T), n_f, n_fit, i_max, flags, ctypes.c_void_p(tr.data_ptr()),
                                     ctypes.byref(n), at.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), self.ctx)
        return n.value, at, tr[:n.value]

    # -- Eqs. (4), (5)
    def specific_energy(self, what=SAMPLE_PAIRS, allow_nopairs=False):
        n = self.n_grids if what == SAMPLE_PAIRS else self.total_chains
        e = np.empty(n)
        cnt = np.empty(n, dtype=np.int64)
        rc = lib().mpr_specific_energy(self.ctx, what, _dptr(e), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        if not (rc == MPR_E_NOPAIRS and allow_nopairs):
            _check(rc, self.ctx)
        return e, cnt

    # -- Algorithm 2
    def fill(self, T, n_eq, n_samp, stride=1, want_std=True):
        """Returns (zhat list, zstd list or None, report dict)."""
        torch = self._torch
        T = self._T(T)
        zhat = torch.empty(self._sites, dtype=torch.float64, device=self.device)
        zstd = torch.empty(self._sites, dtype=torch.float64, device=self.device) if want_std else None
        a_eq = np.empty(self.total_chains)
        acc_eq = np.empty(self.total_chains)
        acc_samp = np.empty(self.total_chains)
        rep = FillReport(0, 0, a_eq.ctypes.data, acc_eq.ctypes.data, acc_samp.ctypes.data)
        _check(lib().mpr_fill(self.ctx, _dptr(T), n_eq, n_samp, stride, ctypes.c_void_p(zhat.data_ptr()),
                              ctypes.c_void_p(zstd.data_ptr() if zstd is not None else 0), ctypes.byref(rep)), self.ctx)
        return self._per_grid(zhat), (self._per_grid(zstd) if zstd is not None else None), dict(
            records=rep.records, a_eq=a_eq, acc_eq=acc_eq, acc_samp=acc_samp)

    def _per_grid(self, flat):
        """Views (ny, nx) of each grid's part of a flat site array."""
        out = []
        for off, n, ny, nx in self._runs:
            out.extend(flat[off:off + n * ny * nx].view(n, ny, nx).unbind(0))
        return out

    def set_grid_q(self, q):
        """mpr_set_grid_q: one modification factor per grid."""
        q = np.ascontiguousarray(np.broadcast_to(np.asarray(q, dtype=np.float64), (self.n_grids,)))
        _check(lib().mpr_set_grid_q(self.ctx, _dptr(q)), self.ctx)

    def validation_measures(self, grid, z_true, zhat):
        """mpr_validation_measures: AAE, ARE, AARE, RASE, R (Sec. 3.3) of
        zhat against the complete field z_true over the grid's gaps (gap
        sites where z_true is NaN are left out)."""
        torch = self._torch
        ny, nx, _ = self.shapes[grid]
        zt = torch.as_tensor(z_true, dtype=torch.float64).to(self.device).contiguous()
        zh = torch.as_tensor(zhat, dtype=torch.float64).to(self.device).contiguous()
        if tuple(zt.shape) != (ny, nx) or tuple(zh.shape) != (ny, nx):
            raise ValueError("z_true and zhat must have the grid's shape")
        out = np.empty(8)
        _check(lib().mpr_validation_measures(self.ctx, grid, ctypes.c_void_p(zt.data_ptr()),
                                             ctypes.c_void_p(zh.data_ptr()), _dptr(out)), self.ctx)
        return dict(AAE=out[0], ARE=out[1], AARE=out[2], RASE=out[3], R=out[4], P=int(out[5]),
                    mean_z=out[6], mean_zhat=out[7])

    # -- state
    def get_phi(self, grid=0, chain=0):
        torch = self._torch
        ny, nx, _ = self.shapes[grid]
        out = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        _check(lib().mpr_get_phi(self.ctx, grid, chain, ctypes.c_void_p(out.data_ptr())), self.ctx)
        return out

    def set_phi(self, phi, grid=0, chain=0):
        torch = self._torch
        ny, nx, _ = self.shapes[grid]
        t = torch.as_tensor(phi, dtype=torch.float64).to(self.device).contiguous()
        if tuple(t.shape) != (ny, nx):
            raise ValueError("phi shape mismatch")
        _check(lib().mpr_set_phi(self.ctx, grid, chain, ctypes.c_void_p(t.data_ptr())), self.ctx)
        self.stream.synchronize()

    def autotune(self, T, trial_sweeps=16):
        """mpr_autotune: returns (sweeps per pass, workgroup size, workgroup
        size of single-sweep passes, 1 if those run on persistent workgroups)
        chosen."""
        T = self._T(T)
        nsw = ctypes.c_int32(0)
        thr = ctypes.c_int32(0)
        thr1 = ctypes.c_int32(0)
        p1 = ctypes.c_int32(0)
        _check(lib().mpr_autotune(self.ctx, _dptr(T), trial_sweeps, ctypes.byref(nsw), ctypes.byref(thr),
                                  ctypes.byref(thr1), ctypes.byref(p1)), self.ctx)
        return nsw.value, thr.value, thr1.value, p1.value

    def set_launch_shape(self, nsw, threads, threads1, persist1=1):
        """mpr_set_launch_shape: sweeps per multi-sweep pass, the two
        workgroup sizes and persistent single-sweep passes, without timing."""
        _check(lib().mpr_set_launch_shape(self.ctx, int(nsw), int(threads), int(threads1), int(persist1)),
               self.ctx)

    def reinit(self):
        """mpr_reinit: hot start again from the z and known tensors given at
        construction (their values may have changed in place)."""
        _check(lib().mpr_reinit(self.ctx), self.ctx)

    def set_graph(self, enable=True):
        """mpr_set_graph: record and replay mpr_fill's sweeps as a hipGraph."""
        _check(lib().mpr_set_graph(self.ctx, 1 if enable else 0), self.ctx)

    def set_timing(self, enable=True):
        _check(lib().mpr_set_timing(self.ctx, 1 if enable else 0), self.ctx)

    def timing(self):
        """(milliseconds in sweep kernels, launches, site-sweeps) since the
        last call; resets the sums."""
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        ss = ctypes.c_int64(0)
        _check(lib().mpr_get_timing(self.ctx, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(ss)), self.ctx)
        return ms.value, n.value, ss.value

    def chain_state(self):
        idx = ctypes.c_int64(0)
        a = np.empty(self.total_chains)
        _check(lib().mpr_get_chain_state(self.ctx, ctypes.byref(idx), _dptr(a)), self.ctx)
        return idx.value, a

    def set_chain_state(self, sweep_index, a=None):
        ap = None
        if a is not None:
            a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (self.total_chains,)))
            ap = _dptr(a)
        _check(lib().mpr_set_chain_state(self.ctx, int(sweep_index), ap), self.ctx)


def temperatures_from_table(e_s, table_T, table_e):
    """T-hat per grid by mpr_match_T; NaN e_s raise."""
    T, st = match_T(e_s, table_T, table_e)
    if np.any(np.isnan(T)):
        raise MPRError(MPR_E_ARG, "e_s is NaN")
    return T, st


TWO_PI = 2.0 * math.pi
