"""ctypes binding of libcfv.so with the C ABI's names (argument marshalling only).

Every computation runs in the HIP library; this module only converts torch
tensors to device pointers and streams.  There is no fallback: if the built
library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .params import Params

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcfv.so")

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class CfvParams(ctypes.Structure):
    _fields_ = [("gamma", c_double), ("c_h", c_double), ("G", c_double), ("vr_star", c_double),
                ("rho_b", c_double), ("T_b", c_double), ("limiter", c_int32), ("inner_mode", c_int32),
                ("outer_exp", c_double * 8), ("outer_vr_mass", c_int32), ("outer_psi_zero", c_int32)]


class CfvTuning(ctypes.Structure):
    _fields_ = [("queue", c_int32), ("blocks_per_cu", c_int32), ("order", c_int32), ("chunk_layers", c_int32)]


class CfvSteadyCfg(ctypes.Structure):
    _fields_ = [("cfl0", c_double), ("cfl_max", c_double), ("every", c_int32), ("max_iters", c_int32),
                ("monitor", c_int32), ("target", c_double), ("m", c_int32), ("max_restarts", c_int32),
                ("rtol", c_double)]


class CfvError(RuntimeError):
    pass


class CfvNonPhysical(CfvError):
    """Status 4: a non-positive or NaN face density or pressure, or a
    non-finite solve.  From a march, hist and cfls hold the steps taken (the
    last one the failing step) and the state is the one before it; from other
    calls they are None."""

    def __init__(self, msg, hist=None, cfls=None):
        super().__init__(msg)
        self.hist, self.cfls = hist, cfls


_lib = None


def lib():
    """Load libcfv.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise CfvError(f"{LIB_PATH} is missing: build it with `python -m paper_2209_04481_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "cfv_last_error": ([], ctypes.c_char_p),
        "cfv_grid_create": ([c_int32, c_int32, P, ctypes.POINTER(P)], c_int32),
        "cfv_grid_destroy": ([P], None),
        "cfv_grid_sizes": ([P, P, P, P], c_int32),
        "cfv_grid_faces_to_host": ([P, P, P, P], c_int32),
        "cfv_grid_geometry_to_host": ([P, P, P, P, P], c_int32),
        "cfv_ctx_create": ([P, ctypes.POINTER(CfvParams), ctypes.POINTER(P)], c_int32),
        "cfv_ctx_destroy": ([P], None),
        "cfv_set_inner_br": ([P, P, c_int64, P], c_int32),
        "cfv_set_inner_btheta": ([P, P, c_int64, P], c_int32),
        "cfv_geometry": ([P, P, P, P, P, P], c_int32),
        "cfv_residual": ([P, P, P, P], c_int32),
        "cfv_jvp": ([P, P, P, P, P, P, P], c_int32),
        "cfv_vjp": ([P, P, P, P, P, P], c_int32),
        "cfv_local_dt": ([P, P, c_double, P, P], c_int32),
        "cfv_dots_noalloc": ([c_int64, P, c_int32, P, P, P], c_int32),
        "cfv_status_flags": ([P, P, P], c_int32),
        "cfv_ensemble_status_flags": ([P, P, P], c_int32),
        "cfv_efield": ([P, P, P, P, P], c_int32),
        "cfv_efree_state": ([P, P, P, P], c_int32),
        "cfv_monitor": ([P, P, P, P, P], c_int32),
        "cfv_steady": ([P, P, ctypes.POINTER(CfvSteadyCfg), P, P, P, P], c_int32),
        "cfv_norms": ([P, P, P, P, P], c_int32),
        "cfv_dots": ([P, P, c_int32, P, P, P], c_int32),
        "cfv_axpby": ([P, c_int64, c_double, P, c_double, P, P], c_int32),
        "cfv_solve": ([P, P, P, P, c_int32, c_int32, c_int32, c_double, P, P, c_int32, P, P, P], c_int32),
        "cfv_be_step": ([P, P, c_double, c_int32, c_int32, c_double, P, P, c_int32, P, P, P], c_int32),
        "cfv_vjp_dir": ([P, P, P, P, c_double, P, P, P, P], c_int32),
        "cfv_jvp_dir": ([P, P, P, P, P, c_double, P, P, P], c_int32),
        "cfv_ensemble_create": ([P, c_int32, P, ctypes.POINTER(P)], c_int32),
        "cfv_ensemble_destroy": ([P], None),
        "cfv_ensemble_set_tuning": ([P, P], c_int32),
        "cfv_ensemble_items": ([P, P, P], c_int32),
        "cfv_ensemble_bind": ([P, P, P, P, P, P], c_int32),
        "cfv_ensemble_run": ([P, P], c_int32),
        "cfv_ensemble_bind_be_step": ([P, P, P, c_double, c_int32, P], c_int32),
        "cfv_ensemble_residual_jvp": ([P, P, P, P, P, P], c_int32),
        "cfv_ensemble_steady": ([P, P, P, ctypes.POINTER(CfvSteadyCfg), P, P, P, P], c_int32),
        "cfv_ensemble_graph_capture": ([P, P], c_int32),
        "cfv_ensemble_graph_launch": ([P, P], c_int32),
        "cfv_ensemble_timing_enable": ([P, c_int32], c_int32),
        "cfv_ensemble_timing_read": ([P, c_int32, P, P, P, P], c_int32),
        "cfv_timing_enable": ([P, c_int32], c_int32),
        "cfv_set_chunk_layers": ([P, c_int32], c_int32),
        "cfv_set_preconditioner": ([P, c_int32], c_int32),
        "cfv_ensemble_set_preconditioner": ([P, c_int32], c_int32),
        "cfv_timing_read": ([P, c_int32, P, P, P, P], c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(status: int):
    if status == 4:
        raise CfvNonPhysical(f"cfv status 4: {lib().cfv_last_error().decode()}")
    if status != 0:
        raise CfvError(f"cfv status {status}: {lib().cfv_last_error().decode()}")


def _ptr(t):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise CfvError("expected a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise CfvError("expected a contiguous float64 tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _timing_read(fn, h, max_names):
    names = ctypes.create_string_buffer(32 * max_names)
    ms = (c_double * max_names)()
    cnt = (c_int64 * max_names)()
    n = c_int32()
    check(fn(h, max_names, names, ms, cnt, ctypes.byref(n)))
    out = {}
    for q in range(n.value):
        nm = names.raw[32 * q:32 * q + 32].split(b"\0", 1)[0].decode()
        out[nm] = (ms[q], cnt[q])
    return out


def _ptr_array(ts, what):
    """Host array of device pointers (None -> NULL array)."""
    if ts is None:
        return None
    arr = (c_void_p * len(ts))()
    for q, t in enumerate(ts):
        arr[q] = _ptr(t).value if t is not None else None
    return arr


def dots_noalloc(V, w, k=None, out=None, stream=None):
    """out[i] = <V[i], w> for the first k rows of V (k <= 32) without a
    context and without device allocation in the library (cfv_dots_noalloc);
    V: (k, n) and w: (n,) contiguous float64 CUDA tensors, out: (k,) or new."""
    import torch
    k = V.shape[0] if k is None else int(k)
    n = w.numel()
    if V.numel() < k * n:
        raise CfvError("V must hold k vectors of w's length")
    o = out if out is not None else torch.empty(k, dtype=torch.float64, device=w.device)
    check(lib().cfv_dots_noalloc(int(n), _ptr(V), int(k), _ptr(w), _ptr(o), _stream(stream)))
    return o


class Grid:
    """Cubed-sphere shell grid (host topology): cfv_grid_*."""

    def __init__(self, N: int, Nr: int, r_nodes):
        r = np.ascontiguousarray(np.asarray(r_nodes, dtype=np.float64))
        if r.size != Nr + 1:
            raise CfvError("r_nodes must have Nr + 1 entries")
        self.N, self.Nr = int(N), int(Nr)
        self.r_nodes = r
        h = c_void_p()
        check(lib().cfv_grid_create(self.N, self.Nr, r.ctypes.data_as(c_void_p), ctypes.byref(h)))
        self._h = h
        nc, nf, nb = c_int64(), c_int64(), c_int64()
        check(lib().cfv_grid_sizes(h, ctypes.byref(nc), ctypes.byref(nf), ctypes.byref(nb)))
        self.ncells, self.nfaces, self.nb = nc.value, nf.value, nb.value

    def faces(self):
        L = np.empty(self.nfaces, np.int64)
        R = np.empty(self.nfaces, np.int64)
        K = np.empty(self.nfaces, np.int8)
        check(lib().cfv_grid_faces_to_host(self._h, L.ctypes.data_as(c_void_p), R.ctypes.data_as(c_void_p),
                                           K.ctypes.data_as(c_void_p)))
        return L, R, K

    def geometry(self):
        """Host geometry as the kernels build it: per face of the canonical
        list its vector area S (L -> R, outward on the boundary) and
        centroid, per cell its volume and centroid."""
        S = np.empty((self.nfaces, 3), dtype=np.float64)
        xf = np.empty((self.nfaces, 3), dtype=np.float64)
        V = np.empty(self.ncells, dtype=np.float64)
        xc = np.empty((self.ncells, 3), dtype=np.float64)
        check(lib().cfv_grid_geometry_to_host(self._h, S.ctypes.data_as(c_void_p), xf.ctypes.data_as(c_void_p),
                                              V.ctypes.data_as(c_void_p), xc.ctypes.data_as(c_void_p)))
        return S, xf, V, xc

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cfv_grid_destroy(h)
            self._h = None


class Context:
    """A grid and parameters bound to the current GPU: cfv_ctx_* and the
    stream-ordered entry points.  Tensors are float64 CUDA tensors in the
    SoA layout [9, ncells]."""

    def __init__(self, grid: Grid, params: Params | None = None):
        self.grid = grid
        self.params = params or Params()
        p = self.params
        cp = CfvParams(p.gamma, p.c_h, p.G, p.vr_star, p.rho_b, p.T_b, int(p.limiter), int(p.inner_mode),
                       (c_double * 8)(*[float(x) for x in p.outer_exp]), int(bool(p.outer_vr_mass)),
                       int(bool(p.outer_psi_zero)))
        h = c_void_p()
        check(lib().cfv_ctx_create(grid._h, ctypes.byref(cp), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cfv_ctx_destroy(h)
            self._h = None

    # ---- helpers
    def _new(self, *shape):
        import torch
        return torch.empty(*shape, dtype=torch.float64, device="cuda")

    def _state(self, t, name):
        if tuple(t.shape) != (9, self.grid.ncells):
            raise CfvError(f"{name} must have shape (9, {self.grid.ncells})")
        return _ptr(t)

    # ---- entry points
    def set_inner_br(self, br, stream=None):
        check(lib().cfv_set_inner_br(self._h, _ptr(br), br.numel(), _stream(stream)))

    def set_inner_btheta(self, bth, stream=None):
        """B_theta map of the large-E inner boundary (inner_mode = 1)."""
        check(lib().cfv_set_inner_btheta(self._h, _ptr(bth), bth.numel(), _stream(stream)))

    def geometry(self, stream=None):
        nc = self.grid.ncells
        xc, vol, xf, S = self._new(nc, 3), self._new(nc), self._new(nc, 6, 3), self._new(nc, 6, 3)
        check(lib().cfv_geometry(self._h, _ptr(xc), _ptr(vol), _ptr(xf), _ptr(S), _stream(stream)))
        return xc, vol, xf, S

    def residual(self, U, out=None, stream=None):
        R = out if out is not None else self._new(9, self.grid.ncells)
        check(lib().cfv_residual(self._h, self._state(U, "U"), self._state(R, "R"), _stream(stream)))
        return R

    def jvp(self, U, v, dbr=None, out=None, R=None, stream=None):
        Jv = out if out is not None else self._new(9, self.grid.ncells)
        check(lib().cfv_jvp(self._h, self._state(U, "U"), self._state(v, "v"), _ptr(dbr), self._state(Jv, "Jv"),
                            None if R is None else self._state(R, "R"), _stream(stream)))
        return Jv

    def vjp(self, U, w, out=None, gbr=None, want_br=True, stream=None):
        gU = out if out is not None else self._new(9, self.grid.ncells)
        if gbr is None and want_br:
            gbr = self._new(self.grid.nb)
        check(lib().cfv_vjp(self._h, self._state(U, "U"), self._state(w, "w"), self._state(gU, "gU"),
                            _ptr(gbr), _stream(stream)))
        return gU, gbr

    def vjp_dir(self, U, w, x, eps=1e-6, out=None, gbr=None, want_br=True, stream=None):
        """d/de of the VJP at U + e x (central difference); returns (gU2, gbr2, h)."""
        gU = out if out is not None else self._new(9, self.grid.ncells)
        if gbr is None and want_br:
            gbr = self._new(self.grid.nb)
        h = c_double()
        check(lib().cfv_vjp_dir(self._h, self._state(U, "U"), self._state(w, "w"), self._state(x, "x"), float(eps),
                                self._state(gU, "gU2"), _ptr(gbr), ctypes.byref(h), _stream(stream)))
        return gU, gbr, h.value

    def jvp_dir(self, U, v, dU, dbr=None, eps=1e-6, out=None, stream=None):
        """d/de of the JVP J(U + e dU, b + e dbr) v (central difference); returns (Jv2, h)."""
        Jv = out if out is not None else self._new(9, self.grid.ncells)
        h = c_double()
        check(lib().cfv_jvp_dir(self._h, self._state(U, "U"), self._state(v, "v"), self._state(dU, "dU"), _ptr(dbr),
                                float(eps), self._state(Jv, "Jv2"), ctypes.byref(h), _stream(stream)))
        return Jv, h.value

    def status_flags(self, stream=None):
        """The context's non-physical flag word since the last read (bit 0: a
        face state with non-positive or NaN density or pressure); clears it."""
        f = c_int32()
        rc = lib().cfv_status_flags(self._h, ctypes.byref(f), _stream(stream))
        if rc != 4:
            check(rc)
        return f.value

    def local_dt(self, U, cfl, out=None, stream=None):
        d = out if out is not None else self._new(self.grid.ncells)
        check(lib().cfv_local_dt(self._h, self._state(U, "U"), float(cfl), _ptr(d), _stream(stream)))
        return d

    def efield(self, U, field=True, stats=None, E=None, stream=None):
        """E = -V x B in spherical components and its statistics (cfv_efield).

        Returns (E, stats): E is [3, ncells] (E_r, E_theta, E_phi), or None
        when field is False; stats holds max |E_r|, |E_theta|, |E_phi|, |E|
        and then the volume-weighted RMS of the same four."""
        o = stats if stats is not None else self._new(8)
        if o.numel() < 8:
            raise CfvError("stats needs 8 entries")
        e = None
        if field:
            e = E if E is not None else self._new(3, self.grid.ncells)
            if tuple(e.shape) != (3, self.grid.ncells):
                raise CfvError(f"E must have shape (3, {self.grid.ncells})")
        check(lib().cfv_efield(self._h, self._state(U, "U"), None if e is None else _ptr(e), _ptr(o),
                               _stream(stream)))
        return e, o

    def efree_state(self, U, out=None, stream=None):
        """U with its velocity projected on B (V x B = 0), cfv_efree_state;
        out may be U itself."""
        o = out if out is not None else self._new(9, self.grid.ncells)
        check(lib().cfv_efree_state(self._h, self._state(U, "U"), self._state(o, "out"), _stream(stream)))
        return o

    def monitor(self, a, b, out=None, stream=None):
        """Eq. 2 monitor of the primitives before the log10 (cfv_monitor): 9 norms."""
        o = out if out is not None else self._new(9)
        check(lib().cfv_monitor(self._h, self._state(a, "a"), self._state(b, "b"), _ptr(o), _stream(stream)))
        return o

    def steady(self, U, max_iters, cfl0=2.0, cfl_max=128.0, every=200, monitor=1, target=-np.inf, m=30,
               max_restarts=0, rtol=0.0, stream=None):
        """March U (updated in place) toward a steady state (cfv_steady).

        Returns (log10 monitor history [iters, 9], CFL per step [iters])."""
        cfg = CfvSteadyCfg(float(cfl0), float(cfl_max), int(every), int(max_iters), int(monitor), float(target),
                           int(m), int(max_restarts), float(rtol))
        hist = np.zeros((max(int(max_iters), 1), 9))
        cfls = np.zeros(max(int(max_iters), 1))
        it = c_int32()
        st = lib().cfv_steady(self._h, self._state(U, "U"), ctypes.byref(cfg), hist.ctypes.data_as(c_void_p),
                              cfls.ctypes.data_as(c_void_p), ctypes.byref(it), _stream(stream))
        if st == 4:
            raise CfvNonPhysical(f"cfv status 4: {lib().cfv_last_error().decode()}", hist[:it.value],
                                 cfls[:it.value])
        check(st)
        return hist[:it.value], cfls[:it.value]

    def norms(self, a, b=None, out=None, stream=None):
        o = out if out is not None else self._new(9)
        check(lib().cfv_norms(self._h, self._state(a, "a"), None if b is None else self._state(b, "b"), _ptr(o),
                              _stream(stream)))
        return o

    def dots(self, V, w, k=None, out=None, stream=None):
        k = V.shape[0] if k is None else k
        o = out if out is not None else self._new(k)
        check(lib().cfv_dots(self._h, _ptr(V), int(k), _ptr(w), _ptr(o), _stream(stream)))
        return o

    def solve(self, U, diag, rhs, transpose=False, m=30, max_restarts=0, rtol=0.0, out=None, stream=None):
        """GMRES on (diag + J) x = rhs or its transpose; returns (x, history)."""
        x = out if out is not None else self._new(9, self.grid.ncells)
        hl = m * (max_restarts + 1)
        hist = np.zeros(hl)
        it = c_int32()
        fr = c_double()
        check(lib().cfv_solve(self._h, self._state(U, "U"), _ptr(diag), self._state(rhs, "rhs"), int(bool(transpose)),
                              int(m), int(max_restarts), float(rtol), self._state(x, "x"),
                              hist.ctypes.data_as(c_void_p), hl, ctypes.byref(it), ctypes.byref(fr), _stream(stream)))
        return x, hist[:it.value]

    def be_step(self, U, cfl=1e3, m=30, max_restarts=0, rtol=0.0, out=None, stream=None):
        """One backward-Euler step; returns (U_new, history)."""
        Un = out if out is not None else self._new(9, self.grid.ncells)
        hl = m * (max_restarts + 1)
        hist = np.zeros(hl)
        it = c_int32()
        fr = c_double()
        check(lib().cfv_be_step(self._h, self._state(U, "U"), float(cfl), int(m), int(max_restarts), float(rtol),
                                self._state(Un, "U_new"), hist.ctypes.data_as(c_void_p), hl, ctypes.byref(it),
                                ctypes.byref(fr), _stream(stream)))
        return Un, hist[:it.value]

    def timing_enable(self, on=True):
        check(lib().cfv_timing_enable(self._h, int(bool(on))))

    def set_preconditioner(self, kind: int):
        """GMRES preconditioner of this context's solves: 0 none, 1 Jacobi
        (right preconditioning by the solve's diagonal)."""
        check(lib().cfv_set_preconditioner(self._h, int(kind)))

    def set_chunk_layers(self, kc: int):
        """Layers per work item of this context's marches, 0 = balanced per
        march (the default); the outputs do not change."""
        check(lib().cfv_set_chunk_layers(self._h, int(kc)))

    def timing_read(self, max_names=32):
        """{kernel name: (total ms, launches)} since the previous read."""
        return _timing_read(lib().cfv_timing_read, self._h, max_names)

    def axpby(self, a, x, b, y, stream=None):
        check(lib().cfv_axpby(self._h, y.numel(), float(a), _ptr(x), float(b), _ptr(y), _stream(stream)))
        return y


class Tuning:
    """Schedule and work-item shape of the ensemble launch (cfv_tuning);
    chunk_layers 0 is the library's default (16)."""

    def __init__(self, queue: int = 1, blocks_per_cu: int = 2, order: int = 1, chunk_layers: int = 0):
        self.queue, self.blocks_per_cu, self.order = int(queue), int(blocks_per_cu), int(order)
        self.chunk_layers = int(chunk_layers)

    def c(self):
        return CfvTuning(self.queue, self.blocks_per_cu, self.order, self.chunk_layers)

    def as_dict(self):
        return {"queue": self.queue, "blocks_per_cu": self.blocks_per_cu, "order": self.order,
                "chunk_layers": self.chunk_layers}

    def __repr__(self):
        return f"Tuning({self.queue}, {self.blocks_per_cu}, {self.order}, {self.chunk_layers})"


class Ensemble:
    """Many instances (contexts) evaluated by one persistent launch per pass:
    cfv_ensemble_*.  Lists of tensors are per instance, in context order."""

    def __init__(self, contexts, tuning: Tuning | None = None):
        self.contexts = list(contexts)
        self.tuning = tuning or Tuning()
        arr = (c_void_p * len(self.contexts))(*[c._h.value for c in self.contexts])
        h = c_void_p()
        t = self.tuning.c()
        check(lib().cfv_ensemble_create(arr, len(self.contexts), ctypes.byref(t), ctypes.byref(h)))
        self._h = h
        self._keep = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cfv_ensemble_destroy(h)
            self._h = None

    def set_preconditioner(self, kind: int):
        """GMRES preconditioner of the batched step (0 none, 1 Jacobi); takes
        effect at the next bind_be_step."""
        check(lib().cfv_ensemble_set_preconditioner(self._h, int(kind)))

    def set_tuning(self, tuning: Tuning):
        t = tuning.c()
        check(lib().cfv_ensemble_set_tuning(self._h, ctypes.byref(t)))
        self.tuning = tuning

    def items(self):
        """(work items, workgroups per launch)."""
        tot, blk = c_int64(), c_int32()
        check(lib().cfv_ensemble_items(self._h, ctypes.byref(tot), ctypes.byref(blk)))
        return tot.value, blk.value

    def _check(self, ts, name, shape_of):
        if ts is None:
            return
        if len(ts) != len(self.contexts):
            raise CfvError(f"{name}: need one tensor per instance")
        for t, c in zip(ts, self.contexts):
            if tuple(t.shape) != shape_of(c):
                raise CfvError(f"{name} must have shape {shape_of(c)}")

    def bind(self, U, v=None, dbr=None, R=None, Jv=None):
        """Bind per-instance buffers (kept alive by the ensemble)."""
        st = lambda c: (9, c.grid.ncells)
        for ts, name, sh in ((U, "U", st), (v, "v", st), (R, "R", st), (Jv, "Jv", st),
                             (dbr, "dbr", lambda c: (c.grid.nb,))):
            self._check(ts, name, sh)
        self._keep = (U, v, dbr, R, Jv)
        check(lib().cfv_ensemble_bind(self._h, _ptr_array(U, "U"), _ptr_array(v, "v"), _ptr_array(dbr, "dbr"),
                                      _ptr_array(R, "R"), _ptr_array(Jv, "Jv")))

    def bind_be_step(self, U, U_new, cfl=1e3, m=30, hist=None):
        """Bind one backward-Euler step of every instance (GMRES(m), on the
        device); hist: optional (n, m) float64 CUDA tensor for the histories."""
        st = lambda c: (9, c.grid.ncells)
        self._check(U, "U", st)
        self._check(U_new, "U_new", st)
        if hist is not None and tuple(hist.shape) != (len(self.contexts), int(m)):
            raise CfvError(f"hist must have shape ({len(self.contexts)}, {int(m)})")
        self._keep = (U, U_new, hist)
        check(lib().cfv_ensemble_bind_be_step(self._h, _ptr_array(U, "U"), _ptr_array(U_new, "U_new"), float(cfl),
                                              int(m), _ptr(hist)))

    def be_step(self, U, cfl=1e3, m=30, stream=None):
        """Bind and run one step; returns (U_new list, (n, m) history tensor)."""
        import torch
        U_new = [torch.empty_like(u) for u in U]
        hist = torch.zeros(len(self.contexts), int(m), dtype=torch.float64, device="cuda")
        self.bind_be_step(U, U_new, cfl, m, hist)
        self.run(stream)
        return U_new, hist

    def run(self, stream=None):
        check(lib().cfv_ensemble_run(self._h, _stream(stream)))

    def steady(self, U, max_iters, cfl0=2.0, cfl_max=128.0, every=200, monitor=1, target=-np.inf, m=30,
               U_work=None, stream=None):
        """March every instance (U, updated in place) toward a steady state in
        lockstep (cfv_ensemble_steady); a graph is captured when stream is a
        created stream.  Returns (log10 monitor history [n, max_iters, 9], NaN
        after an instance stopped; steps per instance)."""
        import torch
        st = lambda c: (9, c.grid.ncells)
        self._check(U, "U", st)
        U_work = U_work if U_work is not None else [torch.empty_like(u) for u in U]
        self._check(U_work, "U_work", st)
        self._keep = (U, U_work)
        n = len(self.contexts)
        cfg = CfvSteadyCfg(float(cfl0), float(cfl_max), int(every), int(max_iters), int(monitor), float(target),
                           int(m), 0, 0.0)
        hist = np.zeros((n, max(int(max_iters), 1), 9))
        steps = np.zeros(n, dtype=np.int32)
        it = c_int32()
        rc = lib().cfv_ensemble_steady(self._h, _ptr_array(U, "U"), _ptr_array(U_work, "U_work"), ctypes.byref(cfg),
                                       hist.ctypes.data_as(c_void_p), steps.ctypes.data_as(c_void_p),
                                       ctypes.byref(it), _stream(stream))
        hist = hist[:, :int(max_iters)]
        if rc == 4:
            raise CfvNonPhysical(f"cfv status 4: {lib().cfv_last_error().decode()}", hist, steps)
        check(rc)
        return hist, steps

    def residual_jvp(self, U, v, R=None, Jv=None, stream=None):
        """Bind and run; returns (R, Jv) lists (allocated when not given)."""
        import torch
        R = R if R is not None else [torch.empty(9, c.grid.ncells, dtype=torch.float64, device="cuda")
                                     for c in self.contexts]
        Jv = Jv if Jv is not None else [torch.empty(9, c.grid.ncells, dtype=torch.float64, device="cuda")
                                        for c in self.contexts]
        self.bind(U, v=v, R=R, Jv=Jv)
        self.run(stream)
        return R, Jv

    def status_flags(self, stream=None):
        """Per-instance non-physical flag words since the last read; clears them."""
        f = np.zeros(len(self.contexts), dtype=np.int32)
        rc = lib().cfv_ensemble_status_flags(self._h, f.ctypes.data_as(c_void_p), _stream(stream))
        if rc != 4:
            check(rc)
        return f

    def capture(self, stream):
        """Capture one run of the bound ensemble into a graph (stream: a torch.cuda.Stream)."""
        check(lib().cfv_ensemble_graph_capture(self._h, _stream(stream)))

    def replay(self, stream):
        check(lib().cfv_ensemble_graph_launch(self._h, _stream(stream)))

    def timing_enable(self, on=True):
        check(lib().cfv_ensemble_timing_enable(self._h, int(bool(on))))

    def timing_read(self, max_names=32):
        return _timing_read(lib().cfv_ensemble_timing_read, self._h, max_names)
