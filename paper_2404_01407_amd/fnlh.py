"""Python binding of libfnlh (include/fnlh.h): argument marshalling only.

Every step of the solve runs in the HIP library; this module converts numpy arrays
(host mesh data) and torch CUDA tensors (device vectors, HIP streams) into the plain
pointers of the C ABI.  There is no fallback: if the built library is missing the
import of this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch before the library: torch carries its own HIP runtime (soname libamdhip64.so.7),
# and libfnlh, loaded after it, binds to that same runtime.  Loaded the other way round,
# libfnlh would bring in /opt/rocm's runtime and torch its own beside it, two HIP and
# HSA runtimes in one process, and the library's hipSetDevice then finds no device.
import torch  # noqa: E402,F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libfnlh.so")

# status codes (fnlh.h)
OK, NOT_CONVERGED, DIVERGED, FELL_BACK = 0, 1, 2, 3
E_ARG, E_MESH, E_SINGULAR, E_OOM, E_HIP, E_ORDER = -1, -2, -3, -4, -5, -6
STORAGE = {"f64": 0, "f32": 1, "bf16": 2}
OUTER = {"exact": 0, "stored": 1}
ORDERING = {"auto": 0, "greedy": 1, "bipartite": 2, "user": 3}
KIND = {"dilu": 0, "sgs": 1, "jacobi": 2, "learned": 3, "pilu": 4}
SCHEME = {"implicit": 0, "explicit": 1}


class FnlhError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fnlh error {code}: {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_edges", C.c_int64), ("n_bfaces", C.c_int64),
                ("n_zones", C.c_int32), ("pad_", C.c_int32),
                ("edges", C.c_void_p), ("area", C.c_void_p), ("volume", C.c_void_p),
                ("zone", C.c_void_p), ("bface_cell", C.c_void_p), ("bface_area", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("storage", C.c_int32), ("outer", C.c_int32), ("ordering", C.c_int32),
                ("factor_slots", C.c_int32), ("user_colour", C.c_void_p), ("device", C.c_int32),
                ("pad_", C.c_int32)]


class RelaxOpts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("max_sweeps", C.c_int32), ("rtol", C.c_double),
                ("check_every", C.c_int32), ("inner_sweeps", C.c_int32), ("inner_rtol", C.c_double),
                ("div_factor", C.c_double), ("use_graph", C.c_int32), ("learn_every", C.c_int32),
                ("history", C.c_void_p), ("history_len", C.c_int32), ("pad_", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("outer", C.c_int32), ("status", C.c_int32),
                ("fallbacks", C.c_int32), ("rel_res", C.c_double), ("res0", C.c_double),
                ("t_factor_ms", C.c_double), ("t_sweep_ms", C.c_double), ("learned", C.c_int32),
                ("pad_", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class GmresOpts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("restart", C.c_int32), ("max_iters", C.c_int32), ("inner_sweeps", C.c_int32),
                ("rtol", C.c_double), ("use_graph", C.c_int32), ("pad_", C.c_int32)]


class GmresReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32), ("learned", C.c_int32),
                ("rel_res", C.c_double), ("res0", C.c_double), ("t_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class TuneResult(C.Structure):
    _fields_ = [("lanes_per_row", C.c_int32), ("sys_per_lane", C.c_int32), ("wave_groups", C.c_int32),
                ("hybrid", C.c_int32), ("ms_best", C.c_double), ("ms_default", C.c_double), ("sweeps", C.c_int32),
                ("candidates", C.c_int32)]


class KernelStats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("alg_bytes", C.c_double)]


KSTAT = {"sweep_update": 0, "sweep_set": 1, "fwd": 2, "bwd": 3, "jacobi": 4, "fwd_last": 5, "remainder": 6,
         "pilu": 7}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfnlh.so not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, V = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    sig = {
        "fnlh_create": (I32, [C.POINTER(P), C.POINTER(Mesh), C.POINTER(Options)]),
        "fnlh_destroy": (I32, [P]),
        "fnlh_assemble_jacobian": (I32, [P, V, V, D, D, I32, V]),
        "fnlh_set_blocks": (I32, [P, V, V, V]),
        "fnlh_get_blocks": (I32, [P, V, V, V]),
        "fnlh_set_harmonics": (I32, [P, I32, V, V]),
        "fnlh_set_phase_lag": (I32, [P, V, I32, V]),
        "fnlh_set_frozen_turbulence": (I32, [P, I32, V]),
        "fnlh_set_partitions": (I32, [P, V, V]),
        "fnlh_gmres": (I32, [P, I32, V, V, V, C.POINTER(GmresOpts), V, V, V]),
        "fnlh_rusanov_residual": (I32, [P, V, V, V, C.POINTER(D), V]),
        "fnlh_rk_mean": (I32, [P, I32, V, V, I32, D, D, I32, C.POINTER(RelaxOpts), V, V]),
        "fnlh_rk_harmonic": (I32, [P, I32, V, V, I32, C.POINTER(RelaxOpts), V, V]),
        "fnlh_residual": (I32, [P, I32, V, V, V, C.POINTER(D), V]),
        "fnlh_relax": (I32, [P, I32, V, V, V, C.POINTER(RelaxOpts), V, V]),
        "fnlh_residual_noalloc": (I32, [P, I32, V, V, V, V, V]),
        "fnlh_noalloc_scratch_bytes": (C.c_size_t, []),
        "fnlh_get_ordering": (I32, [P, V, C.POINTER(I32)]),
        "fnlh_memory": (I32, [P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "fnlh_last_error": (C.c_char_p, [P]),
        "fnlh_order_mesh": (I32, [C.POINTER(Mesh), C.POINTER(Options), V, V, C.POINTER(I32)]),
        "fnlh_version": (C.c_char_p, []),
        "fnlh_stats_enable": (I32, [P, I32]),
        "fnlh_tune": (I32, [P, I32, I32]),
        "fnlh_autotune": (I32, [P, I32, D, I32, C.POINTER(TuneResult), V]),
        "fnlh_batch_create": (I32, [C.POINTER(P), I32, V]),
        "fnlh_batch_destroy": (I32, [P]),
        "fnlh_batch_relax": (I32, [P, V, V, V, V, C.POINTER(RelaxOpts), V, V]),
        "fnlh_batch_last_error": (C.c_char_p, [P]),
        "fnlh_batch_set_loop_cells": (I32, [P, I64]),
        "fnlh_batch_autotune": (I32, [P, V, V, V, V, C.POINTER(RelaxOpts), I32, V, C.POINTER(I64), V, V]),
        "fnlh_stats_get": (I32, [P, I32, C.POINTER(KernelStats)]),
        "fnlh_nn_create": (I32, [C.POINTER(P), P, I32]),
        "fnlh_nn_generate": (I32, [P, I32, V, I32, I32, I32, C.c_uint64, V]),
        "fnlh_nn_get_pair": (I32, [P, I64, C.POINTER(I32), V, V, V]),
        "fnlh_nn_save": (I32, [P, C.c_char_p]),
        "fnlh_nn_load": (I32, [P, C.c_char_p]),
        "fnlh_nn_copy_state": (I32, [P, P]),
        "fnlh_nn_destroy": (I32, [P]),
        "fnlh_nn_set_grad_groups": (I32, [P, I32]),
        "fnlh_nn_set_weights": (I32, [P, V]),
        "fnlh_nn_get_weights": (I32, [P, V]),
        "fnlh_nn_apply": (I32, [P, I32, V, V, V]),
        "fnlh_nn_loss_grad": (I32, [P, I32, V, V, V, V, C.POINTER(D), V]),
        "fnlh_nn_add_pairs": (I32, [P, I32, V, V, V, V]),
        "fnlh_nn_clear_pairs": (I32, [P]),
        "fnlh_nn_reserve_pairs": (I32, [P, I64, V]),
        "fnlh_nn_pairs": (I32, [P, C.POINTER(I64)]),
        "fnlh_nn_train": (I32, [P, I32, I32, C.c_float, C.c_uint64, V, V]),
        "fnlh_nn_selftest": (I32, [P, V, V, V]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev_tensor(t, shape, name, dtype="complex128", device=None):
    """Check a device argument before its pointer crosses the ABI: a torch tensor of the
    expected dtype (complex128 vectors, float64 states and blocks), shape and layout, on
    the context's HIP device.  Every check runs before any library call, so a wrong
    tensor never reaches a kernel that would read or write past its end."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    want = getattr(torch, dtype)
    if t.dtype != want:
        raise TypeError(f"{name}: dtype {t.dtype} != {want}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA (HIP) tensor, got one on {t.device}")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name}: tensor on cuda:{t.device.index}, context on cuda:{device}")
    return t


class _MeshArrays:
    """Keeps contiguous host copies alive for the duration of a call."""

    def __init__(self, mesh, n_zones=None):
        self.edges = np.ascontiguousarray(mesh.edges, dtype=np.int32)
        self.area = np.ascontiguousarray(mesh.area, dtype=np.float64)
        self.volume = np.ascontiguousarray(mesh.volume, dtype=np.float64)
        z = getattr(mesh, "zone", None)
        self.zone = None if z is None else np.ascontiguousarray(z, dtype=np.int32)
        self.bface_cell = np.ascontiguousarray(mesh.bface_cell, dtype=np.int32)
        self.bface_area = np.ascontiguousarray(mesh.bface_area, dtype=np.float64)
        nz = n_zones if n_zones is not None else getattr(mesh, "n_zones", 1)
        self.s = Mesh(self.volume.shape[0], self.edges.shape[0], self.bface_cell.shape[0], int(nz), 0,
                      _ptr(self.edges), _ptr(self.area), _ptr(self.volume), _ptr(self.zone),
                      _ptr(self.bface_cell), _ptr(self.bface_area))


def _options(storage="f64", outer="exact", ordering="auto", factor_slots=0, user_colour=None, device=0):
    uc = None if user_colour is None else np.ascontiguousarray(user_colour, dtype=np.int32)
    o = Options(STORAGE[storage], OUTER[outer], ORDERING[ordering], int(factor_slots), _ptr(uc), int(device), 0)
    return o, uc


def order_mesh(mesh, ordering="auto", user_colour=None):
    """Host-only: the colouring and internal permutation fnlh_create would build."""
    m = _MeshArrays(mesh)
    o, uc = _options(ordering=ordering, user_colour=user_colour)
    n = m.s.n_cells
    colour = np.empty(n, np.int32)
    perm = np.empty(n, np.int32)
    nc = C.c_int32(0)
    rc = LIB.fnlh_order_mesh(C.byref(m.s), C.byref(o), _ptr(colour), _ptr(perm), C.byref(nc))
    if rc != OK:
        raise FnlhError(rc, LIB.fnlh_last_error(None).decode())
    return colour, perm, nc.value


class Context:
    """One mesh, one stored Jacobian, any number of shifted systems."""

    def __init__(self, mesh, storage="f64", outer="exact", ordering="auto", factor_slots=0,
                 user_colour=None, device=0):
        self.mesh_arrays = _MeshArrays(mesh)
        self.n = int(self.mesh_arrays.s.n_cells)
        self.E = int(self.mesh_arrays.s.n_edges)
        self.B = int(self.mesh_arrays.s.n_bfaces)
        self.n_zones = int(self.mesh_arrays.s.n_zones)
        self.storage = storage
        self.device = int(device)
        o, uc = _options(storage, outer, ordering, factor_slots, user_colour, device)
        h = C.c_void_p()
        rc = LIB.fnlh_create(C.byref(h), C.byref(self.mesh_arrays.s), C.byref(o))
        if rc != OK:
            raise FnlhError(rc, LIB.fnlh_last_error(None).decode())
        self.h = h
        self.n_sys = 0

    def _check(self, rc, allow_positive=False):
        if rc < 0 or (rc > 0 and not allow_positive):
            raise FnlhError(rc, LIB.fnlh_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            LIB.fnlh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def assemble_jacobian(self, state, bstate=None, eps=0.6, sigma=50.0, scheme="implicit", stream=None):
        _dev_tensor(state, (self.n, 6), "state", "float64", self.device)
        if bstate is not None:
            _dev_tensor(bstate, (self.B, 6), "bstate", "float64", self.device)
        self._check(LIB.fnlh_assemble_jacobian(self.h, _ptr(state), _ptr(bstate), float(eps), float(sigma),
                                               SCHEME[scheme], _stream(stream)))

    def set_blocks(self, diag, offd, stream=None):
        _dev_tensor(diag, (self.n, 6, 6), "diag", "float64", self.device)
        _dev_tensor(offd, (self.E, 2, 6, 6), "offd", "float64", self.device)
        self._check(LIB.fnlh_set_blocks(self.h, _ptr(diag), _ptr(offd), _stream(stream)))

    def get_blocks(self, stream=None):
        import torch
        diag = torch.empty((self.n, 6, 6), dtype=torch.float64, device="cuda")
        offd = torch.empty((self.E, 2, 6, 6), dtype=torch.float64, device="cuda")
        self._check(LIB.fnlh_get_blocks(self.h, _ptr(diag), _ptr(offd), _stream(stream)))
        return diag, offd

    def set_harmonics(self, omega, stream=None):
        om = np.ascontiguousarray(omega, dtype=np.float64).reshape(-1, self.n_zones)
        self._check(LIB.fnlh_set_harmonics(self.h, om.shape[0], _ptr(om), _stream(stream)))
        self.n_sys = om.shape[0]

    def set_phase_lag(self, edge_phase, sigma):
        """Per-system inter-blade phase angles on the mesh's periodic edges (edge_phase:
        int [E] in {-1, 0, 1}, sigma: [n_sys] radians); edge_phase None removes them."""
        if edge_phase is None:
            self._check(LIB.fnlh_set_phase_lag(self.h, None, 0, None))
            return
        ep = np.ascontiguousarray(edge_phase, dtype=np.int8).reshape(-1)
        sg = np.ascontiguousarray(sigma, dtype=np.float64).reshape(-1)
        if ep.size != self.E:
            raise ValueError(f"edge_phase: {ep.size} entries for {self.E} edges")
        self._check(LIB.fnlh_set_phase_lag(self.h, _ptr(ep), sg.size, _ptr(sg)))

    def residual(self, sys, x, b, r=None, stream=None):
        for t, nm in ((x, "x"), (b, "b")):
            _dev_tensor(t, (self.n, 6), nm, device=self.device)
        if r is not None:
            _dev_tensor(r, (self.n, 6), "r", device=self.device)
        n2 = C.c_double(0.0)
        self._check(LIB.fnlh_residual(self.h, int(sys), _ptr(x), _ptr(b), _ptr(r), C.byref(n2), _stream(stream)))
        return n2.value

    def residual_noalloc(self, sys, x, b, r=None, norm2=None, stream=None):
        """r = b - K_s x without device allocation (scratch held by the library); norm2:
        a float64 CUDA tensor of one element receiving ||r||^2 on the device, or None."""
        for t, nm in ((x, "x"), (b, "b")):
            _dev_tensor(t, (self.n, 6), nm, device=self.device)
        if r is not None:
            _dev_tensor(r, (self.n, 6), "r", device=self.device)
        if norm2 is not None:
            _dev_tensor(norm2, (1,), "norm2", "float64", self.device)
        self._check(LIB.fnlh_residual_noalloc(self.h, int(sys), _ptr(x), _ptr(b), _ptr(r), _ptr(norm2),
                                              _stream(stream)))

    def relax(self, systems, xs, bs, kind="dilu", max_sweeps=500, rtol=1e-8, check_every=8,
              inner_sweeps=0, inner_rtol=0.0, div_factor=0.0, use_graph=False, learn_every=0, history=False,
              stream=None):
        """Solve (K + i omega_s V) x = b for each s in ``systems``; xs (in: x0, out: x) and
        bs are complex128 CUDA tensors [N, 6].  Returns (status, list of report dicts), or
        with history=True (status, reports, histories): histories[j][m] the residual norm
        after m sweeps (entry sweeps: the returned x's)."""
        n = len(systems)
        if len(xs) != n or len(bs) != n:
            raise ValueError(f"{n} systems need {n} x and {n} b vectors")
        for t in list(xs) + list(bs):
            _dev_tensor(t, (self.n, 6), "vector", device=self.device)
        sysarr = np.ascontiguousarray(systems, dtype=np.int32)
        xp = (C.c_void_p * n)(*[_ptr(t) for t in xs])
        bp = (C.c_void_p * n)(*[_ptr(t) for t in bs])
        hist = np.full((n, int(max_sweeps) + 2), np.nan) if history else None
        o = RelaxOpts(KIND[kind], int(max_sweeps), float(rtol), int(check_every), int(inner_sweeps),
                      float(inner_rtol), float(div_factor), int(bool(use_graph)), int(learn_every), _ptr(hist),
                      0 if hist is None else hist.shape[1], 0)
        rep = (Report * n)()
        rc = LIB.fnlh_relax(self.h, n, _ptr(sysarr), C.cast(xp, C.c_void_p), C.cast(bp, C.c_void_p),
                            C.byref(o), C.cast(rep, C.c_void_p), _stream(stream))
        self._check(rc, allow_positive=True)
        reps = [r.as_dict() for r in rep]
        if history:
            return rc, reps, [h[:r["sweeps"] + 1] for h, r in zip(hist, reps)]
        return rc, reps

    def gmres(self, systems, xs, bs, kind="dilu", restart=20, max_iters=500, rtol=1e-8, inner_sweeps=1,
              use_graph=False, history=False, stream=None):
        """Restarted flexible GMRES with the DILU/SGS/Jacobi preconditioner, or the
        learned one (kind="learned": the attached Network's correction, then DILU sweeps),
        for up to 16 systems at once; xs (in: x0, out: x) and bs complex128 CUDA tensors
        [N, 6].
        Returns (status, reports) or, with history=True, (status, reports, histories) where
        histories[j] holds the residual norm after each iteration (index 0: ||r0||)."""
        n = len(systems)
        if len(xs) != n or len(bs) != n:
            raise ValueError(f"{n} systems need {n} x and {n} b vectors")
        for t in list(xs) + list(bs):
            _dev_tensor(t, (self.n, 6), "vector", device=self.device)
        sysarr = np.ascontiguousarray(systems, dtype=np.int32)
        xp = (C.c_void_p * n)(*[_ptr(t) for t in xs])
        bp = (C.c_void_p * n)(*[_ptr(t) for t in bs])
        o = GmresOpts(KIND[kind], int(restart), int(max_iters), int(inner_sweeps), float(rtol), int(bool(use_graph)), 0)
        rep = (GmresReport * n)()
        hist = np.full((n, int(max_iters) + 1), np.nan) if history else None
        rc = LIB.fnlh_gmres(self.h, n, _ptr(sysarr), C.cast(xp, C.c_void_p), C.cast(bp, C.c_void_p), C.byref(o),
                            C.cast(rep, C.c_void_p), _ptr(hist), _stream(stream))
        self._check(rc, allow_positive=True)
        reps = [r.as_dict() for r in rep]
        if history:
            return rc, reps, [h[:r["iters"] + 1] for h, r in zip(hist, reps)]
        return rc, reps

    def set_partitions(self, part, stream=None):
        """Drop the couplings between cells of different partitions (part: [N] int labels
        per user cell) from the matrix the solves use; None clears them."""
        if part is None:
            self._check(LIB.fnlh_set_partitions(self.h, None, _stream(stream)))
            return
        a = np.ascontiguousarray(part, dtype=np.int32)
        if a.shape != (self.n,):
            raise ValueError(f"part must have shape ({self.n},)")
        self._check(LIB.fnlh_set_partitions(self.h, _ptr(a), _stream(stream)))

    def set_frozen_turbulence(self, flags):
        """Per-system frozen-turbulence flags (leading 5x5 sub-system, sixth unknown held at
        zero); None clears them."""
        if flags is None:
            self._check(LIB.fnlh_set_frozen_turbulence(self.h, 0, None))
            return
        f = np.ascontiguousarray(np.asarray(flags).astype(np.int8))
        self._check(LIB.fnlh_set_frozen_turbulence(self.h, int(f.size), _ptr(f)))

    def rusanov_residual(self, state, bstate=None, stream=None):
        """R(Q) of the first-order Rusanov scheme (device [N, 6] float64) and ||R||^2."""
        import torch
        _dev_tensor(state, (self.n, 6), "state", "float64", self.device)
        if bstate is not None:
            _dev_tensor(bstate, (self.B, 6), "bstate", "float64", self.device)
        R = torch.empty_like(state)
        n2 = C.c_double(0.0)
        self._check(LIB.fnlh_rusanov_residual(self.h, _ptr(state), _ptr(bstate), _ptr(R), C.byref(n2),
                                              _stream(stream)))
        return R, n2.value

    @staticmethod
    def _lin(kind, max_sweeps, rtol, check_every, use_graph):
        return RelaxOpts(KIND[kind], int(max_sweeps), float(rtol), int(check_every), 0, 0.0, 0.0,
                         int(bool(use_graph)), 0)

    def rk_mean(self, sys, state, n_steps, eps=0.6, sigma=50.0, scheme="implicit", bstate=None, kind="dilu",
                max_sweeps=10, rtol=1e-2, check_every=10, use_graph=False, stream=None):
        """n_steps RK(5,3) pseudo-time steps of the mean flow (state updated in place);
        returns (status, ||R|| at the start of each step)."""
        _dev_tensor(state, (self.n, 6), "state", "float64", self.device)
        if bstate is not None:
            _dev_tensor(bstate, (self.B, 6), "bstate", "float64", self.device)
        hist = np.zeros(max(int(n_steps), 1))
        o = self._lin(kind, max_sweeps, rtol, check_every, use_graph)
        rc = LIB.fnlh_rk_mean(self.h, int(sys), _ptr(state), _ptr(bstate), int(n_steps), float(eps), float(sigma),
                              SCHEME[scheme], C.byref(o), _ptr(hist), _stream(stream))
        self._check(rc, allow_positive=True)
        return rc, hist[:int(n_steps)]

    def rk_harmonic(self, sys, qhat, fhat, n_steps, kind="dilu", max_sweeps=10, rtol=1e-2, check_every=10,
                    use_graph=False, stream=None):
        """n_steps RK(5,3) pseudo-time steps of harmonic sys about the assembled state
        (qhat updated in place); returns (status, ||R_l|| at the start of each step)."""
        for t, nm in ((qhat, "qhat"), (fhat, "fhat")):
            _dev_tensor(t, (self.n, 6), nm, device=self.device)
        hist = np.zeros(max(int(n_steps), 1))
        o = self._lin(kind, max_sweeps, rtol, check_every, use_graph)
        rc = LIB.fnlh_rk_harmonic(self.h, int(sys), _ptr(qhat), _ptr(fhat), int(n_steps), C.byref(o), _ptr(hist),
                                  _stream(stream))
        self._check(rc, allow_positive=True)
        return rc, hist[:int(n_steps)]

    def tune(self, sys_per_lane=0, lanes_per_row=0, wave_groups=None, hybrid=None, pilu_unit=None,
             pilu_threads=None):
        """Set the sweep-kernel shape (0 = automatic); wave_groups (0/1), hybrid (0/1:
        two-colour passes plus remainder passes for nearly two-coloured orderings),
        pilu_unit (kind "pilu": cells per work unit, 0 = automatic) and pilu_threads
        (kind "pilu": sweep workgroup size 64/128/256, 0 = automatic) when given."""
        self._check(LIB.fnlh_tune(self.h, 0, int(sys_per_lane)))
        self._check(LIB.fnlh_tune(self.h, 1, int(lanes_per_row)))
        if wave_groups is not None:
            self._check(LIB.fnlh_tune(self.h, 2, int(wave_groups)))
        if hybrid is not None:
            self._check(LIB.fnlh_tune(self.h, 3, int(hybrid)))
        if pilu_unit is not None:
            self._check(LIB.fnlh_tune(self.h, 4, int(pilu_unit)))
        if pilu_threads is not None:
            self._check(LIB.fnlh_tune(self.h, 5, int(pilu_threads)))

    def autotune(self, n_sys, rtol=1e-8, max_sweeps=6000, cache=None, stream=None):
        """Pick the sweep configuration (path, kernel shape, workgroup mapping) by the
        time of whole solves to rtol (native autotuner).  ``cache``: path of a JSON file
        keyed by mesh signature, storage, system count, tolerance and device; a hit
        applies the stored choice without timing."""
        import json
        key = None
        if cache:
            import torch
            col, nc = self.ordering()
            dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
            key = f"{self.n}:{self.E}:{nc}:{int(np.bincount(col).max())}:{self.storage}:{n_sys}:{rtol}:{dev}"
            try:
                db = json.load(open(cache))
            except (OSError, ValueError):
                db = {}
            if key in db:
                r = db[key]
                self.tune(r["sys_per_lane"], r["lanes_per_row"], wave_groups=r["wave_groups"], hybrid=r["hybrid"])
                return dict(r, cached=True)
        res = TuneResult()
        self._check(LIB.fnlh_autotune(self.h, int(n_sys), float(rtol), int(max_sweeps), C.byref(res),
                                      _stream(stream)))
        out = {k: getattr(res, k) for k, _ in res._fields_}
        if cache:
            try:
                db = json.load(open(cache))
            except (OSError, ValueError):
                db = {}
            db[key] = out
            with open(cache, "w") as f:
                json.dump(db, f, indent=1)
        return dict(out, cached=False)

    def stats_enable(self, on=True, period=1):
        self._check(LIB.fnlh_stats_enable(self.h, int(period) if on else 0))

    def stats(self):
        out = {}
        for name, k in KSTAT.items():
            st = KernelStats()
            self._check(LIB.fnlh_stats_get(self.h, k, C.byref(st)))
            out[name] = {"launches": st.launches, "total_ms": st.total_ms, "alg_bytes": st.alg_bytes}
        return out

    def ordering(self):
        colour = np.empty(self.n, np.int32)
        nc = C.c_int32(0)
        self._check(LIB.fnlh_get_ordering(self.h, _ptr(colour), C.byref(nc)))
        return colour, nc.value

    def memory(self):
        a, b, c = C.c_size_t(0), C.c_size_t(0), C.c_size_t(0)
        self._check(LIB.fnlh_memory(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return {"matrix_bytes": a.value, "factor_bytes": b.value, "vector_bytes": c.value}


class Batch:
    """Independent instances (contexts) solved together: one launch per colour phase and
    system-count group over all instances, sweeps replayed from a captured graph."""

    def __init__(self, contexts):
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        h = C.c_void_p()
        rc = LIB.fnlh_batch_create(C.byref(h), len(self.contexts), C.cast(arr, C.c_void_p))
        if rc != OK:
            raise FnlhError(rc, LIB.fnlh_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            LIB.fnlh_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_loop_cells(self, loop_cells):
        """Instances of at least loop_cells cells are iterated one after another inside
        relax (cache-resident working set); smaller ones share the batched launches."""
        rc = LIB.fnlh_batch_set_loop_cells(self.h, int(loop_cells))
        if rc < 0:
            raise FnlhError(rc, "batch: set_loop_cells")

    def _args(self, systems, xs, bs, kind, max_sweeps, rtol, check_every, inner_sweeps, inner_rtol, div_factor,
              use_graph, learn_every):
        n = len(self.contexts)
        nsys = np.array([len(sy) for sy in systems], np.int32)
        keep = []
        sys_ptrs = (C.c_void_p * n)()
        x_ptrs = (C.c_void_p * n)()
        b_ptrs = (C.c_void_p * n)()
        for i, ctx in enumerate(self.contexts):
            if len(xs[i]) != len(systems[i]) or len(bs[i]) != len(systems[i]):
                raise ValueError(f"instance {i}: {len(systems[i])} systems need as many x and b vectors")
            for t in list(xs[i]) + list(bs[i]):
                _dev_tensor(t, (ctx.n, 6), "vector", device=ctx.device)
            sa = np.ascontiguousarray(systems[i], dtype=np.int32)
            xa = (C.c_void_p * len(xs[i]))(*[_ptr(t) for t in xs[i]])
            ba = (C.c_void_p * len(bs[i]))(*[_ptr(t) for t in bs[i]])
            keep += [sa, xa, ba]
            sys_ptrs[i] = sa.ctypes.data
            x_ptrs[i] = C.cast(xa, C.c_void_p).value
            b_ptrs[i] = C.cast(ba, C.c_void_p).value
        o = RelaxOpts(KIND[kind], int(max_sweeps), float(rtol), int(check_every), int(inner_sweeps),
                      float(inner_rtol), float(div_factor), int(bool(use_graph)), int(learn_every))
        return nsys, sys_ptrs, x_ptrs, b_ptrs, o, keep

    def relax(self, systems, xs, bs, kind="dilu", max_sweeps=500, rtol=1e-8, check_every=8, inner_sweeps=0,
              inner_rtol=0.0, div_factor=0.0, use_graph=True, learn_every=0, stream=None):
        """systems[i]: system ids of instance i; xs[i][j], bs[i][j]: complex128 CUDA
        tensors [N_i, 6].  Returns (status, reports per instance)."""
        nsys, sys_ptrs, x_ptrs, b_ptrs, o, keep = self._args(systems, xs, bs, kind, max_sweeps, rtol, check_every,
                                                             inner_sweeps, inner_rtol, div_factor, use_graph,
                                                             learn_every)
        total = int(nsys.sum())
        rep = (Report * total)()
        rc = LIB.fnlh_batch_relax(self.h, _ptr(nsys), C.cast(sys_ptrs, C.c_void_p), C.cast(x_ptrs, C.c_void_p),
                                  C.cast(b_ptrs, C.c_void_p), C.byref(o), C.cast(rep, C.c_void_p), _stream(stream))
        if rc < 0:
            raise FnlhError(rc, LIB.fnlh_batch_last_error(self.h).decode())
        out, k = [], 0
        for i in range(len(self.contexts)):
            out.append([rep[k + j].as_dict() for j in range(nsys[i])])
            k += nsys[i]
        return rc, out

    def autotune(self, systems, xs, bs, candidates=(0, 40000, 80000, 160000, 1 << 40), kind="dilu",
                 max_sweeps=5000, rtol=1e-8, check_every=16, use_graph=True, stream=None):
        """Native batch autotuner over the size threshold of the schedule (see
        set_loop_cells): times a whole batched solve for each candidate, keeps the
        fastest; xs are overwritten with the solution of the picked schedule.  Returns
        (status, pick, {candidate: ms})."""
        nsys, sys_ptrs, x_ptrs, b_ptrs, o, keep = self._args(systems, xs, bs, kind, max_sweeps, rtol, check_every,
                                                             0, 0.0, 0.0, use_graph, 0)
        cand = np.ascontiguousarray(candidates, dtype=np.int64)
        ms = np.zeros(cand.size)
        pick = C.c_int64(0)
        rc = LIB.fnlh_batch_autotune(self.h, _ptr(nsys), C.cast(sys_ptrs, C.c_void_p), C.cast(x_ptrs, C.c_void_p),
                                     C.cast(b_ptrs, C.c_void_p), C.byref(o), int(cand.size), _ptr(cand),
                                     C.byref(pick), _ptr(ms), _stream(stream))
        if rc < 0:
            raise FnlhError(rc, LIB.fnlh_batch_last_error(self.h).decode())
        return rc, pick.value, {int(c): float(t) for c, t in zip(cand, ms)}


NN_PARAMS = 26624


class Network:
    """Learned preconditioner attached to one context (fnlh_nn_*): weights are a flat
    float32 array of NN_PARAMS values, W1..W5 each row-major [in][out]."""

    def __init__(self, ctx, hidden=64):
        self.ctx = ctx
        h = C.c_void_p()
        ctx._check(LIB.fnlh_nn_create(C.byref(h), ctx.h, int(hidden)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            LIB.fnlh_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
        if w.size != NN_PARAMS:
            raise ValueError(f"expected {NN_PARAMS} weights, got {w.size}")
        self.ctx._check(LIB.fnlh_nn_set_weights(self.h, _ptr(w)))

    def set_grad_groups(self, groups):
        """Workgroups of the gradient kernels (each sums the partials of several tiles
        when fewer than the tiles); 0 = automatic."""
        self.ctx._check(LIB.fnlh_nn_set_grad_groups(self.h, int(groups)))

    def get_weights(self):
        w = np.empty(NN_PARAMS, np.float32)
        self.ctx._check(LIB.fnlh_nn_get_weights(self.h, _ptr(w)))
        return w

    def apply(self, sys, r, dx=None, stream=None):
        import torch
        _dev_tensor(r, (self.ctx.n, 6), "r", device=self.ctx.device)
        if dx is None:
            dx = torch.empty_like(r)
        _dev_tensor(dx, (self.ctx.n, 6), "dx", device=self.ctx.device)
        self.ctx._check(LIB.fnlh_nn_apply(self.h, int(sys), _ptr(r), _ptr(dx), _stream(stream)))
        return dx

    @staticmethod
    def _lists(systems, rs, es, n_cells, device=None):
        n = len(systems)
        if len(rs) != n or len(es) != n:
            raise ValueError(f"{n} systems need {n} r and {n} e vectors")
        for t in list(rs) + list(es):
            _dev_tensor(t, (n_cells, 6), "vector", device=device)
        sa = np.ascontiguousarray(systems, dtype=np.int32)
        rp = (C.c_void_p * n)(*[_ptr(t) for t in rs])
        ep = (C.c_void_p * n)(*[_ptr(t) for t in es])
        return n, sa, rp, ep

    def loss_grad(self, systems, rs, es, stream=None):
        """Mean loss and its gradient (float32 [NN_PARAMS]) over pairs (r, e)."""
        n, sa, rp, ep = self._lists(systems, rs, es, self.ctx.n, self.ctx.device)
        g = np.empty(NN_PARAMS, np.float32)
        loss = C.c_double(0.0)
        self.ctx._check(LIB.fnlh_nn_loss_grad(self.h, n, _ptr(sa), C.cast(rp, C.c_void_p), C.cast(ep, C.c_void_p),
                                              _ptr(g), C.byref(loss), _stream(stream)))
        return loss.value, g

    def add_pairs(self, systems, rs, es, stream=None):
        n, sa, rp, ep = self._lists(systems, rs, es, self.ctx.n, self.ctx.device)
        self.ctx._check(LIB.fnlh_nn_add_pairs(self.h, n, _ptr(sa), C.cast(rp, C.c_void_p), C.cast(ep, C.c_void_p),
                                              _stream(stream)))

    def reserve_pairs(self, n, stream=None):
        self.ctx._check(LIB.fnlh_nn_reserve_pairs(self.h, int(n), _stream(stream)))

    def generate(self, systems, starts, snapshots, every, seed=0, stream=None):
        """Training pairs from the plain solver, generated in the library: random starts,
        `snapshots` x `every` DILU sweeps with b = 0, each snapshot stored as (-K x, -x)."""
        sa = np.ascontiguousarray(systems, dtype=np.int32)
        self.ctx._check(LIB.fnlh_nn_generate(self.h, int(sa.size), _ptr(sa), int(starts), int(snapshots), int(every),
                                             int(seed) & 0xFFFFFFFFFFFFFFFF, _stream(stream)))

    def get_pair(self, k, stream=None):
        """Stored pair k as (system, r, e), r and e complex128 CUDA tensors [N, 6]."""
        import torch
        r = torch.empty((self.ctx.n, 6), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        e = torch.empty_like(r)
        sy = C.c_int32(0)
        self.ctx._check(LIB.fnlh_nn_get_pair(self.h, int(k), C.byref(sy), _ptr(r), _ptr(e), _stream(stream)))
        return sy.value, r, e

    def save(self, path):
        """Checkpoint: FP32 weights, Adam moments and step count."""
        self.ctx._check(LIB.fnlh_nn_save(self.h, os.fsencode(path)))

    def load(self, path):
        self.ctx._check(LIB.fnlh_nn_load(self.h, os.fsencode(path)))

    def copy_state_from(self, other):
        """Take other's weights, Adam moments and step count (device to device)."""
        self.ctx._check(LIB.fnlh_nn_copy_state(self.h, other.h))

    def clear_pairs(self):
        self.ctx._check(LIB.fnlh_nn_clear_pairs(self.h))

    def n_pairs(self):
        n = C.c_int64(0)
        self.ctx._check(LIB.fnlh_nn_pairs(self.h, C.byref(n)))
        return n.value

    def train(self, steps, batch=8, lr=1e-3, seed=0, stream=None):
        """Adam steps on the stored pairs; returns the per-step batch losses."""
        loss = np.zeros(max(int(steps), 1), np.float32)
        self.ctx._check(LIB.fnlh_nn_train(self.h, int(steps), int(batch), float(lr), int(seed), _ptr(loss),
                                          _stream(stream)))
        return loss[:int(steps)]


def mfma_selftest(ctx, a_bits, bt_bits):
    """out = A B on the matrix cores for 64x64 BF16 operands given as uint16 bit patterns
    (bt_bits = B^T)."""
    a = np.ascontiguousarray(a_bits, dtype=np.uint16)
    bt = np.ascontiguousarray(bt_bits, dtype=np.uint16)
    out = np.empty((64, 64), np.float32)
    ctx._check(LIB.fnlh_nn_selftest(ctx.h, _ptr(a), _ptr(bt), _ptr(out)))
    return out


def version():
    return LIB.fnlh_version().decode()
