"""ctypes binding of librcurves.so (the C ABI declared in include/rcurves.h).

Argument marshalling only: every function here checks tensor placement,
dtype and shape, passes raw device pointers and the current HIP stream to
the library, and turns a non-zero status into :class:`RcError`.  No compute
happens in Python.  Loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librcurves.so")

RC_F64, RC_F32 = 0, 1
RC_C_BARYCENTER, RC_C_TOTAL_LENGTH, RC_C_EDGE_LENGTH = 1, 2, 4
RC_SURFACE_SPHERE, RC_SURFACE_TORUS = 1, 2
RC_SOLVE_DENSE, RC_SOLVE_PCG_JACOBI, RC_SOLVE_PCG_MG, RC_SOLVE_PCG_LEARNED, RC_SOLVE_MG_FMG = 0, 1, 2, 4, 5

STATUS = {
    0: "RC_OK", 1: "RC_ERR_ARG", 2: "RC_ERR_PARAM_RANGE", 3: "RC_ERR_DEGENERATE", 4: "RC_ERR_NONFINITE",
    5: "RC_ERR_NOT_CONVERGED", 6: "RC_ERR_PROJECTION", 7: "RC_ERR_LINESEARCH", 8: "RC_ERR_SINGULAR",
    9: "RC_ERR_NOMEM", 10: "RC_ERR_HIP", 11: "RC_ERR_UNSUPPORTED",
}

EXPORTED = [
    "rc_default_solve_opts", "rc_default_ls_opts", "rc_last_error", "rc_create", "rc_destroy", "rc_energy",
    "rc_differential", "rc_sobolev_apply", "rc_sobolev_apply_prec", "rc_sobolev_diag", "rc_assemble_dense",
    "rc_set_constraints", "rc_set_point_constraints", "rc_set_surface_constraints", "rc_set_tangent_constraints",
    "rc_constraint_values",
    "rc_constraint_count", "rc_project",
    "rc_sobolev_gradient",
    "rc_line_search_step", "rc_step", "rc_bh_differential", "rc_bh_refit_differential", "rc_bh_last_work",
    "rc_midpoint_differential",
    "rc_profile_enable", "rc_profile_read", "rc_lowp_assemble", "rc_lowp_apply", "rc_set_obstacle",
    "rc_set_penalties", "rc_set_surface_potential",
    "rc_create_batch", "rc_batch_size", "rc_batch_energies", "rc_batch_tiling", "rc_default_batch_opts",
    "rc_batch_set_constraints", "rc_batch_gradient", "rc_batch_step", "rc_batch_pcg_state", "rc_batch_autotune",
    "rc_batch_sobolev_apply", "rc_mlp_n_params", "rc_mlp_create", "rc_mlp_destroy", "rc_mlp_get", "rc_mlp_set", "rc_mlp_forward",
    "rc_mlp_backward", "rc_mlp_adam", "rc_learned_attach", "rc_learned_levels", "rc_learned_features",
    "rc_learned_targets", "rc_mlp_fit_step", "rc_sync_status",
    "rc_differential_noalloc", "rc_use_vertex_pairs", "rc_first_collision_time", "rc_bct_build", "rc_bct_stats",
    "rc_sobolev_apply_bct",
]

RC_FLAG_INPUT_NONFINITE, RC_FLAG_ZERO_EDGE, RC_FLAG_PAIR_OVERFLOW, RC_FLAG_RESULT_NONFINITE = 1, 2, 4, 8
RC_FLAG_NOT_CONVERGED, RC_FLAG_SINGULAR, RC_FLAG_PROJECTION, RC_FLAG_LINESEARCH = 16, 32, 64, 128


class RcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class SolveOpts(C.Structure):
    _fields_ = [("solver", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("replace_every", C.c_int32), ("mg_min_vertices", C.c_int32), ("cheb_degree", C.c_int32),
                ("op_f64", C.c_int32), ("lowp", C.c_int32), ("lowp_band", C.c_int32),
                ("lowp_min_vertices", C.c_int32), ("lowp_outer", C.c_int32), ("inner_tol", C.c_double),
                ("fallback_after", C.c_int32), ("bct_theta", C.c_double), ("bct_min_vertices", C.c_int32)]


class BatchOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("ls_rounds", C.c_int32), ("proj_iters", C.c_int32),
                ("proj_max_iter", C.c_int32), ("proj_tol", C.c_double), ("accept_tol", C.c_double),
                ("c_armijo", C.c_double), ("tau0", C.c_double), ("graph", C.c_int32), ("check_every", C.c_int32),
                ("coarse", C.c_int32), ("op_assembled", C.c_int32), ("refine", C.c_int32),
                ("inner_tol", C.c_double)]


class LsOpts(C.Structure):
    _fields_ = [("c_armijo", C.c_double), ("shrink", C.c_double), ("tau0", C.c_double),
                ("max_backtracks", C.c_int32), ("max_proj_iter", C.c_int32), ("proj_tol", C.c_double),
                ("proj_solve_tol", C.c_double), ("ccd", C.c_int32), ("bh_theta", C.c_double),
                ("bh_refit", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("energy", C.c_double), ("energy_new", C.c_double), ("grad_norm", C.c_double),
                ("residual", C.c_double), ("tau", C.c_double), ("iterations", C.c_int32),
                ("proj_solve_iterations", C.c_int32), ("backtracks", C.c_int32), ("proj_iters", C.c_int32),
                ("status", C.c_int32), ("sweeps", C.c_int32), ("t_eval_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("t_search_ms", C.c_double), ("fallback", C.c_int32), ("flags", C.c_uint32),
                ("tau_max", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Load librcurves.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = C.CDLL(LIB_PATH)
    P, I32, D, U32 = C.c_void_p, C.c_int32, C.c_double, C.c_uint32
    sig = {
        "rc_default_solve_opts": (None, [C.POINTER(SolveOpts)]),
        "rc_default_ls_opts": (None, [C.POINTER(LsOpts)]),
        "rc_last_error": (C.c_char_p, []),
        "rc_create": (I32, [I32, I32, P, D, D, I32, P, C.POINTER(P)]),
        "rc_destroy": (I32, [P]),
        "rc_energy": (I32, [P, P, P]),
        "rc_differential": (I32, [P, P, P, P]),
        "rc_sobolev_apply": (I32, [P, P, P, P]),
        "rc_sobolev_apply_prec": (I32, [P, P, P, P, I32]),
        "rc_sobolev_diag": (I32, [P, P, P]),
        "rc_assemble_dense": (I32, [P, P, P]),
        "rc_set_constraints": (I32, [P, U32, P, P, D, P]),
        "rc_set_point_constraints": (I32, [P, I32, P, P]),
        "rc_set_surface_constraints": (I32, [P, I32, P, I32, P]),
        "rc_set_tangent_constraints": (I32, [P, I32, P, P]),
        "rc_set_surface_potential": (I32, [P, I32, P, I32, P, D, D]),
        "rc_constraint_values": (I32, [P, P, P]),
        "rc_constraint_count": (I32, [P]),
        "rc_project": (I32, [P, P, P, P]),
        "rc_sobolev_gradient": (I32, [P, P, P, P, C.POINTER(SolveOpts), C.POINTER(Stats)]),
        "rc_line_search_step": (I32, [P, P, D, P, P, C.POINTER(LsOpts), C.POINTER(SolveOpts), C.POINTER(D),
                                      C.POINTER(Stats)]),
        "rc_step": (I32, [P, P, C.POINTER(SolveOpts), C.POINTER(LsOpts), C.POINTER(Stats)]),
        "rc_bh_differential": (I32, [P, P, D, I32, P, P]),
        "rc_bh_refit_differential": (I32, [P, P, D, P, P]),
        "rc_midpoint_differential": (I32, [P, P, P, P]),
        "rc_bh_last_work": (I32, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(I32), C.POINTER(I32)]),
        "rc_profile_enable": (I32, [P, I32]),
        "rc_profile_read": (I32, [P, I32, C.POINTER(D), C.POINTER(I32)]),
        "rc_lowp_assemble": (I32, [P, P, I32, I32, I32]),
        "rc_set_obstacle": (I32, [P, P, D, D]),
        "rc_set_penalties": (I32, [P, D, D, D, P]),
        "rc_create_batch": (I32, [I32, P, I32, I32, P, D, D, I32, P, P]),
        "rc_batch_size": (I32, [P]),
        "rc_batch_energies": (I32, [P, P, P, P]),
        "rc_batch_tiling": (I32, [P, I32, I32]),
        "rc_default_batch_opts": (None, [P]),
        "rc_batch_set_constraints": (I32, [P, P]),
        "rc_batch_gradient": (I32, [P, P, P, P, P]),
        "rc_batch_step": (I32, [P, P, P, P]),
        "rc_batch_pcg_state": (I32, [P, P, P]),
        "rc_batch_autotune": (I32, [P, P, C.c_char_p, C.POINTER(I32), C.POINTER(I32), C.POINTER(D)]),
        "rc_lowp_apply": (I32, [P, P, P, I32]),
        "rc_batch_sobolev_apply": (I32, [P, P, P, P, I32]),
        "rc_mlp_n_params": (I32, []),
        "rc_mlp_create": (I32, [P, P, C.POINTER(P)]),
        "rc_mlp_destroy": (I32, [P]),
        "rc_mlp_get": (I32, [P, P]),
        "rc_mlp_set": (I32, [P, P]),
        "rc_mlp_forward": (I32, [P, P, I32, P]),
        "rc_mlp_backward": (I32, [P, P, I32, P, P]),
        "rc_mlp_adam": (I32, [P, P, C.c_float]),
        "rc_learned_attach": (I32, [P, P]),
        "rc_sync_status": (I32, [P, C.POINTER(Stats)]),
        "rc_differential_noalloc": (I32, [P, I32, P, I32, D, D, P, P, P]),
        "rc_use_vertex_pairs": (I32, [P, I32]),
        "rc_first_collision_time": (I32, [P, P, P, D, P]),
        "rc_bct_build": (I32, [P, P, D, I32]),
        "rc_bct_stats": (I32, [P, C.POINTER(C.c_int64)]),
        "rc_sobolev_apply_bct": (I32, [P, P, P, P]),
        "rc_learned_levels": (I32, [P, I32, P, I32, C.POINTER(I32)]),
        "rc_learned_features": (I32, [P, P, I32, P, P]),
        "rc_learned_targets": (I32, [P, P, I32, P]),
        "rc_mlp_fit_step": (I32, [P, P, P, I32, C.c_float, C.POINTER(D), P]),
    }
    for name, (res, args) in sig.items():
        if not hasattr(lib, name):
            continue
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != 0:
        raise RcError(status, load().rc_last_error().decode())


def _ptr(t, shape=None, dtype=None, name="tensor"):
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch

    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_solve_opts(**kw):
    o = SolveOpts()
    load().rc_default_solve_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_batch_opts(**kw):
    o = BatchOpts()
    load().rc_default_batch_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_ls_opts(**kw):
    o = LsOpts()
    load().rc_default_ls_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def differential_noalloc(gamma, edges, alpha, beta, energy, dE):
    """rc_differential_noalloc: FP64 energy and differential with no context and no allocation.
    gamma, dE: device float64 [nV, 3]; edges: device int32 [nE, 2]; energy: device float64 [1] or None."""
    import torch

    nV = int(gamma.shape[0])
    if not isinstance(edges, torch.Tensor) or edges.dtype != torch.int32 or edges.ndim != 2 or edges.shape[1] != 2:
        raise TypeError("edges must be a device int32 tensor [n_edges, 2]")
    _check(load().rc_differential_noalloc(_ptr(gamma, (nV, 3), torch.float64, "gamma"), nV,
                                          _ptr(edges, None, torch.int32, "edges"), int(edges.shape[0]), float(alpha),
                                          float(beta), _ptr(energy, (1,), torch.float64, "energy"),
                                          _ptr(dE, (nV, 3), torch.float64, "dE"), _stream()))


class Context:
    """Owns one rc_ctx (one curve network) bound to the current stream."""

    def __init__(self, n_vertices, edges, alpha, beta, dtype=RC_F32):
        import torch

        lib = load()
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32))
        if e.ndim != 2 or e.shape[1] != 2:
            raise ValueError("edges must be [n_edges, 2]")
        self.nV, self.nE = int(n_vertices), int(e.shape[0])
        self.alpha, self.beta, self.dtype = float(alpha), float(beta), int(dtype)
        h = C.c_void_p()
        _check(lib.rc_create(self.nV, self.nE, e.ctypes.data_as(C.c_void_p), self.alpha, self.beta, self.dtype,
                             _stream(), C.byref(h)))
        self.h = h
        self._f64 = torch.float64

    def close(self):
        if getattr(self, "h", None):
            load().rc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _v(self, t, name):
        return _ptr(t, (self.nV, 3), self._f64, name)

    def rc_use_vertex_pairs(self, enable=True):
        _check(load().rc_use_vertex_pairs(self.h, 1 if enable else 0))

    def rc_bct_build(self, gamma, theta, leaf_size=32):
        _check(load().rc_bct_build(self.h, self._v(gamma, "gamma"), float(theta), int(leaf_size)))

    def rc_bct_stats(self):
        out = (C.c_int64 * 4)()
        _check(load().rc_bct_stats(self.h, out))
        return {"nodes": out[0], "far_blocks": out[1], "near_blocks": out[2], "near_pairs": out[3]}

    def rc_sobolev_apply_bct(self, gamma, X, Y):
        _check(load().rc_sobolev_apply_bct(self.h, self._v(gamma, "gamma"), self._v(X, "X"), self._v(Y, "Y")))

    def rc_first_collision_time(self, gamma, D, horizon, t):
        _check(load().rc_first_collision_time(self.h, self._v(gamma, "gamma"), self._v(D, "D"), float(horizon),
                                              _ptr(t, (1,), self._f64, "t")))

    def rc_energy(self, gamma, energy):
        _check(load().rc_energy(self.h, self._v(gamma, "gamma"), _ptr(energy, (1,), self._f64, "energy")))

    def rc_differential(self, gamma, energy, dE):
        _check(load().rc_differential(self.h, self._v(gamma, "gamma"), _ptr(energy, (1,), self._f64, "energy"),
                                      self._v(dE, "dE")))

    def rc_sobolev_apply(self, gamma, X, Y, prec=None):
        if prec is None:
            _check(load().rc_sobolev_apply(self.h, self._v(gamma, "gamma"), self._v(X, "X"), self._v(Y, "Y")))
        else:
            _check(load().rc_sobolev_apply_prec(self.h, self._v(gamma, "gamma"), self._v(X, "X"),
                                                self._v(Y, "Y"), int(prec)))

    def rc_sobolev_diag(self, gamma, diag):
        _check(load().rc_sobolev_diag(self.h, self._v(gamma, "gamma"), _ptr(diag, (self.nV,), self._f64, "diag")))

    def rc_assemble_dense(self, gamma, A):
        _check(load().rc_assemble_dense(self.h, self._v(gamma, "gamma"),
                                        _ptr(A, (self.nV, self.nV), self._f64, "A")))

    def rc_set_constraints(self, mask, gamma_ref, x0=None, total_len0=-1.0, edge_len0=None):
        x0p = None
        if x0 is not None:
            self._x0 = (C.c_double * 3)(*[float(v) for v in x0])
            x0p = C.cast(self._x0, C.c_void_p)
        _check(load().rc_set_constraints(self.h, int(mask), self._v(gamma_ref, "gamma_ref"), x0p,
                                         float(total_len0), _ptr(edge_len0, (self.nE,), self._f64, "edge_len0")))

    def rc_set_point_constraints(self, vertices=(), targets=()):
        """Pin vertices[j] to targets[j] (host sequences: ints, [m][3] floats)."""
        v = [int(i) for i in vertices]
        t = [float(x) for row in targets for x in row]
        if len(t) != 3 * len(v):
            raise ValueError("targets must hold three coordinates per vertex")
        self._pv = (C.c_int32 * max(len(v), 1))(*v)
        self._px = (C.c_double * max(len(t), 1))(*t)
        _check(load().rc_set_point_constraints(self.h, len(v), C.cast(self._pv, C.c_void_p),
                                               C.cast(self._px, C.c_void_p)))

    def rc_set_surface_constraints(self, kind=0, params=(), vertices=()):
        """Hold vertices on the sphere (kind 1, params c, r) or torus (kind 2, params c, R, r)."""
        v = [int(i) for i in vertices]
        p = [float(x) for x in params]
        self._sv = (C.c_int32 * max(len(v), 1))(*v)
        self._sp = (C.c_double * max(len(p), 5))(*p)
        _check(load().rc_set_surface_constraints(self.h, int(kind), C.cast(self._sp, C.c_void_p), len(v),
                                                 C.cast(self._sv, C.c_void_p)))

    def rc_set_tangent_constraints(self, edges=(), directions=()):
        """Hold the unit tangent of edges[j] parallel to directions[j]."""
        ed = [int(i) for i in edges]
        d = [float(x) for row in directions for x in row]
        if len(d) != 3 * len(ed):
            raise ValueError("directions must hold three coordinates per edge")
        self._te = (C.c_int32 * max(len(ed), 1))(*ed)
        self._td = (C.c_double * max(len(d), 1))(*d)
        _check(load().rc_set_tangent_constraints(self.h, len(ed), C.cast(self._te, C.c_void_p),
                                                 C.cast(self._td, C.c_void_p)))

    def rc_constraint_count(self):
        return int(load().rc_constraint_count(self.h))

    def rc_constraint_values(self, gamma, phi):
        _check(load().rc_constraint_values(self.h, self._v(gamma, "gamma"),
                                           _ptr(phi, (self.rc_constraint_count(),), self._f64, "phi")))

    def rc_project(self, gamma, X, Y):
        _check(load().rc_project(self.h, self._v(gamma, "gamma"), self._v(X, "X"), self._v(Y, "Y")))

    def rc_sobolev_gradient(self, gamma, dE, g, opts=None, check=True):
        """Returns the solve statistics; check=False returns them (with the status)
        instead of raising when the solve does not converge."""
        st = Stats()
        o = opts if opts is not None else default_solve_opts()
        status = load().rc_sobolev_gradient(self.h, self._v(gamma, "gamma"), self._v(dE, "dE"), self._v(g, "g"),
                                            C.byref(o), C.byref(st))
        if check or status != 5:  # RC_ERR_NOT_CONVERGED
            _check(status)
        return st.as_dict()

    def rc_line_search_step(self, gamma, energy0, dE, g, ls=None, so=None):
        st = Stats()
        tau = C.c_double(0.0)
        l = ls if ls is not None else default_ls_opts()
        o = so if so is not None else default_solve_opts()
        _check(load().rc_line_search_step(self.h, self._v(gamma, "gamma"), float(energy0), self._v(dE, "dE"),
                                          self._v(g, "g"), C.byref(l), C.byref(o), C.byref(tau), C.byref(st)))
        return tau.value, st.as_dict()

    def rc_step(self, gamma, so=None, ls=None):
        st = Stats()
        o = so if so is not None else default_solve_opts()
        l = ls if ls is not None else default_ls_opts()
        _check(load().rc_step(self.h, self._v(gamma, "gamma"), C.byref(o), C.byref(l), C.byref(st)))
        return st.as_dict()

    def rc_sync_status(self):
        """(status, flags): the rc_status the latched RC_FLAG_* bits mean, and the bits (then cleared)."""
        st = Stats()
        status = load().rc_sync_status(self.h, C.byref(st))
        return int(status), int(st.flags)

    def rc_bh_differential(self, gamma, theta, leaf_size, energy, dE):
        _check(load().rc_bh_differential(self.h, self._v(gamma, "gamma"), float(theta), int(leaf_size),
                                         _ptr(energy, (1,), self._f64, "energy"), self._v(dE, "dE")))

    def rc_bh_refit_differential(self, gamma, theta, energy, dE):
        _check(load().rc_bh_refit_differential(self.h, self._v(gamma, "gamma"), float(theta),
                                               _ptr(energy, (1,), self._f64, "energy"), self._v(dE, "dE")))

    def rc_midpoint_differential(self, gamma, energy, dE):
        _check(load().rc_midpoint_differential(self.h, self._v(gamma, "gamma"),
                                               _ptr(energy, (1,), self._f64, "energy"), self._v(dE, "dE")))

    def rc_profile_enable(self, enable=True):
        _check(load().rc_profile_enable(self.h, 1 if enable else 0))

    def rc_profile_read(self, which):
        ms, n = C.c_double(0.0), C.c_int32(0)
        _check(load().rc_profile_read(self.h, int(which), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def rc_lowp_assemble(self, gamma, fmt, band, with_f32=False):
        _check(load().rc_lowp_assemble(self.h, self._v(gamma, "gamma"), int(fmt), int(band), 1 if with_f32 else 0))

    def rc_lowp_apply(self, X, Y, f32=False):
        _check(load().rc_lowp_apply(self.h, self._v(X, "X"), self._v(Y, "Y"), 1 if f32 else 0))

    def rc_set_obstacle(self, center, radius, weight=1.0):
        self._c = (C.c_double * 3)(*[float(v) for v in center])
        _check(load().rc_set_obstacle(self.h, C.cast(self._c, C.c_void_p), float(radius), float(weight)))

    def rc_set_penalties(self, w_length=0.0, w_diff=0.0, w_field=0.0, field=(0.0, 0.0, 1.0)):
        self._f = (C.c_double * 3)(*[float(v) for v in field])
        _check(load().rc_set_penalties(self.h, float(w_length), float(w_diff), float(w_field),
                                       C.cast(self._f, C.c_void_p)))

    def rc_set_surface_potential(self, P, F, weight=1.0, theta=0.0):
        """Triangulated-surface potential of the mesh (P [nP][3], F [nF][3]) with a weight and
        tree opening parameter theta (0 = every triangle)."""
        P = np.ascontiguousarray(P, dtype=np.float64).reshape(-1, 3)
        F = np.ascontiguousarray(F, dtype=np.int32).reshape(-1, 3)
        self._spP, self._spF = P, F
        _check(load().rc_set_surface_potential(self.h, len(P), P.ctypes.data_as(C.c_void_p), len(F),
                                               F.ctypes.data_as(C.c_void_p), float(weight), float(theta)))

    def rc_bh_last_work(self):
        f, n, nodes, depth = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32()
        _check(load().rc_bh_last_work(self.h, C.byref(f), C.byref(n), C.byref(nodes), C.byref(depth)))
        return {"far": f.value, "near": n.value, "nodes": nodes.value, "depth": depth.value}

    # learned smoother weights of the V-cycle
    def rc_learned_attach(self, mlp):
        self._mlp = mlp  # the context does not own it: keep it alive
        _check(load().rc_learned_attach(self.h, None if mlp is None else mlp.h))

    def rc_learned_levels(self, n_min):
        sizes, nl = (C.c_int32 * 64)(), C.c_int32()
        _check(load().rc_learned_levels(self.h, int(n_min), C.cast(sizes, C.c_void_p), 64, C.byref(nl)))
        return [sizes[i] for i in range(nl.value)]

    def rc_learned_features(self, gamma, n_min, X, diag=None):
        import torch

        N = sum(self.rc_learned_levels(n_min))
        _check(load().rc_learned_features(self.h, self._v(gamma, "gamma"), int(n_min),
                                          _ptr(X, (N, 8), torch.float32, "X"),
                                          None if diag is None else _ptr(diag, (N,), self._f64, "diag")))

    def rc_learned_targets(self, gamma, n_min, R):
        import torch

        N = sum(self.rc_learned_levels(n_min))
        _check(load().rc_learned_targets(self.h, self._v(gamma, "gamma"), int(n_min),
                                         _ptr(R, (N,), torch.float32, "R")))


def mlp_n_params():
    return int(load().rc_mlp_n_params())


class Mlp:
    """Owns one rc_mlp (the network of the learned smoother weights) on the current stream."""

    def __init__(self, theta=None):
        lib = load()
        self.n = mlp_n_params()
        h = C.c_void_p()
        t = None
        if theta is not None:
            t = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
            if t.shape != (self.n,):
                raise ValueError(f"theta must have {self.n} entries")
        _check(lib.rc_mlp_create(None if t is None else t.ctypes.data_as(C.c_void_p), _stream(), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().rc_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self):
        out = np.zeros(self.n, dtype=np.float32)
        _check(load().rc_mlp_get(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set(self, theta):
        t = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
        if t.shape != (self.n,):
            raise ValueError(f"theta must have {self.n} entries")
        _check(load().rc_mlp_set(self.h, t.ctypes.data_as(C.c_void_p)))

    def forward(self, X, Y):
        import torch

        N = int(X.shape[0])
        _check(load().rc_mlp_forward(self.h, _ptr(X, (N, 8), torch.float32, "X"), N,
                                     _ptr(Y, (N,), torch.float32, "Y")))

    def backward(self, X, dY, grad):
        import torch

        N = int(X.shape[0])
        _check(load().rc_mlp_backward(self.h, _ptr(X, (N, 8), torch.float32, "X"), N,
                                      _ptr(dY, (N,), torch.float32, "dY"),
                                      _ptr(grad, (self.n,), torch.float32, "grad")))

    def adam(self, grad, lr):
        import torch

        _check(load().rc_mlp_adam(self.h, _ptr(grad, (self.n,), torch.float32, "grad"), float(lr)))

    def fit_step(self, X, R, lr, grad=None):
        """One regression step on (X, R); returns the loss before the step."""
        import torch

        N = int(X.shape[0])
        loss = C.c_double()
        _check(load().rc_mlp_fit_step(self.h, _ptr(X, (N, 8), torch.float32, "X"), _ptr(R, (N,), torch.float32, "R"),
                                      N, float(lr), C.byref(loss),
                                      None if grad is None else _ptr(grad, (self.n,), torch.float32, "grad")))
        return loss.value


class Batch(Context):
    """A batch context: independent instances (vertex ranges) in one library context."""

    def __init__(self, inst_vertex_off, edges, alpha, beta, dtype=RC_F32):
        lib = load()
        off = np.ascontiguousarray(np.asarray(inst_vertex_off, dtype=np.int32))
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32))
        if off.ndim != 1 or len(off) < 2:
            raise ValueError("inst_vertex_off must be [n_inst + 1]")
        if e.ndim != 2 or e.shape[1] != 2:
            raise ValueError("edges must be [n_edges, 2]")
        self.nV, self.nE, self.n_inst = int(off[-1]), int(e.shape[0]), len(off) - 1
        self.alpha, self.beta, self.dtype = float(alpha), float(beta), int(dtype)
        h = C.c_void_p()
        _check(lib.rc_create_batch(self.n_inst, off.ctypes.data_as(C.c_void_p), self.nV, self.nE,
                                   e.ctypes.data_as(C.c_void_p), self.alpha, self.beta, self.dtype, _stream(),
                                   C.byref(h)))
        self.h = h
        import torch

        self._f64 = torch.float64

    def rc_batch_energies(self, gamma, energies, dE=None):
        _check(load().rc_batch_energies(self.h, self._v(gamma, "gamma"),
                                        _ptr(energies, (self.n_inst,), self._f64, "energies"),
                                        None if dE is None else self._v(dE, "dE")))

    def rc_batch_tiling(self, src_chunk, blocks_per_cu):
        _check(load().rc_batch_tiling(self.h, int(src_chunk), int(blocks_per_cu)))

    def rc_batch_set_constraints(self, gamma_ref):
        _check(load().rc_batch_set_constraints(self.h, self._v(gamma_ref, "gamma_ref")))

    def rc_batch_gradient(self, gamma, dE, g, opts=None):
        o = opts if opts is not None else default_batch_opts()
        _check(load().rc_batch_gradient(self.h, self._v(gamma, "gamma"), self._v(dE, "dE"), self._v(g, "g"),
                                        C.byref(o)))

    def rc_batch_step(self, gamma, opts=None, stats=True):
        o = opts if opts is not None else default_batch_opts()
        out = np.zeros((self.n_inst, 8)) if stats else None
        _check(load().rc_batch_step(self.h, self._v(gamma, "gamma"), C.byref(o),
                                    None if out is None else out.ctypes.data_as(C.c_void_p)))
        return out

    def rc_batch_autotune(self, gamma, cache_path=None):
        a, b, ms = C.c_int32(), C.c_int32(), C.c_double()
        path = None if cache_path is None else str(cache_path).encode()
        _check(load().rc_batch_autotune(self.h, self._v(gamma, "gamma"), path, C.byref(a), C.byref(b), C.byref(ms)))
        return {"src_chunk": a.value, "blocks_per_cu": b.value, "ms": ms.value}

    def rc_batch_sobolev_apply(self, gamma, X, Y, assembled=True):
        _check(load().rc_batch_sobolev_apply(self.h, self._v(gamma, "gamma"), self._v(X, "X"), self._v(Y, "Y"),
                                             1 if assembled else 0))

    def rc_batch_pcg_state(self):
        it, res = np.zeros(self.n_inst), np.zeros(self.n_inst)
        _check(load().rc_batch_pcg_state(self.h, it.ctypes.data_as(C.c_void_p), res.ctypes.data_as(C.c_void_p)))
        return it, res
