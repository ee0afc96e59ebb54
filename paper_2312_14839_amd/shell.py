"""ctypes binding of libbhem.so, the C ABI declared in include/bhem_shell.h.

Argument marshalling only: every step of the thin-shell hot path runs in the
library's HIP kernels.  Device arrays are passed as ``torch`` CUDA(HIP)
tensors, used for device memory and streams only.  Importing this module
fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbhem.so")

SHELL_OK = 0
SHELL_E_INVAL = -1
SHELL_E_NOMEM = -2
SHELL_E_DEVICE = -3
SHELL_E_NOT_CONVERGED = -4
SHELL_E_INDEFINITE = -5
SHELL_E_NONFINITE = -6
SHELL_E_LINESEARCH = -7
SHELL_FP64, SHELL_MIXED = 0, 1
SHELL_HESS_EXACT, SHELL_HESS_PSEUDO = 0, 1
SHELL_WS_NONE, SHELL_WS_MLP = 0, 1

STATUS_NAMES = {0: "OK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_NOT_CONVERGED",
                -5: "E_INDEFINITE", -6: "E_NONFINITE", -7: "E_LINESEARCH"}


class shell_desc(C.Structure):
    _fields_ = [
        ("n1", C.c_int32), ("n2", C.c_int32), ("periodic1", C.c_int32),
        ("dxi1", C.c_double), ("dxi2", C.c_double),
        ("ref_host", C.POINTER(C.c_double)), ("fixed_host", C.POINTER(C.c_uint8)),
        ("young", C.c_double), ("poisson", C.c_double),
        ("thickness", C.c_double), ("density", C.c_double),
        ("gravity", C.c_double * 3), ("damping", C.c_double),
    ]


class shell_opts(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("hessian", C.c_int32), ("warm_start", C.c_int32),
        ("newton_maxit", C.c_int32), ("pcg_maxit", C.c_int32),
        ("newton_rtol", C.c_double), ("pcg_rtol", C.c_double),
        ("device", C.c_int32), ("stream", C.c_void_p), ("graphs", C.c_int32), ("cg_resident", C.c_int32),
        ("device_newton", C.c_int32),
    ]


class shell_tune_result(C.Structure):
    _fields_ = [
        ("threads", C.c_int32), ("rows_per_block", C.c_int32), ("blocks", C.c_int32),
        ("default_threads", C.c_int32), ("default_rows_per_block", C.c_int32),
        ("candidates", C.c_int32), ("from_cache", C.c_int32),
        ("us_per_iter", C.c_double), ("us_per_iter_default", C.c_double),
        ("hess_waves", C.c_int32), ("energy_patches", C.c_int32),
        ("hess_us", C.c_double), ("hess_us_default", C.c_double), ("energy_us", C.c_double),
        ("energy_us_default", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class shell_step_stats(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("newton_iters", C.c_int32), ("pcg_iters_total", C.c_int32),
        ("ls_backtracks", C.c_int32), ("refine_sweeps", C.c_int32), ("warm_start_used", C.c_int32),
        ("grad_norm0", C.c_double), ("grad_norm", C.c_double), ("grad_floor", C.c_double),
        ("reg_delta", C.c_double),
        ("t_assemble_ms", C.c_double), ("t_pcg_ms", C.c_double), ("t_step_ms", C.c_double),
        ("alm_residual", C.c_double), ("alm_outer", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SHELL_T_NGROUPS = 5
TIMING_GROUPS = ["energy_grad", "hessian", "bj_factor", "cg", "spmv"]


class shell_timing(C.Structure):
    _fields_ = [
        ("ms", C.c_double * SHELL_T_NGROUPS), ("launches", C.c_int64 * SHELL_T_NGROUPS),
        ("patch_evals", C.c_int64), ("cg_iter_rows", C.c_int64), ("cg_iter_blocks", C.c_int64),
        ("cg_iters_max", C.c_int64),
    ]

    def as_dict(self):
        return {"ms": dict(zip(TIMING_GROUPS, self.ms[:])), "launches": dict(zip(TIMING_GROUPS, self.launches[:])),
                "patch_evals": self.patch_evals, "cg_iter_rows": self.cg_iter_rows,
                "cg_iter_blocks": self.cg_iter_blocks, "cg_iters_max": self.cg_iters_max}


class shell_ray_opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("newton_tol", C.c_double), ("hole", C.c_double),
                ("newton_iters", C.c_int32), ("max_depth", C.c_int32), ("heap_cap", C.c_int32),
                ("device", C.c_int32), ("stream", C.c_void_p)]


SHELL_COLLIDER_PLANE, SHELL_COLLIDER_SPHERE = 0, 1


class shell_collider(C.Structure):
    _fields_ = [("kind", C.c_int32), ("point", C.c_double * 3), ("normal", C.c_double * 3), ("radius", C.c_double)]


class shell_collide_opts(C.Structure):
    _fields_ = [("samples", C.c_int32), ("friction", C.c_double), ("push_out", C.c_double),
                ("simultaneous", C.c_double), ("rtol", C.c_double)]


class shell_collide_stats(C.Structure):
    _fields_ = [("t_contact", C.c_double), ("contacts", C.c_int32), ("approaching", C.c_int32),
                ("impulse_iters", C.c_int32), ("push_iters", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class shell_point_constraint(C.Structure):
    _fields_ = [("shell", C.c_int32), ("kind", C.c_int32), ("xi1", C.c_double), ("xi2", C.c_double),
                ("target", C.c_double * 3)]


class shell_alm_opts(C.Structure):
    _fields_ = [("penalty", C.c_double), ("tol", C.c_double), ("max_outer", C.c_int32)]


def colliders(specs):
    """shell_collider array from ("plane", point, normal) / ("sphere", centre, radius) tuples."""
    arr = (shell_collider * max(len(specs), 1))()
    for k, sp in enumerate(specs):
        c = arr[k]
        c.kind = SHELL_COLLIDER_PLANE if sp[0] == "plane" else SHELL_COLLIDER_SPHERE
        for i in range(3):
            c.point[i] = float(sp[1][i])
        if sp[0] == "plane":
            for i in range(3):
                c.normal[i] = float(sp[2][i])
        else:
            c.radius = float(sp[2])
    return arr


class ShellError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(the HIP library is required, there is no fallback)")
    lib = C.CDLL(LIB_PATH)
    P, vp = C.POINTER, C.c_void_p
    lib.shell_default_opts.argtypes = [P(shell_opts)]
    lib.shell_default_opts.restype = None
    lib.shell_create.argtypes = [P(shell_desc), C.c_int32, P(shell_opts), P(vp)]
    lib.shell_create.restype = C.c_int32
    lib.shell_destroy.argtypes = [vp]
    lib.shell_destroy.restype = None
    lib.shell_last_error.argtypes = [vp]
    lib.shell_last_error.restype = C.c_char_p
    lib.shell_sizes.argtypes = [vp, P(C.c_int32), P(C.c_int32), P(C.c_int64)]
    lib.shell_sizes.restype = C.c_int32
    lib.shell_energy_grad_hess.argtypes = [vp, vp, P(C.c_double), vp, C.c_int32]
    lib.shell_energy_grad_hess.restype = C.c_int32
    lib.shell_assemble.argtypes = [vp, vp, C.c_double, C.c_int32]
    lib.shell_assemble.restype = C.c_int32
    lib.shell_get_bsr.argtypes = [vp, C.c_int32, P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_double)]
    lib.shell_get_bsr.restype = C.c_int32
    lib.shell_spmv.argtypes = [vp, vp, vp, C.c_int32]
    lib.shell_spmv.restype = C.c_int32
    lib.shell_pcg_solve.argtypes = [vp, vp, vp, C.c_double, C.c_int32, P(C.c_int32), P(C.c_double)]
    lib.shell_pcg_solve.restype = C.c_int32
    lib.shell_newton_step.argtypes = [vp, C.c_double, vp, vp, vp, vp, vp, P(shell_step_stats)]
    lib.shell_newton_step.restype = C.c_int32
    lib.shell_timing_enable.argtypes = [vp, C.c_int32]
    lib.shell_timing_enable.restype = C.c_int32
    lib.shell_timing_get.argtypes = [vp, P(shell_timing)]
    lib.shell_timing_get.restype = C.c_int32
    lib.shell_set_pressure.argtypes = [vp, P(C.c_double)]
    lib.shell_set_pressure.restype = C.c_int32
    lib.shell_pressure_load.argtypes = [vp, vp, vp]
    lib.shell_pressure_load.restype = C.c_int32
    lib.shell_set_point_constraints.argtypes = [vp, P(shell_point_constraint), C.c_int32, P(shell_alm_opts)]
    lib.shell_set_point_constraints.restype = C.c_int32
    lib.shell_get_point_multipliers.argtypes = [vp, P(C.c_double)]
    lib.shell_get_point_multipliers.restype = C.c_int32
    lib.shell_set_point_multipliers.argtypes = [vp, P(C.c_double)]
    lib.shell_set_point_multipliers.restype = C.c_int32
    lib.shell_set_nodal_forces.argtypes = [vp, vp]
    lib.shell_set_nodal_forces.restype = C.c_int32
    lib.shell_point_load.argtypes = [P(shell_desc), C.c_double, C.c_double, P(C.c_double), P(C.c_double)]
    lib.shell_point_load.restype = C.c_int32
    lib.shell_autotune.argtypes = [vp, C.c_int32, P(shell_tune_result)]
    lib.shell_autotune.restype = C.c_int32
    lib.shell_set_patch_tiles.argtypes = [vp, C.c_int32, C.c_int32]
    lib.shell_set_patch_tiles.restype = C.c_int32
    lib.shell_set_assembly.argtypes = [vp, C.c_int32]
    lib.shell_set_assembly.restype = C.c_int32
    lib.shell_cg_trace_enable.argtypes = [vp, C.c_int32]
    lib.shell_cg_trace_enable.restype = C.c_int32
    lib.shell_cg_trace_get.argtypes = [vp, P(C.c_int32), P(C.c_int32), C.c_void_p]
    lib.shell_cg_trace_get.restype = C.c_int32
    lib.shell_mlp_set_params.argtypes = [vp, P(C.c_float)]
    lib.shell_mlp_set_params.restype = C.c_int32
    lib.shell_mlp_get_params.argtypes = [vp, P(C.c_float)]
    lib.shell_mlp_get_params.restype = C.c_int32
    lib.shell_mlp_forward.argtypes = [vp, vp, vp, C.c_int64]
    lib.shell_mlp_forward.restype = C.c_int32
    lib.shell_mlp_loss_grad.argtypes = [vp, vp, vp, C.c_int64, vp, C.c_int32, P(C.c_double), P(C.c_float)]
    lib.shell_mlp_loss_grad.restype = C.c_int32
    lib.shell_mlp_train.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_uint64,
                                    P(C.c_double)]
    lib.shell_mlp_train.restype = C.c_int32
    lib.shell_mlp_record.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, C.c_uint64]
    lib.shell_mlp_record.restype = C.c_int32
    lib.shell_mlp_recorded.argtypes = [vp, P(C.c_int64)]
    lib.shell_mlp_recorded.restype = C.c_int32
    lib.shell_collide_default_opts.argtypes = [P(shell_collide_opts)]
    lib.shell_collide_default_opts.restype = None
    lib.shell_collide.argtypes = [vp, C.c_double, vp, vp, vp, P(shell_collider), C.c_int32, P(shell_collide_opts),
                                  vp, vp, P(shell_collide_stats)]
    lib.shell_collide.restype = C.c_int32
    lib.shell_bezier.argtypes = [vp, vp, vp]
    lib.shell_bezier.restype = C.c_int32
    lib.shell_ray_default_opts.argtypes = [P(shell_ray_opts)]
    lib.shell_ray_default_opts.restype = None
    lib.shell_ray_cast.argtypes = [vp, C.c_int32, vp, C.c_int64, P(shell_ray_opts), vp, vp, vp]
    lib.shell_ray_cast.restype = C.c_int32
    lib.shell_ray_cast_noalloc.argtypes = [vp, C.c_int32, vp, C.c_int64, P(shell_ray_opts), vp, vp, vp]
    lib.shell_ray_cast_noalloc.restype = C.c_int32
    lib.shell_ccd.argtypes = [vp, vp, C.c_int32, vp, C.c_int64, C.c_double, P(shell_ray_opts), vp, vp, vp]
    lib.shell_ccd.restype = C.c_int32
    return lib


lib = _load()

EXPORTED = ["shell_default_opts", "shell_create", "shell_destroy", "shell_last_error", "shell_sizes",
            "shell_energy_grad_hess", "shell_assemble", "shell_get_bsr", "shell_spmv", "shell_pcg_solve",
            "shell_newton_step", "shell_timing_enable", "shell_timing_get", "shell_mlp_set_params",
            "shell_mlp_get_params", "shell_mlp_forward", "shell_mlp_loss_grad", "shell_mlp_train",
            "shell_mlp_record", "shell_mlp_recorded", "shell_autotune", "shell_set_patch_tiles", "shell_set_nodal_forces",
            "shell_cg_trace_enable", "shell_cg_trace_get", "shell_set_assembly",
            "shell_point_load", "shell_bezier", "shell_ray_default_opts", "shell_ray_cast", "shell_ray_cast_noalloc",
            "shell_ccd", "shell_collide_default_opts", "shell_collide", "shell_set_pressure", "shell_pressure_load",
            "shell_set_point_constraints", "shell_get_point_multipliers", "shell_set_point_multipliers"]

MLP_IN, MLP_HIDDEN, MLP_OUT = 60, 128, 12
MLP_PARAMS = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_OUT + MLP_OUT


def _ptr(t):
    """Device pointer of a contiguous torch tensor (or None)."""
    if t is None:
        return None
    assert t.is_contiguous(), "device arrays must be contiguous"
    return C.c_void_p(t.data_ptr())


def default_opts() -> shell_opts:
    o = shell_opts()
    lib.shell_default_opts(C.byref(o))
    return o


class ShellContext:
    """One context over one or more shells.  ``cases`` are objects with the
    fields of paper_2312_14839_amd.workloads.Case (n1, n2, periodic1, dxi1,
    dxi2, young, poisson, thickness, density, gravity, ref, fixed)."""

    def __init__(self, cases: Sequence, precision=SHELL_FP64, hessian=SHELL_HESS_EXACT,
                 newton_rtol=1e-10, pcg_rtol=1e-10, newton_maxit=50, pcg_maxit=100000,
                 device=0, stream=None, warm_start=SHELL_WS_NONE, graphs=True, cg_resident=True,
                 device_newton=True):
        self._keep = []
        self._lib = lib   # kept for close() during interpreter shutdown
        descs = (shell_desc * len(cases))()
        for k, cs in enumerate(cases):
            ref = np.ascontiguousarray(cs.ref, dtype=np.float64)
            fixed = np.ascontiguousarray(cs.fixed, dtype=np.uint8) if cs.fixed is not None else None
            self._keep += [ref, fixed]
            d = descs[k]
            d.n1, d.n2, d.periodic1 = int(cs.n1), int(cs.n2), int(cs.periodic1)
            d.dxi1, d.dxi2 = float(cs.dxi1), float(cs.dxi2)
            d.ref_host = ref.ctypes.data_as(C.POINTER(C.c_double))
            d.fixed_host = fixed.ctypes.data_as(C.POINTER(C.c_uint8)) if fixed is not None else None
            d.young, d.poisson = float(cs.young), float(cs.poisson)
            d.thickness, d.density = float(cs.thickness), float(cs.density)
            for i in range(3):
                d.gravity[i] = float(cs.gravity[i])
            d.damping = float(getattr(cs, "damping", 0.0))
        o = default_opts()
        o.precision, o.hessian, o.warm_start = int(precision), int(hessian), int(warm_start)
        o.newton_rtol, o.pcg_rtol = float(newton_rtol), float(pcg_rtol)
        o.newton_maxit, o.pcg_maxit = int(newton_maxit), int(pcg_maxit)
        o.device = int(device)
        o.graphs = int(bool(graphs))
        o.cg_resident = int(bool(cg_resident))
        o.device_newton = int(bool(device_newton))
        o.stream = C.c_void_p(stream) if stream else None
        h = C.c_void_p()
        rc = lib.shell_create(descs, len(cases), C.byref(o), C.byref(h))
        if rc != SHELL_OK:
            raise ShellError(rc, lib.shell_last_error(None).decode())
        self.h = h
        self.n_shells = len(cases)
        n, p, nb = C.c_int32(), C.c_int32(), C.c_int64()
        lib.shell_sizes(h, C.byref(n), C.byref(p), C.byref(nb))
        self.total_nodes, self.total_patches, self.nnzb = n.value, p.value, nb.value

    def close(self):
        if getattr(self, "h", None) and self._lib is not None:
            self._lib.shell_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, rc, allow=()):
        if rc != SHELL_OK and rc not in allow:
            raise ShellError(rc, lib.shell_last_error(self.h).decode())
        return rc

    def energy_grad_hess(self, q, grad=None, hessian=False):
        e = (C.c_double * self.n_shells)()
        self._check(lib.shell_energy_grad_hess(self.h, _ptr(q), e, _ptr(grad), int(hessian)))
        return np.array(e[:])

    def bezier(self, q, ctrl):
        """Bezier control points ctrl [total_patches, 4, 4, 3] of state q."""
        self._check(lib.shell_bezier(self.h, _ptr(q), _ptr(ctrl)))

    def assemble(self, q, mass_scale=0.0, elastic=True):
        self._check(lib.shell_assemble(self.h, _ptr(q), float(mass_scale), int(elastic)))

    def get_bsr(self, shell=0):
        nb = C.c_int32()
        self._check(lib.shell_get_bsr(self.h, shell, C.byref(nb), None, None, None))
        # nodes of this shell = len(row_ptr) - 1; query via a second call with arrays
        nblk = nb.value
        rows = self._shell_nodes(shell)
        row_ptr = np.zeros(rows + 1, np.int32)
        col_idx = np.zeros(nblk, np.int32)
        vals = np.zeros((nblk, 12, 12))
        self._check(lib.shell_get_bsr(self.h, shell, C.byref(nb),
                                      row_ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                                      col_idx.ctypes.data_as(C.POINTER(C.c_int32)),
                                      vals.ctypes.data_as(C.POINTER(C.c_double))))
        return row_ptr, col_idx, vals

    def _shell_nodes(self, shell):
        return self._node_counts[shell]

    def set_node_counts(self, counts: List[int]):
        self._node_counts = list(counts)

    def spmv(self, x, y, masked=True):
        self._check(lib.shell_spmv(self.h, _ptr(x), _ptr(y), int(masked)))

    def pcg_solve(self, b, x, rtol=1e-10, maxit=100000, allow_fail=False):
        its = (C.c_int32 * self.n_shells)()
        rel = (C.c_double * self.n_shells)()
        rc = lib.shell_pcg_solve(self.h, _ptr(b), _ptr(x), float(rtol), int(maxit), its, rel)
        if not allow_fail:
            self._check(rc)
        return rc, np.array(its[:]), np.array(rel[:])

    def newton_step(self, dt, q_n, v_n, q_presc, q_out, v_out, allow_fail=False):
        st = (shell_step_stats * self.n_shells)()
        rc = lib.shell_newton_step(self.h, float(dt), _ptr(q_n), _ptr(v_n), _ptr(q_presc), _ptr(q_out),
                                   _ptr(v_out), st)
        if not allow_fail:
            self._check(rc)
        return rc, [s.as_dict() for s in st]


    def collide(self, dt, q_n, q_np1, v, specs, q_out, v_out, **kw):
        """shell_collide against the colliders `specs` (see colliders());
        keyword arguments set shell_collide_opts fields.  Returns the stats."""
        o = shell_collide_opts()
        lib.shell_collide_default_opts(C.byref(o))
        for k, v_ in kw.items():
            setattr(o, k, v_)
        st = shell_collide_stats()
        self._check(lib.shell_collide(self.h, float(dt), _ptr(q_n), _ptr(q_np1), _ptr(v), colliders(specs),
                                      len(specs), C.byref(o), _ptr(q_out), _ptr(v_out), C.byref(st)))
        return st.as_dict()

    def set_pressure(self, pressures):
        """Pressure per shell (Pa, along a_1 x a_2); None removes it."""
        if pressures is None:
            self._check(lib.shell_set_pressure(self.h, None))
            return
        arr = np.ascontiguousarray(pressures, dtype=np.float64)
        assert arr.size == self.n_shells
        self._check(lib.shell_set_pressure(self.h, arr.ctypes.data_as(C.POINTER(C.c_double))))

    def pressure_load(self, q, f):
        self._check(lib.shell_pressure_load(self.h, _ptr(q), _ptr(f)))

    def set_point_constraints(self, points, penalty=1e4, tol=1e-10, max_outer=30):
        """Point constraints (shell, kind, xi1, xi2, target[3]) imposed by the
        augmented Lagrangian method in later Newton steps; [] removes them.
        Multipliers start at zero."""
        n = len(points)
        arr = (shell_point_constraint * max(n, 1))()
        for i, (sh, kind, xi1, xi2, tgt) in enumerate(points):
            arr[i].shell, arr[i].kind, arr[i].xi1, arr[i].xi2 = int(sh), int(kind), float(xi1), float(xi2)
            for k in range(3):
                arr[i].target[k] = float(tgt[k])
        o = shell_alm_opts(float(penalty), float(tol), int(max_outer))
        self._check(lib.shell_set_point_constraints(self.h, arr if n else None, n, C.byref(o)))
        self._n_points = n

    def point_multipliers(self):
        lam = np.zeros((getattr(self, "_n_points", 0), 3))
        self._check(lib.shell_get_point_multipliers(self.h, lam.ctypes.data_as(C.POINTER(C.c_double))))
        return lam

    def set_point_multipliers(self, lam):
        arr = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
        assert arr.size == 3 * getattr(self, "_n_points", 0)
        self._check(lib.shell_set_point_multipliers(self.h, arr.ctypes.data_as(C.POINTER(C.c_double))))

    def set_nodal_forces(self, f):
        self._check(lib.shell_set_nodal_forces(self.h, _ptr(f)))

    def cg_trace_enable(self, on=True):
        self._check(lib.shell_cg_trace_enable(self.h, int(bool(on))))

    def cg_trace_get(self):
        """The last CG launch's phase timestamps, uint64 [blocks][iters][6]
        (ticks of the GPU's 100 MHz constant clock)."""
        nb, it = C.c_int32(), C.c_int32()
        self._check(lib.shell_cg_trace_get(self.h, C.byref(nb), C.byref(it), None))
        out = np.zeros((nb.value, it.value, 6), np.uint64)
        self._check(lib.shell_cg_trace_get(self.h, C.byref(nb), C.byref(it), out.ctypes.data_as(C.c_void_p)))
        return out

    def set_assembly(self, single_launch):
        self._check(lib.shell_set_assembly(self.h, int(bool(single_launch))))

    def set_patch_tiles(self, hess_waves, energy_patches):
        self._check(lib.shell_set_patch_tiles(self.h, int(hess_waves), int(energy_patches)))

    def autotune(self, cg_iters=100):
        r = shell_tune_result()
        self._check(lib.shell_autotune(self.h, int(cg_iters), C.byref(r)))
        return r.as_dict()

    # ---- warm-start network
    def mlp_set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.size == MLP_PARAMS
        self._check(lib.shell_mlp_set_params(self.h, th.ctypes.data_as(C.POINTER(C.c_float))))

    def mlp_get_params(self):
        th = np.zeros(MLP_PARAMS, np.float32)
        self._check(lib.shell_mlp_get_params(self.h, th.ctypes.data_as(C.POINTER(C.c_float))))
        return th

    def mlp_forward(self, feat, out):
        self._check(lib.shell_mlp_forward(self.h, _ptr(feat), _ptr(out), int(feat.shape[0])))

    def mlp_loss_grad(self, feat, tgt, idx):
        loss = C.c_double()
        g = np.zeros(MLP_PARAMS, np.float32)
        self._check(lib.shell_mlp_loss_grad(self.h, _ptr(feat), _ptr(tgt), int(feat.shape[0]), _ptr(idx),
                                            int(idx.shape[0]), C.byref(loss),
                                            g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g

    def mlp_train(self, feat, tgt, n_samples, batch, steps, lr, seed=0):
        losses = np.zeros(max(int(steps), 1))
        self._check(lib.shell_mlp_train(self.h, _ptr(feat), _ptr(tgt), int(n_samples), int(batch), int(steps),
                                        float(lr), int(seed), losses.ctypes.data_as(C.POINTER(C.c_double))))
        return losses[:int(steps)]

    def mlp_record(self, feat, tgt, capacity, per_shell, seed=0):
        self._check(lib.shell_mlp_record(self.h, _ptr(feat), _ptr(tgt), int(capacity), int(per_shell), int(seed)))

    def mlp_recorded(self):
        n = C.c_int64()
        self._check(lib.shell_mlp_recorded(self.h, C.byref(n)))
        return n.value

    def timing_enable(self, on=True):
        self._check(lib.shell_timing_enable(self.h, int(on)))

    def timing_get(self):
        t = shell_timing()
        self._check(lib.shell_timing_get(self.h, C.byref(t)))
        return t.as_dict()


def point_load(case, xi1, xi2, force, f_nodal=None):
    """Add the consistent nodal load of a point force at parameter point
    (xi1, xi2) of `case` into f_nodal [nodes, 12] (new zeros if None)."""
    d = shell_desc()
    d.n1, d.n2, d.periodic1 = int(case.n1), int(case.n2), int(case.periodic1)
    d.dxi1, d.dxi2 = float(case.dxi1), float(case.dxi2)
    out = np.zeros((case.nodes, 12)) if f_nodal is None else f_nodal
    assert out.dtype == np.float64 and out.flags["C_CONTIGUOUS"] and out.shape == (case.nodes, 12)
    fv = (C.c_double * 3)(*[float(v) for v in force])
    rc = lib.shell_point_load(C.byref(d), float(xi1), float(xi2), fv, out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != SHELL_OK:
        raise ShellError(rc, "point outside the shell's parameter domain or invalid descriptor")
    return out


def ray_opts(**kw) -> shell_ray_opts:
    """shell_ray_opts with the library's defaults, then the given fields."""
    o = shell_ray_opts()
    lib.shell_ray_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def ray_cast(ctrl, rays, hit, patch, pops=None, stream=None, noalloc=False, **kw):
    """shell_ray_cast (shell_ray_cast_noalloc if ``noalloc``) on device
    tensors: ctrl [P, 4, 4, 3] float64 (or None for no patches), rays [n, 6]
    float64, hit [n, 3] float64, patch [n] int32, pops [n] int32 or None;
    ``stream`` a hipStream_t handle (int) or None for the null stream.
    Keyword arguments set fields of shell_ray_opts."""
    o = ray_opts(**kw)
    o.device = rays.device.index or 0
    o.stream = C.c_void_p(stream)  # None: the null stream
    n_patches = ctrl.shape[0] if ctrl is not None else 0
    fn = lib.shell_ray_cast_noalloc if noalloc else lib.shell_ray_cast
    rc = fn(_ptr(ctrl) if n_patches else None, n_patches, _ptr(rays), rays.shape[0], C.byref(o),
            _ptr(hit), _ptr(patch), _ptr(pops))
    if rc != SHELL_OK:
        raise ShellError(rc, lib.shell_last_error(None).decode())


def ccd(ctrl, vel, points, dt, hit, patch, pops=None, stream=None, **kw):
    """shell_ccd on device tensors: ctrl, vel [P, 4, 4, 3] float64 (or None
    for no patches), points [n, 6] float64, hit [n, 3] float64, patch [n]
    int32, pops [n] int32 or None.  Keyword arguments set shell_ray_opts."""
    o = ray_opts(**kw)
    o.device = points.device.index or 0
    o.stream = C.c_void_p(stream)  # None: the null stream
    n_patches = ctrl.shape[0] if ctrl is not None else 0
    rc = lib.shell_ccd(_ptr(ctrl) if n_patches else None, _ptr(vel) if n_patches else None, n_patches,
                       _ptr(points), points.shape[0], float(dt), C.byref(o), _ptr(hit), _ptr(patch), _ptr(pops))
    if rc != SHELL_OK:
        raise ShellError(rc, lib.shell_last_error(None).decode())


def context_for(cases, **kw) -> ShellContext:
    """ShellContext that also knows each shell's node count (for get_bsr)."""
    ctx = ShellContext(cases, **kw)
    ctx.set_node_counts([c.nodes for c in cases])
    return ctx
