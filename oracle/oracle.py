"""ctypes wrapper of the BHEM CPU oracle.

TEST INFRASTRUCTURE ONLY.  The oracle is a plain FP64 implementation of the
paper's formulas (arXiv 2312.14839, Sec. 3-4, 6.1 and Appendices A-B) used to
check the HIP library.  Only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of bench.py may import this module; the product path
never does.

Array conventions: nodal arrays are ``[nodes, 12]`` float64 with DOF
``3*k + component`` for kind k (0: x, 1: x_xi1, 2: x_xi2, 3: x_xi1xi2); per-patch
arrays are ``[48]`` with local DOF ``12*c + 3*k + component`` for corner
``c = p + 2q`` (node ``(i+p, j+q)`` of patch ``(i, j)``).
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")


class Shell(C.Structure):
    _fields_ = [
        ("n1", C.c_int32), ("n2", C.c_int32), ("periodic1", C.c_int32),
        ("dxi1", C.c_double), ("dxi2", C.c_double),
        ("young", C.c_double), ("poisson", C.c_double),
        ("thickness", C.c_double), ("density", C.c_double),
        ("gravity", C.c_double * 3), ("damping", C.c_double),
    ]


class NewtonOpts(C.Structure):
    _fields_ = [
        ("solver", C.c_int), ("pseudo", C.c_int), ("newton_maxit", C.c_int),
        ("newton_rtol", C.c_double), ("pcg_maxit", C.c_int), ("pcg_rtol", C.c_double),
    ]


class NewtonStats(C.Structure):
    _fields_ = [
        ("newton_iters", C.c_int), ("pcg_iters_total", C.c_int),
        ("ls_backtracks", C.c_int), ("pad", C.c_int),
        ("grad_norm0", C.c_double), ("grad_norm", C.c_double), ("grad_floor", C.c_double),
        ("reg_delta", C.c_double),
    ]


class NewtonTrace(C.Structure):
    _fields_ = [
        ("cap_iters", C.c_int), ("n_iters", C.c_int),
        ("delta", C.POINTER(C.c_double)), ("energy", C.POINTER(C.c_double)), ("slope", C.POINTER(C.c_double)),
        ("steepest", C.POINTER(C.c_int)), ("n_trials", C.POINTER(C.c_int)),
        ("alpha", C.POINTER(C.c_double)), ("e_trial", C.POINTER(C.c_double)),
        ("q_iter", C.POINTER(C.c_double)), ("d_iter", C.POINTER(C.c_double)),
    ]


class PointConstraint(C.Structure):
    _fields_ = [("pi", C.c_int), ("pj", C.c_int), ("t1", C.c_double), ("t2", C.c_double), ("kind", C.c_int),
                ("target", C.c_double * 3)]


class AlmOpts(C.Structure):
    _fields_ = [("n", C.c_int), ("pts", C.POINTER(PointConstraint)), ("penalty", C.c_double), ("tol", C.c_double),
                ("max_outer", C.c_int), ("lam", C.POINTER(C.c_double)), ("outer_iters", C.c_int),
                ("residual", C.c_double)]


def _load(path=_LIB_PATH):
    if not os.path.exists(path):
        from . import build_oracle
        build_oracle.build(out=path)
    lib = C.CDLL(path)
    d = C.POINTER(C.c_double)
    sp = C.POINTER(Shell)
    lib.orc_num_nodes.argtypes = [sp]
    lib.orc_patch_nodes.argtypes = [sp, C.c_int, C.c_int, C.POINTER(C.c_int)]
    lib.orc_hermite_1d.argtypes = [C.c_double, d, d, d]
    lib.orc_shape_functions.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, d]
    lib.orc_gauss4.argtypes = [d, d]
    for name in ("orc_patch_energy", "orc_patch_energy_voigt"):
        getattr(lib, name).argtypes = [sp, d, d]
        getattr(lib, name).restype = C.c_double
    lib.orc_patch_gradient.argtypes = [sp, d, d, d]
    lib.orc_patch_hessian.argtypes = [sp, d, d, C.c_int, d]
    lib.orc_patch_mass.argtypes = [sp, d, d]
    lib.orc_patch_gravity.argtypes = [sp, d, d]
    lib.orc_patch_energy_cs.argtypes = [sp, d, d, d, d, d]
    lib.orc_patch_gradient_cs.argtypes = [sp, d, d, d, d, d]
    lib.orc_energy.argtypes = [sp, d, d]
    lib.orc_energy.restype = C.c_double
    lib.orc_gradient.argtypes = [sp, d, d, d]
    lib.orc_gravity.argtypes = [sp, d, d]
    lib.orc_patch_pressure.argtypes = [sp, d, C.c_double, d]
    lib.orc_pressure_load.argtypes = [sp, d, C.c_double, d]
    lib.orc_matrix_blocks.argtypes = [sp, d, d, C.c_int, C.c_int, C.c_int,
                                      C.POINTER(C.c_int), C.POINTER(C.c_int), d]
    lib.orc_matrix_blocks.restype = C.c_int
    lib.orc_matrix_dense.argtypes = [sp, d, d, C.c_int, C.c_int, d]
    lib.orc_newton_step.argtypes = [sp, d, C.POINTER(C.c_uint8), C.c_double, d, d, d, d,
                                    C.POINTER(NewtonOpts), d, d, C.POINTER(NewtonStats)]
    lib.orc_newton_step.restype = C.c_int
    lib.orc_newton_step_traced.argtypes = [sp, d, C.POINTER(C.c_uint8), C.c_double, d, d, d, d,
                                           C.POINTER(NewtonOpts), d, d, C.POINTER(NewtonStats),
                                           C.POINTER(NewtonTrace)]
    lib.orc_newton_step_traced.restype = C.c_int
    lib.orc_newton_step_alm.argtypes = [sp, d, C.POINTER(C.c_uint8), C.c_double, d, d, d, d,
                                        C.POINTER(NewtonOpts), d, d, C.POINTER(NewtonStats), C.POINTER(AlmOpts)]
    lib.orc_newton_step_alm.restype = C.c_int
    lib.orc_linear_solve.argtypes = [sp, d, d, C.POINTER(C.c_uint8), C.c_double, C.c_int, d, d,
                                     C.c_double, C.c_int, C.POINTER(C.c_int)]
    lib.orc_linear_solve.restype = C.c_int
    i64 = C.POINTER(C.c_int64)
    lib.orc_bh_to_bezier.argtypes = [d, C.c_double, C.c_double, d]
    lib.orc_bezier_eval.argtypes = [d, C.c_double, C.c_double, d, d, d]
    lib.orc_ray_cast.argtypes = [d, C.c_int, d, C.c_double, C.c_int, C.c_double, C.c_double, C.c_int, d, i64]
    lib.orc_ray_cast.restype = C.c_int
    lib.orc_ray_cast_many.argtypes = [d, C.c_int, d, C.c_int64, C.c_double, C.c_int, C.c_double, C.c_double,
                                      C.c_int, d, C.POINTER(C.c_int), i64]
    lib.orc_ccd_many.argtypes = [d, d, C.c_int, d, C.c_int64, C.c_double, C.c_double, C.c_int, C.c_double,
                                 C.c_double, C.c_int, d, C.POINTER(C.c_int), i64]
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_shell(n1, n2, dxi1, dxi2, young, poisson, thickness, density,
               gravity=(0.0, 0.0, 0.0), periodic1=0, damping=0.0):
    s = Shell()
    s.damping = float(damping)
    s.n1, s.n2, s.periodic1 = int(n1), int(n2), int(periodic1)
    s.dxi1, s.dxi2 = float(dxi1), float(dxi2)
    s.young, s.poisson, s.thickness, s.density = float(young), float(poisson), float(thickness), float(density)
    for i in range(3):
        s.gravity[i] = float(gravity[i])
    return s


def shell_from_case(case):
    """Oracle shell description from a workload case (see the package's workloads module)."""
    return make_shell(case.n1, case.n2, case.dxi1, case.dxi2, case.young, case.poisson,
                      case.thickness, case.density, case.gravity, case.periodic1, getattr(case, "damping", 0.0))


# ------------------------------------------------------------------ basis
def hermite_1d(t):
    w, d1, d2 = (np.zeros((2, 2)) for _ in range(3))
    lib().orc_hermite_1d(float(t), _d(w), _d(d1), _d(d2))
    return w, d1, d2


def shape_functions(t1, t2, dxi1, dxi2):
    out = np.zeros((6, 16))
    lib().orc_shape_functions(float(t1), float(t2), float(dxi1), float(dxi2), _d(out))
    return out


def gauss4():
    th, w = np.zeros(4), np.zeros(4)
    lib().orc_gauss4(_d(th), _d(w))
    return th, w


# -------------------------------------------------------------- per patch
def num_nodes(shell):
    return lib().orc_num_nodes(C.byref(shell))


def patch_nodes(shell, pi, pj):
    n = (C.c_int * 4)()
    lib().orc_patch_nodes(C.byref(shell), int(pi), int(pj), n)
    return list(n)


def gather(shell, x, pi, pj):
    x = np.asarray(x).reshape(-1, 12)
    return np.concatenate([x[n] for n in patch_nodes(shell, pi, pj)])


def patch_energy(shell, q, qb, form="tensor"):
    q, qb = _f64(q), _f64(qb)
    f = lib().orc_patch_energy if form == "tensor" else lib().orc_patch_energy_voigt
    return f(C.byref(shell), _d(q), _d(qb))


def patch_gradient(shell, q, qb):
    q, qb = _f64(q), _f64(qb)
    g = np.zeros(48)
    lib().orc_patch_gradient(C.byref(shell), _d(q), _d(qb), _d(g))
    return g


def patch_hessian(shell, q, qb, pseudo=False):
    q, qb = _f64(q), _f64(qb)
    h = np.zeros((48, 48))
    lib().orc_patch_hessian(C.byref(shell), _d(q), _d(qb), int(pseudo), _d(h))
    return h


def patch_mass(shell, qb):
    qb = _f64(qb)
    m = np.zeros((48, 48))
    lib().orc_patch_mass(C.byref(shell), _d(qb), _d(m))
    return m


def patch_gravity(shell, qb):
    qb = _f64(qb)
    f = np.zeros(48)
    lib().orc_patch_gravity(C.byref(shell), _d(qb), _d(f))
    return f


def patch_energy_cs(shell, q, q_im, qb):
    q, q_im, qb = _f64(q), _f64(q_im), _f64(qb)
    re, im = C.c_double(), C.c_double()
    lib().orc_patch_energy_cs(C.byref(shell), _d(q), _d(q_im), _d(qb), C.byref(re), C.byref(im))
    return re.value, im.value


def patch_gradient_cs(shell, q, q_im, qb):
    q, q_im, qb = _f64(q), _f64(q_im), _f64(qb)
    gr, gi = np.zeros(48), np.zeros(48)
    lib().orc_patch_gradient_cs(C.byref(shell), _d(q), _d(q_im), _d(qb), _d(gr), _d(gi))
    return gr, gi


# ------------------------------------------------------------------ global
def energy(shell, q, qb):
    q, qb = _f64(q), _f64(qb)
    return lib().orc_energy(C.byref(shell), _d(q), _d(qb))


def gradient(shell, q, qb):
    q, qb = _f64(q), _f64(qb)
    g = np.zeros_like(q)
    lib().orc_gradient(C.byref(shell), _d(q), _d(qb), _d(g))
    return g


def gravity(shell, qb):
    qb = _f64(qb)
    f = np.zeros_like(qb)
    lib().orc_gravity(C.byref(shell), _d(qb), _d(f))
    return f


def patch_pressure(shell, q, p):
    """Nodal generalized force [48] of a pressure p on one patch at state q
    (per unit current area, along a_1 x a_2)."""
    q = _f64(q)
    f = np.zeros(48)
    lib().orc_patch_pressure(C.byref(shell), _d(q), float(p), _d(f))
    return f


def pressure_load(shell, q, p):
    """Nodal generalized force [nodes, 12] of a pressure p on the shell at state q."""
    q = _f64(q)
    f = np.zeros_like(q)
    lib().orc_pressure_load(C.byref(shell), _d(q), float(p), _d(f))
    return f


def matrix_blocks(shell, q, qb, which="hessian", pseudo=False):
    """Global matrix as node blocks: (rows[nb], cols[nb], vals[nb, 12, 12])."""
    q, qb = _f64(q), _f64(qb)
    w = 0 if which == "hessian" else 1
    nb = lib().orc_matrix_blocks(C.byref(shell), _d(q), _d(qb), w, int(pseudo), 0, None, None, None)
    rows = np.zeros(nb, np.int32)
    cols = np.zeros(nb, np.int32)
    vals = np.zeros((nb, 12, 12))
    lib().orc_matrix_blocks(C.byref(shell), _d(q), _d(qb), w, int(pseudo), nb,
                            rows.ctypes.data_as(C.POINTER(C.c_int)),
                            cols.ctypes.data_as(C.POINTER(C.c_int)), _d(vals))
    return rows, cols, vals


def matrix_dense(shell, q, qb, which="hessian", pseudo=False):
    q, qb = _f64(q), _f64(qb)
    n = q.size
    out = np.zeros((n, n))
    lib().orc_matrix_dense(C.byref(shell), _d(q), _d(qb), 0 if which == "hessian" else 1, int(pseudo), _d(out))
    return out


def newton_step(shell, qb, fixed, dt, qn, vn, qpresc=None, solver="ldlt", pseudo=False,
                newton_rtol=1e-10, newton_maxit=50, pcg_rtol=1e-10, pcg_maxit=100000, f_ext=None, trace=0,
                pressure=0.0, points=None, penalty=0.0, alm_tol=1e-10, max_outer=30, lam=None):
    """One implicit-Euler step (mass-proportional damping from shell.damping,
    optional external nodal forces f_ext [nodes, 12]).  Returns (status,
    q_next, v_next, stats dict); with trace = K > 0 the stats also hold
    "trace", a record of the first K Newton iterations (regulariser delta,
    energy, slope, steepest-descent fallback, line-search trials, iterate
    and direction of each)."""
    qb, qn, vn = _f64(qb), _f64(qn), _f64(vn)
    if pressure:
        # follower pressure, its direction taken at the step's start (a dead
        # load within the step, so the step stays a minimisation)
        pl = pressure_load(shell, qn, pressure).reshape(qn.shape)
        f_ext = pl if f_ext is None else _f64(f_ext).reshape(qn.shape) + pl
    fe = _f64(f_ext) if f_ext is not None else None
    fx = np.ascontiguousarray(fixed, dtype=np.uint8) if fixed is not None else None
    qp = _f64(qpresc) if qpresc is not None else None
    o = NewtonOpts(0 if solver == "ldlt" else 1, int(pseudo), int(newton_maxit), float(newton_rtol),
                   int(pcg_maxit), float(pcg_rtol))
    st = NewtonStats()
    q1, v1 = np.zeros_like(qn), np.zeros_like(qn)
    args = (C.byref(shell), _d(qb), fx.ctypes.data_as(C.POINTER(C.c_uint8)) if fx is not None else None,
            float(dt), _d(qn), _d(vn), _d(qp) if qp is not None else None,
            _d(fe) if fe is not None else None, C.byref(o), _d(q1), _d(v1), C.byref(st))
    if points is not None:
        # points: list of (pi, pj, t1, t2, kind, target[3]); lam: [3 n] start (zeros if None)
        arr = (PointConstraint * max(len(points), 1))()
        for k, (pi, pj, t1, t2, kind, tgt) in enumerate(points):
            arr[k].pi, arr[k].pj, arr[k].t1, arr[k].t2, arr[k].kind = int(pi), int(pj), float(t1), float(t2), int(kind)
            for c in range(3):
                arr[k].target[c] = float(tgt[c])
        lam_arr = np.zeros(3 * len(points)) if lam is None else np.array(lam, dtype=np.float64).reshape(-1).copy()
        al = AlmOpts(len(points), arr, float(penalty), float(alm_tol), int(max_outer), _d(lam_arr), 0, 0.0)
        rc = lib().orc_newton_step_alm(*args, C.byref(al))
        stats = {k: getattr(st, k) for k, _ in NewtonStats._fields_ if k != "pad"}
        stats.update(lam=lam_arr, outer_iters=al.outer_iters, residual=al.residual)
        return rc, q1, v1, stats
    if trace:
        K, n = int(trace), qn.size
        rec = {"delta": np.zeros(K), "energy": np.zeros(K), "slope": np.zeros(K),
               "steepest": np.zeros(K, np.int32), "n_trials": np.zeros(K, np.int32),
               "alpha": np.zeros((K, 20)), "e_trial": np.zeros((K, 20)),
               "q_iter": np.zeros((K, n)), "d_iter": np.zeros((K, n))}
        tr = NewtonTrace(K, 0, *[rec[k].ctypes.data_as(C.POINTER(C.c_int if rec[k].dtype == np.int32
                                                                   else C.c_double))
                                 for k in ("delta", "energy", "slope", "steepest", "n_trials", "alpha",
                                           "e_trial", "q_iter", "d_iter")])
        rc = lib().orc_newton_step_traced(*args, C.byref(tr))
        m = tr.n_iters
        rec = {k: v[:m] for k, v in rec.items()}
    else:
        rc = lib().orc_newton_step(*args)
        rec = None
    stats = {k: getattr(st, k) for k, _ in NewtonStats._fields_ if k != "pad"}
    if rec is not None:
        stats["trace"] = rec
    return rc, q1, v1, stats


def linear_solve(shell, q, qb, fixed, mass_scale, b, solver="ldlt", rtol=1e-10, maxit=100000):
    """Solve (K(q) + mass_scale M) x = b with identity rows/columns on fixed DOFs."""
    q, qb, b = _f64(q), _f64(qb), _f64(b)
    fx = np.ascontiguousarray(fixed, dtype=np.uint8) if fixed is not None else None
    x = np.zeros_like(b)
    its = C.c_int()
    rc = lib().orc_linear_solve(C.byref(shell), _d(q), _d(qb),
                                fx.ctypes.data_as(C.POINTER(C.c_uint8)) if fx is not None else None,
                                float(mass_scale), 0 if solver == "ldlt" else 1, _d(b), _d(x),
                                float(rtol), int(maxit), C.byref(its))
    return rc, x, its.value
