"""Ray--patch intersection in the CPU oracle (Sec. 5 of arXiv 2312.14839).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only tests/,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of bench.py may use
it.  Thin numpy wrappers over ``oracle/ray.cpp``:

* ``bezier_patch`` / ``bezier_grid``: the Bezier control points of bicubic
  Hermite patches (Sec. 5, the Bernstein form of the patch);
* ``bezier_eval``: x, x_u, x_v of a Bezier surface;
* ``ray_cast``: the static ray--patch intersection of Sec. 5.1 (AABB tests
  of Eq. ineqray, min-heap of candidate surfaces, De Casteljau splits,
  optional Newton acceleration with the split of Fig. subany);
* ``ccd``: the dynamic intersection of Sec. 5.2 (a moving point against
  moving patches over one step, boxes by Eq. ineqccd).

Control points are ``[patches, 4, 4, 3]`` float64, ``p[i, j]`` with ``i``
along xi1 (local parameter u) and ``j`` along xi2 (v); rays are ``[n, 6]``
(origin, direction).
"""
import ctypes as C

import numpy as np

from . import oracle as O

_i64 = C.POINTER(C.c_int64)


def bezier_patch(corner48, dxi1, dxi2):
    """Control points [4, 4, 3] of one patch from its corner DOFs [4, 12]
    (corner c = p + 2q for node (i+p, j+q))."""
    c = O._f64(np.asarray(corner48).reshape(48))
    out = np.empty(48)
    O.lib().orc_bh_to_bezier(O._d(c), float(dxi1), float(dxi2), O._d(out))
    return out.reshape(4, 4, 3)


def bezier_grid(shell, x):
    """Control points [n1*n2, 4, 4, 3] of every patch of an oracle ``Shell``
    at nodal state x [nodes, 12], patch p = pj*n1 + pi."""
    x = np.asarray(x).reshape(-1, 12)
    out = np.empty((shell.n1 * shell.n2, 4, 4, 3))
    nd = (C.c_int * 4)()
    for pj in range(shell.n2):
        for pi in range(shell.n1):
            O.lib().orc_patch_nodes(C.byref(shell), pi, pj, nd)
            out[pj * shell.n1 + pi] = bezier_patch(x[list(nd)], shell.dxi1, shell.dxi2)
    return out


def bezier_eval(ctrl, u, v):
    """(x, x_u, x_v) of one Bezier surface ctrl [4, 4, 3] at (u, v)."""
    c = O._f64(np.asarray(ctrl).reshape(48))
    x, xu, xv = np.empty(3), np.empty(3), np.empty(3)
    O.lib().orc_bezier_eval(O._d(c), float(u), float(v), O._d(x), O._d(xu), O._d(xv))
    return x, xu, xv


def ray_cast(ctrl, rays, eps=1e-10, newton_iters=0, newton_tol=1e-12, hole=1e-3, max_depth=60, stats=False):
    """Closest hit of each ray with the patches ctrl [P, 4, 4, 3].

    Returns (hit [n, 3] = tau, u, v with tau = inf on a miss, patch [n] int32
    with -1 on a miss) and, with ``stats``, [n, 2] int64 = surfaces popped and
    the largest heap size of each ray."""
    c = O._f64(np.asarray(ctrl).reshape(-1, 48))
    r = O._f64(np.asarray(rays).reshape(-1, 6))
    n = r.shape[0]
    hit = np.empty((n, 3))
    patch = np.empty(n, dtype=np.int32)
    st = np.empty((n, 2), dtype=np.int64)
    O.lib().orc_ray_cast_many(O._d(c), c.shape[0], O._d(r), n, float(eps), int(newton_iters), float(newton_tol),
                              float(hole), int(max_depth), O._d(hit), patch.ctypes.data_as(C.POINTER(C.c_int)),
                              st.ctypes.data_as(_i64))
    return (hit, patch, st) if stats else (hit, patch)


def ccd(ctrl, vel, points, dt, eps=1e-10, newton_iters=0, newton_tol=1e-12, hole=1e-3, max_depth=60, stats=False):
    """Earliest contact over [0, dt] of each moving point (points [n, 6]:
    x0, velocity) with the moving patches (ctrl, vel [P, 4, 4, 3]: control
    points and their velocities), Sec. 5.2.  Returns (hit [n, 3] = t, u, v,
    t = inf when there is none, patch [n] int32, -1 none) and, with
    ``stats``, [n, 2] int64 = candidates examined and the largest heap."""
    c = O._f64(np.asarray(ctrl).reshape(-1, 48))
    v = O._f64(np.asarray(vel).reshape(-1, 48))
    pts = O._f64(np.asarray(points).reshape(-1, 6))
    n = pts.shape[0]
    hit = np.empty((n, 3))
    patch = np.empty(n, dtype=np.int32)
    st = np.empty((n, 2), dtype=np.int64)
    O.lib().orc_ccd_many(O._d(c), O._d(v), c.shape[0], O._d(pts), n, float(dt), float(eps), int(newton_iters),
                         float(newton_tol), float(hole), int(max_depth), O._d(hit),
                         patch.ctypes.data_as(C.POINTER(C.c_int)), st.ctypes.data_as(_i64))
    return (hit, patch, st) if stats else (hit, patch)
