"""Collision handling of a shell against static colliders (Sec. 6.2,
"Collision Handling") -- CPU oracle, TEST INFRASTRUCTURE ONLY.

Only tests/ and the benchmark's CPU-baseline leg may import this module; the
HIP library never does.  Dense numpy on top of the oracle's own shape
functions (Appendix A.1) and consistent mass matrix (Eq. mass), so only for
small grids.

The steps, in the section's order:
  1. sampling: the midsurface of every patch is sampled uniformly at s x s
     parameter points theta = ((a + 1/2)/s, (b + 1/2)/s);
  2. continuous detection: within a step the generalized coordinates move
     linearly from q^n to q^{n+1} (implicit Euler keeps the velocity
     constant over the step), so every sample moves on a straight line;
     its contact time is the earliest tau in [0, dt] at which it reaches a
     collider (plane: the root of a linear function; sphere: the smaller
     root of a quadratic; 0 if it starts on or inside);
  3. rollback to the earliest contact tau* (the state at tau*), keeping the
     step's velocity; the contacts resolved together are the samples whose
     contact time is within `simultaneous` * dt of tau* (the section's
     "earliest simultaneous collision pairs");
  4. impulses: zero restitution, each approaching contact c a linear
     constraint on the generalized velocities, n_c . v(xi_c) = 0 (with
     friction also the two tangential components), v(xi_c) = sum_I
     Phi^I(xi_c) qdot_I; the velocity change is dqdot = M^-1 J^T lambda with
     lambda the minimum-norm least-squares solution of
     (J M^-1 J^T) lambda = -J qdot (momentum: the generalized impulse
     J^T lambda changes M qdot); with friction each contact's tangential
     impulse is then scaled into the Coulomb cone |lambda_t| <= mu lambda_n
     (none if lambda_n <= 0) and dqdot recomputed;
  5. push-out: each resolved contact point moved to `push` (1e-4 m) off the
     collider along its normal, the position constraints
     n_c . (x(xi_c) - p_c) = push solved the same way: dq = M^-1 J_n^T mu.
Prescribed DOFs do not move: M^-1 acts on the free DOFs only.

Colliders: ("plane", point, unit normal) with the shell on the side the
normal points to; ("sphere", centre, radius) with the shell outside.
"""
import numpy as np

from . import oracle as O


def sample_thetas(s):
    """The s x s parameter points of one patch, (theta1, theta2), theta1 fastest."""
    g = (np.arange(s) + 0.5) / s
    return [(t1, t2) for t2 in g for t1 in g]


def _patch_dofs(shell, pi, pj):
    """Global DOF indices of the 48 local coordinates 12 c + 3 k + comp."""
    nodes = O.patch_nodes(shell, pi, pj)
    return np.array([12 * nodes[c] + 3 * k + comp for c in range(4) for k in range(4) for comp in range(3)])


def sample_operators(shell, s):
    """Per sample: (patch index, theta1, theta2, dofs[48], phi[16]) with
    x(xi) = sum_I phi[I] q[dofs of I] (I = 4 c + k)."""
    out = []
    for pj in range(shell.n2):
        for pi in range(shell.n1):
            dofs = _patch_dofs(shell, pi, pj)
            for t1, t2 in sample_thetas(s):
                phi = O.shape_functions(t1, t2, shell.dxi1, shell.dxi2)[0]
                out.append((pj * shell.n1 + pi, t1, t2, dofs, phi))
    return out


def point_of(op, q):
    """x(xi) of one sample at state q (flat [nodes*12])."""
    _, _, _, dofs, phi = op
    loc = q[dofs].reshape(16, 3)
    return phi @ loc


def contact_time(x0, x1, dt, col):
    """Earliest tau in [0, dt] at which the point moving from x0 (tau = 0) to
    x1 (tau = dt) reaches the collider, or inf."""
    v = (x1 - x0) / dt
    if col[0] == "plane":
        _, p, n = col
        d0 = n @ (x0 - p)
        if d0 <= 0.0:
            return 0.0
        dv = n @ v
        if dv >= 0.0:
            return np.inf
        t = -d0 / dv
        return t if t <= dt else np.inf
    _, c, R = col
    e = x0 - c
    c0 = e @ e - R * R
    if c0 <= 0.0:
        return 0.0
    a, b = v @ v, 2.0 * (e @ v)
    if b >= 0.0 or a == 0.0:
        return np.inf
    disc = b * b - 4.0 * a * c0
    if disc < 0.0:
        return np.inf
    t = (-b - np.sqrt(disc)) / (2.0 * a)
    return t if t <= dt else np.inf


def normal_and_point(x, col):
    """Collider normal at (and point on it nearest to) a contact at x."""
    if col[0] == "plane":
        _, p, n = col
        return n, x - (n @ (x - p)) * n
    _, c, R = col
    n = (x - c) / np.linalg.norm(x - c)
    return n, c + R * n


def tangents(n):
    """Two unit vectors spanning the plane normal to n (the axis least aligned with n, crossed)."""
    e = np.zeros(3)
    e[int(np.argmin(np.abs(n)))] = 1.0
    t1 = np.cross(e, n)
    t1 /= np.linalg.norm(t1)
    return t1, np.cross(n, t1)


def _masked_mass(shell, ref, fixed):
    M = O.matrix_dense(shell, ref, ref, "mass")
    fx = fixed.reshape(-1).astype(bool) if fixed is not None else np.zeros(M.shape[0], bool)
    M[fx, :] = 0.0
    M[:, fx] = 0.0
    M[fx, fx] = 1.0
    return M, fx


def _solve_constraints(M, fx, J, r):
    """Minimum-norm least-squares lambda of (J M^-1 J^T) lambda = r and
    dq = M^-1 J^T lambda (zero on prescribed DOFs)."""
    Jm = J.copy()
    Jm[:, fx] = 0.0
    Minv_Jt = np.linalg.solve(M, Jm.T)
    S = Jm @ Minv_Jt
    lam = np.linalg.lstsq(S, r, rcond=None)[0]
    return lam, Minv_Jt @ lam


def collide(shell, ref, fixed, dt, q_n, q_np1, v, colliders, s=3, mu=0.0, push=1e-4, simultaneous=1e-3):
    """One collision pass of a step (flat [nodes*12] or [nodes, 12] arrays).
    Returns a dict: t_star (inf: no contact), q, v (the state to continue
    from: the rolled-back, pushed-out positions and the responded velocity;
    q_np1 and v unchanged without contact), contacts (list of (sample,
    collider, normal, point)), lam (impulses: per contact lambda_n, or
    (lambda_n, lambda_t1, lambda_t2) with friction), mu_push."""
    qn, q1, vv = (np.asarray(a, dtype=np.float64).reshape(-1) for a in (q_n, q_np1, v))
    ops = sample_operators(shell, s)
    tc = np.full(len(ops), np.inf)
    cid = np.full(len(ops), -1)
    for i, op in enumerate(ops):
        x0, x1 = point_of(op, qn), point_of(op, q1)
        for k, col in enumerate(colliders):
            t = contact_time(x0, x1, dt, col)
            if t < tc[i]:
                tc[i], cid[i] = t, k
    t_star = tc.min() if len(tc) else np.inf
    if not np.isfinite(t_star):
        return {"t_star": np.inf, "q": q1.copy(), "v": vv.copy(), "contacts": [], "approach": [],
                "lam": np.zeros(0), "mu_push": np.zeros(0), "tc": tc}
    qs = qn + (t_star / dt) * (q1 - qn)
    chosen = [i for i in range(len(ops)) if tc[i] <= t_star + simultaneous * dt]
    contacts = []
    for i in chosen:
        x = point_of(ops[i], qs)
        n, p = normal_and_point(x, colliders[cid[i]])
        contacts.append((i, int(cid[i]), n, p))
    M, fx = _masked_mass(shell, ref, fixed)
    ndof = qn.size

    def row(i, d):
        _, _, _, dofs, phi = ops[i]
        r = np.zeros(ndof)
        r[dofs] = np.kron(phi, d)
        return r

    # impulses on the approaching contacts (zero restitution)
    approach = [c for c in contacts if c[2] @ point_of(ops[c[0]], vv) < 0.0]
    dirs = []
    for i, _, n, _ in approach:
        dirs.append([n] + (list(tangents(n)) if mu > 0.0 else []))
    m = 3 if mu > 0.0 else 1
    v_out = vv.copy()
    lam = np.zeros((len(approach), m))
    if approach:
        J = np.array([row(c[0], d) for c, ds in zip(approach, dirs) for d in ds])
        lam_flat, _ = _solve_constraints(M, fx, J, -J @ vv)
        lam = lam_flat.reshape(-1, m)
        if mu > 0.0:
            for c in range(len(lam)):
                ln, lt = lam[c, 0], lam[c, 1:]
                nt = np.linalg.norm(lt)
                if ln <= 0.0:
                    lam[c, 1:] = 0.0
                elif nt > mu * ln:
                    lam[c, 1:] = lt * (mu * ln / nt)
        Jm = J.copy()
        Jm[:, fx] = 0.0
        v_out = vv + np.linalg.solve(M, Jm.T @ lam.reshape(-1))
    # push-out of every resolved contact
    Jn = np.array([row(i, n) for i, _, n, _ in contacts])
    r = np.array([push - n @ (point_of(ops[i], qs) - p) for i, _, n, p in contacts])
    mu_push, dq = _solve_constraints(M, fx, Jn, r)
    return {"t_star": float(t_star), "q": qs + dq, "v": v_out, "contacts": contacts, "approach": approach,
            "lam": lam if mu > 0.0 else lam[:, 0], "mu_push": mu_push, "tc": tc, "q_rollback": qs}


def momentum(shell, ref, q, v):
    """Linear and angular momentum (about the origin) of the shell:
    P = integral rho h xdot dA = sum_IJ M_IJ qdot_J over position rows,
    L = integral rho h x x xdot dA = sum_IJ M_IJ q_I x qdot_J."""
    M = O.matrix_dense(shell, ref, ref, "mass")
    Mv = (M @ np.asarray(v).reshape(-1)).reshape(-1, 4, 3)
    qq = np.asarray(q).reshape(-1, 4, 3)
    P = Mv[:, 0, :].sum(axis=0)
    L = np.cross(qq, Mv).sum(axis=(0, 1))
    return P, L
