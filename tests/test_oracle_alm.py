"""Pins of the oracle's positional constraints at arbitrary midsurface points
(Sec. 4.2) imposed by the augmented Lagrangian method (Sec. 6.1), CPU only.

* KKT: at the result the constraints hold (max |c| <= tol) and the
  gradient of the incremental potential -- from the oracle's separate
  energy, mass and load routines -- equals C^T lambda: the multipliers are
  the constraint forces.
* A constraint placed exactly at a node is the nodal Dirichlet (kind 0) or
  Neumann (kind 1, 2) constraint of Sec. 4.2, which the oracle imposes by
  removing those DOFs: both steps must end at the same state.
* A target that moves with a free, unloaded sheet in uniform translation is
  met by the free motion: lambda = 0 and the step is the free flight.
Planted mistakes are caught (tests/test_oracle_mutants.py)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2312_14839_amd import workloads as W

from test_oracle_newton import Potential


def _C_rows(s, case, points):
    rows = []
    for (pi, pj, t1, t2, kind, _) in points:
        psi = O.shape_functions(t1, t2, s.dxi1, s.dxi2)[kind]
        nodes = O.patch_nodes(s, pi, pj)
        for comp in range(3):
            r = np.zeros(case.nodes * 12)
            for I in range(16):
                r[12 * nodes[I >> 2] + 3 * (I & 3) + comp] += psi[I]
            rows.append(r)
    return np.array(rows)


POINTS = [(4, 4, 0.4, 0.4, 0, (0.55, 0.55, 0.0)), (6, 2, 0.7, 0.25, 2, (0.0, 1.0, 0.05))]


def test_kkt_at_the_result():
    case = W.case_small_sheet()
    s = O.shell_from_case(case)
    rc, q1, _, st = O.newton_step(s, case.ref, case.fixed, case.dt, case.q0, case.v0, points=POINTS, penalty=1e4,
                                  alm_tol=1e-11)
    assert rc == 0 and st["outer_iters"] > 0 and st["residual"] <= 1e-11
    C = _C_rows(s, case, POINTS)
    tgt = np.concatenate([np.asarray(p[5], float) for p in POINTS])
    assert np.abs(C @ q1.reshape(-1) - tgt).max() <= 1e-11
    P = Potential(case, case.q0, case.v0)
    g = P.grad(q1.reshape(-1))
    force = C.T @ st["lam"]
    force[P.fixed] = 0.0
    assert np.linalg.norm(g - force) <= 1e-7 * np.linalg.norm(force), np.linalg.norm(g - force)
    assert np.linalg.norm(force) > 1e-3


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_constraint_at_a_node_is_the_nodal_constraint(kind):
    """Node (3, 5) is corner 0 of patch (3, 5) (theta = 0): prescribing x, x_xi1
    or x_xi2 there through the augmented Lagrangian equals fixing those three
    DOFs of the node."""
    case = W.case_small_sheet()
    s = O.shell_from_case(case)
    nd = 5 * 9 + 3
    target = case.q0[nd, 3 * kind:3 * kind + 3] + np.array([0.0, 0.0, 2e-3 if kind == 0 else 0.05])
    rc, q_alm, _, st = O.newton_step(s, case.ref, case.fixed, case.dt, case.q0, case.v0,
                                     points=[(3, 5, 0.0, 0.0, kind, target)], penalty=1e5, alm_tol=1e-12)
    assert rc == 0 and st["residual"] <= 1e-12
    fixed = case.fixed.copy()
    fixed[nd, 3 * kind:3 * kind + 3] = 1
    qp = case.q0.copy()
    qp[nd, 3 * kind:3 * kind + 3] = target
    rc2, q_fix, _, _ = O.newton_step(s, case.ref, fixed, case.dt, case.q0, case.v0, qpresc=qp)
    assert rc2 == 0
    disp = np.abs(q_fix - case.q0).max()
    assert np.abs(q_alm - q_fix).max() <= 1e-7 * disp, (np.abs(q_alm - q_fix).max(), disp)


def test_moving_target_of_a_free_sheet_needs_no_force():
    case = W.sheet_case(4, edges=(), sigma=0.0, gravity=(0.0, 0.0, 0.0))
    s = O.shell_from_case(case)
    v = np.zeros_like(case.ref)
    v[:, 0:3] = (0.2, -0.1, 0.3)
    dt = 1e-2
    x0 = np.array([0.3, 0.6, 0.0])    # the point (t1, t2) = (0.2, 0.4) of patch (1, 2)
    target = x0 + dt * v[0, 0:3]
    rc, q1, _, st = O.newton_step(s, case.ref, case.fixed, dt, case.ref, v, points=[(1, 2, 0.2, 0.4, 0, target)],
                                  penalty=1e3, alm_tol=1e-13)
    assert rc == 0
    np.testing.assert_allclose(st["lam"], 0.0, atol=1e-12)
    np.testing.assert_allclose(q1, case.ref + dt * v, rtol=0, atol=1e-13)
