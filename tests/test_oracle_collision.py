"""Pins of the collision-handling oracle (Sec. 6.2), CPU only.

Closed forms: a flat sheet dropped flat on a plane touches it everywhere at
t* = h / v_z, and zero restitution stops its normal velocity exactly while
the tangential velocity is kept (frictionless) or reduced by mu times the
normal change (Coulomb, sliding) or stopped (sticking); every resolved point
ends `push` off the plane.  Invariants: normal impulses on a plane leave the
horizontal momentum and the vertical angular momentum unchanged; on a
sphere every normal passes through its centre, so the angular momentum
about the centre is unchanged; after the response no approaching contact
still moves into its collider; prescribed DOFs never move; the rolled-back
state touches the collider at the earliest sample and nowhere penetrates.
Momenta are computed from the oracle's consistent mass matrix (itself
pinned to the textbook Hermite mass, see test_oracle_mechanics).
Planted mistakes in a copy of the oracle's source are each caught."""
import importlib.util
import os
import tempfile

import numpy as np
import pytest

from oracle import collision as OC
from oracle import oracle as O
from paper_2312_14839_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _flat_drop(n=3, h0=0.05, v=(0.3, -0.2, -2.0), dt=0.04):
    case = W.sheet_case(n, edges=(), sigma=0.0)
    s = O.shell_from_case(case)
    qn = case.ref.copy()
    qn[:, 2] += h0
    vv = np.zeros_like(qn)
    vv[:, 0:3] = v
    return case, s, qn, qn + dt * vv, vv, dt


def test_flat_drop_on_a_plane_closed_form(OCm=OC):
    case, s, qn, q1, v, dt = _flat_drop()
    r = OCm.collide(s, case.ref, case.fixed, dt, qn, q1, v, [("plane", np.zeros(3), np.array([0.0, 0.0, 1.0]))])
    assert abs(r["t_star"] - 0.05 / 2.0) <= 1e-15
    assert len(r["contacts"]) == 9 * case.patches
    vo, qo = r["v"].reshape(-1, 12), r["q"].reshape(-1, 12)
    # the constraint system is rank deficient here (9 samples per patch, 4
    # DOFs per node): its least-squares solution is resolved to ~1e-10 of
    # the velocity
    np.testing.assert_allclose(vo[:, 2], 0.0, atol=2e-9)
    np.testing.assert_allclose(vo[:, 0:2], v[:, 0:2], atol=2e-9)
    np.testing.assert_allclose(vo[:, 3:], 0.0, atol=2e-9)
    np.testing.assert_allclose(qo[:, 2], 1e-4, atol=1e-13)
    np.testing.assert_allclose(qo[:, 0:2], qn[:, 0:2] + r["t_star"] * v[:, 0:2], atol=1e-13)
    np.testing.assert_allclose(qo[:, 3:], qn[:, 3:], atol=1e-13)


@pytest.mark.parametrize("mu", [0.1, 10.0])
def test_flat_slide_coulomb_friction_closed_form(mu, OCm=OC):
    """Sliding (mu |dv_n| < |v_t|): the tangential speed drops by mu |dv_n|;
    sticking: it stops."""
    case, s, qn, q1, v, dt = _flat_drop(v=(1.5, 0.0, -2.0))
    r = OCm.collide(s, case.ref, case.fixed, dt, qn, q1, v, [("plane", np.zeros(3), np.array([0.0, 0.0, 1.0]))],
                    mu=mu)
    vo = r["v"].reshape(-1, 12)
    vx = max(1.5 - mu * 2.0, 0.0)
    np.testing.assert_allclose(vo[:, 0], vx, atol=2e-9)
    np.testing.assert_allclose(vo[:, 1:3], 0.0, atol=2e-9)


def _deformed_drop(seed=3, n=4, clamp=()):
    """A deformed 4x4 sheet moving down onto a sphere below its middle."""
    case = W.sheet_case(n, edges=clamp, sigma=0.0)
    s = O.shell_from_case(case)
    rng = np.random.default_rng(seed)
    qn = W.random_state(case, seed, 2e-3, 2e-2)
    qn[:, 2] += 0.3
    v = np.zeros_like(qn)
    v[:, 0:3] = (0.1, -0.05, -1.0)
    v[:, 0:3] += rng.normal(0.0, 0.05, size=(case.nodes, 3))
    v[:, 3:] += rng.normal(0.0, 0.05, size=(case.nodes, 9))
    if clamp:
        v[case.fixed.astype(bool)] = 0.0
    dt = 0.2
    sphere = ("sphere", np.array([0.52, 0.47, -0.5]), 0.75)
    return case, s, qn, qn + dt * v, v, dt, sphere


def test_sphere_impulses_conserve_angular_momentum_about_the_centre(OCm=OC):
    case, s, qn, q1, v, dt, sphere = _deformed_drop()
    r = OCm.collide(s, case.ref, case.fixed, dt, qn, q1, v, [sphere])
    assert np.isfinite(r["t_star"]) and 0 < len(r["approach"]) < 40
    qr = r["q_rollback"]
    c = sphere[1]
    P0, L0 = OC.momentum(s, case.ref, qr, v)
    P1, L1 = OC.momentum(s, case.ref, qr, r["v"])
    dLc = (L1 - np.cross(c, P1)) - (L0 - np.cross(c, P0))
    assert np.linalg.norm(P1 - P0) > 1e-3 * np.linalg.norm(P0)          # impulses were applied
    assert np.linalg.norm(dLc) <= 1e-12 * max(np.linalg.norm(L0), 1.0), dLc


def test_plane_impulses_keep_horizontal_momentum(OCm=OC):
    case, s, qn, q1, v, dt, _ = _deformed_drop(seed=4)
    plane = ("plane", np.array([0.0, 0.0, 0.27]), np.array([0.0, 0.0, 1.0]))
    r = OCm.collide(s, case.ref, case.fixed, dt, qn, q1, v, [plane])
    assert np.isfinite(r["t_star"]) and len(r["approach"]) > 0
    qr = r["q_rollback"]
    P0, L0 = OC.momentum(s, case.ref, qr, v)
    P1, L1 = OC.momentum(s, case.ref, qr, r["v"])
    assert P1[2] - P0[2] > 1e-3 * abs(P0[2])
    np.testing.assert_allclose(P1[0:2], P0[0:2], rtol=0, atol=1e-13 * np.linalg.norm(P0))
    assert abs(L1[2] - L0[2]) <= 1e-13 * np.linalg.norm(L0)


def _distance(x, col):
    if col[0] == "plane":
        return col[2] @ (x - col[1])
    return np.linalg.norm(x - col[1]) - col[2]


@pytest.mark.parametrize("clamp", [(), ("x0",)])
def test_contacts_stop_approaching_and_are_pushed_out(clamp, OCm=OC):
    case, s, qn, q1, v, dt, sphere = _deformed_drop(seed=5, clamp=clamp)
    r = OCm.collide(s, case.ref, case.fixed, dt, qn, q1, v, [sphere])
    ops = OC.sample_operators(s, 3)
    assert len(r["approach"]) > 0
    for i, _, n, _ in r["approach"]:
        vn = n @ OC.point_of(ops[i], r["v"].reshape(-1))
        assert abs(vn) <= 1e-10, vn
    # pushed out: the position constraint n . (x - p) = push at the contact's
    # normal and collider point (the sphere's tangent plane there)
    for i, _, n, p in r["contacts"]:
        d = n @ (OC.point_of(ops[i], r["q"].reshape(-1)) - p)
        assert abs(d - 1e-4) <= 1e-12, d
        assert _distance(OC.point_of(ops[i], r["q"].reshape(-1)), sphere) > 0.0
    # rollback: the earliest sample touches, none penetrates
    dists = np.array([_distance(OC.point_of(op, r["q_rollback"]), sphere) for op in ops])
    assert abs(dists.min()) <= 1e-12 and dists.min() >= -1e-12
    if clamp:
        fx = case.fixed.reshape(-1).astype(bool)
        np.testing.assert_array_equal(r["v"].reshape(-1)[fx], v.reshape(-1)[fx])
        np.testing.assert_array_equal(r["q"].reshape(-1)[fx], qn.reshape(-1)[fx])


def test_no_contact_passes_the_step_through(OCm=OC):
    case, s, qn, q1, v, dt = _flat_drop(h0=0.5)
    r = OCm.collide(s, case.ref, case.fixed, dt, qn, q1, v, [("plane", np.zeros(3), np.array([0.0, 0.0, 1.0]))])
    assert r["t_star"] == np.inf and not r["contacts"]
    np.testing.assert_array_equal(r["q"], q1.reshape(-1))
    np.testing.assert_array_equal(r["v"], v.reshape(-1))


# ------------------------------------------------------- planted mistakes
MUTANTS = [
    ("push-out toward the collider", "r = np.array([push - n @ (point_of(ops[i], qs) - p) for i, _, n, p in contacts])",
     "r = np.array([-push - n @ (point_of(ops[i], qs) - p) for i, _, n, p in contacts])"),
    ("impulses weighted by the identity instead of the mass matrix", "Minv_Jt = np.linalg.solve(M, Jm.T)",
     "Minv_Jt = Jm.T.copy()"),
    ("rollback fraction from the end of the step", "qs = qn + (t_star / dt) * (q1 - qn)",
     "qs = qn + (1.0 - t_star / dt) * (q1 - qn)"),
    ("sphere normal pointing inward", "n = (x - c) / np.linalg.norm(x - c)", "n = (c - x) / np.linalg.norm(x - c)"),
    ("Coulomb cone without the normal impulse", "elif nt > mu * ln:\n                    lam[c, 1:] = lt * (mu * ln / nt)",
     "elif nt > mu:\n                    lam[c, 1:] = lt * (mu / nt)"),
    ("sphere contact time from the larger root", "t = (-b - np.sqrt(disc)) / (2.0 * a)",
     "t = (-b + np.sqrt(disc)) / (2.0 * a)"),
]


def _pins():
    return [test_flat_drop_on_a_plane_closed_form, lambda m: test_flat_slide_coulomb_friction_closed_form(0.1, m),
            lambda m: test_flat_slide_coulomb_friction_closed_form(10.0, m),
            test_sphere_impulses_conserve_angular_momentum_about_the_centre, test_plane_impulses_keep_horizontal_momentum,
            lambda m: test_contacts_stop_approaching_and_are_pushed_out((), m),
            lambda m: test_contacts_stop_approaching_and_are_pushed_out(("x0",), m), test_no_contact_passes_the_step_through]


def _mutant_module(old, new):
    src = open(os.path.join(os.path.dirname(HERE), "oracle", "collision.py")).read()
    assert src.count(old) == 1, old
    src = src.replace(old, new).replace("from . import oracle as O", "from oracle import oracle as O")
    d = tempfile.mkdtemp(prefix="orc_coll_")
    path = os.path.join(d, "collision_mutant.py")
    open(path, "w").write(src)
    spec = importlib.util.spec_from_file_location("collision_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_unchanged_copy_passes_every_pin():
    mod = _mutant_module("import numpy as np", "import numpy as np")
    for pin in _pins():
        pin(mod)


@pytest.mark.parametrize("i", range(len(MUTANTS)), ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(i):
    mod = _mutant_module(MUTANTS[i][1], MUTANTS[i][2])
    failed = 0
    for pin in _pins():
        try:
            pin(mod)
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            failed += 1
    assert failed > 0, MUTANTS[i][0]
