"""Pins of the oracle's mechanics (Sec. 3, 4.3 and Appendix B) against what
the mathematics fixes independently of the oracle's own formulas:
closed-form energies, rigid-motion invariance, complex-step and finite-
difference derivatives, symmetry, and the textbook cubic-Hermite mass matrix.
CPU only."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2312_14839_amd import workloads as W


def _rot(rng):
    a = rng.normal(size=(3, 3))
    qm, r = np.linalg.qr(a)
    qm *= np.sign(np.diag(r))
    if np.linalg.det(qm) < 0:
        qm[:, 0] *= -1
    return qm


def _rigid(q, R, t):
    out = q.reshape(-1, 4, 3) @ R.T
    out[:, 0, :] += t
    return out.reshape(q.shape)


def _patch_cases():
    """(shell, q, qb) per-patch triples: flat sheet with unequal cells, and a cylinder patch."""
    rng = np.random.default_rng(7)
    out = []
    s = O.make_shell(3, 2, 0.31, 0.47, 1e5, 0.3, 2e-3, 200.0)
    ref = W.flat_sheet_ref(1, 1, 0.31, 0.47)
    qb = np.concatenate([ref[n] for n in (0, 1, 2, 3)])
    q = qb + np.concatenate([np.r_[rng.normal(0, 2e-2, 3), rng.normal(0, 1e-1, 9)] for _ in range(4)])
    out.append((s, q, qb))
    cyl = W.case_cylinder(8, 4)
    sc = O.shell_from_case(cyl)
    qb = O.gather(sc, cyl.ref, 7, 2)       # patch across the periodic seam
    q = qb + rng.normal(0, 1e-2, 48)
    out.append((sc, q, qb))
    return out


# ------------------------------------------------------------ energies
def test_tensor_and_voigt_energy_agree():
    for s, q, qb in _patch_cases():
        et = O.patch_energy(s, q, qb, "tensor")
        ev = O.patch_energy(s, q, qb, "voigt")
        assert et > 0
        assert abs(et - ev) <= 1e-13 * abs(et)


def test_zero_energy_and_force_at_rest_and_under_rigid_motion():
    rng = np.random.default_rng(3)
    for case in (W.sheet_case(3), W.case_cylinder(8, 3)):
        s = O.shell_from_case(case)
        qb = case.ref
        assert abs(O.energy(s, qb, qb)) < 1e-25
        assert np.abs(O.gradient(s, qb, qb)).max() < 1e-14
        R, t = _rot(rng), rng.normal(size=3)
        qr = _rigid(qb, R, t)
        assert abs(O.energy(s, qr, qb)) < 1e-20
        assert np.abs(O.gradient(s, qr, qb)).max() < 1e-12
        # at a deformed state the energy is invariant and the gradient rotates
        q = W.random_state(case, 11)
        qr = _rigid(q, R, t)
        e, er = O.energy(s, q, qb), O.energy(s, qr, qb)
        assert abs(e - er) <= 1e-11 * e
        g, gr = O.gradient(s, q, qb), O.gradient(s, qr, qb)
        np.testing.assert_allclose(gr, _rigid(g, R, np.zeros(3)), atol=1e-10 * np.abs(g).max())


def test_uniform_stretch_matches_plane_stress_stvk():
    """Affine reference X = G xi and affine current x = F xi: the discrete energy
    equals area * h * ((lam/2) tr(E)^2 + mu tr(E^2)) with the physical Green
    strain E of the in-plane deformation gradient (integrand is constant, so
    the quadrature is exact)."""
    rng = np.random.default_rng(5)
    Y, nu, h = 3.3e5, 0.35, 1.7e-3
    lam, mu = Y * nu / (1 - nu ** 2), Y / (2 * (1 + nu))
    n1, n2, d1, d2 = 3, 2, 0.4, 0.7
    G = rng.normal(size=(3, 2))
    F = G + 0.05 * rng.normal(size=(3, 2))
    s = O.make_shell(n1, n2, d1, d2, Y, nu, h, 1.0)
    qb = np.zeros(((n1 + 1) * (n2 + 1), 12))
    q = np.zeros_like(qb)
    for j in range(n2 + 1):
        for i in range(n1 + 1):
            xi = np.array([i * d1, j * d2])
            qb[j * (n1 + 1) + i] = np.r_[G @ xi, G[:, 0], G[:, 1], 0, 0, 0]
            q[j * (n1 + 1) + i] = np.r_[F @ xi, F[:, 0], F[:, 1], 0, 0, 0]
    Q, Rm = np.linalg.qr(G)                      # in-plane orthonormal frame, X = Rm xi
    Fx = F @ np.linalg.inv(Rm)
    E = 0.5 * (Fx.T @ Fx - np.eye(2))
    area = abs(np.linalg.det(Rm)) * n1 * d1 * n2 * d2
    exact = area * h * (0.5 * lam * np.trace(E) ** 2 + mu * np.trace(E @ E))
    got = O.energy(s, q, qb)
    assert abs(got - exact) <= 1e-12 * exact


def test_cylindrical_bending_converges_to_kirchhoff():
    """A flat sheet rolled isometrically onto a cylinder of radius R stores
    D/(2R^2) per unit area, D = Y h^3 / (12 (1 - nu^2)).  The Hermite sampling
    of the rolled shape converges to it at high order."""
    Y, nu, h, R = 1e5, 0.3, 1e-2, 0.5
    D = Y * h ** 3 / (12 * (1 - nu ** 2))
    exact = D / (2 * R * R) * 1.0
    errs = []
    for n in (2, 4, 8):
        s = O.make_shell(n, n, 1.0 / n, 1.0 / n, Y, nu, h, 1.0)
        qb = W.flat_sheet_ref(n, n)
        q = qb.copy()
        for idx in range(q.shape[0]):
            x1, x2 = qb[idx, 0], qb[idx, 1]
            a = x1 / R
            q[idx] = np.r_[R * math.sin(a), x2, R - R * math.cos(a), math.cos(a), 0, math.sin(a), 0, 1, 0, 0, 0, 0]
        errs.append(abs(O.energy(s, q, qb) - exact) / exact)
    assert errs[-1] < 1e-4
    assert errs[0] / errs[1] > 8 and errs[1] / errs[2] > 8


# ------------------------------------------------------------ gradient
@pytest.mark.parametrize("k", [0, 1])
def test_gradient_matches_complex_step(k):
    s, q, qb = _patch_cases()[k]
    g = O.patch_gradient(s, q, qb)
    hstep = 1e-30
    gcs = np.array([O.patch_energy_cs(s, q, hstep * np.eye(48)[i], qb)[1] / hstep for i in range(48)])
    assert np.abs(g - gcs).max() <= 1e-12 * np.abs(gcs).max()


def test_gradient_matches_central_differences():
    s, q, qb = _patch_cases()[0]
    g = O.patch_gradient(s, q, qb)
    fd = np.zeros(48)
    for i in range(48):
        e = np.zeros(48)
        e[i] = 1e-6 * max(1.0, abs(q[i]))
        fd[i] = (O.patch_energy(s, q + e, qb) - O.patch_energy(s, q - e, qb)) / (2 * e[i])
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(g).max()


def test_net_force_and_torque_vanish():
    for s, q, qb in _patch_cases():
        g = O.patch_gradient(s, q, qb).reshape(16, 3)
        qq = q.reshape(16, 3)
        scale = np.abs(g).max() * np.abs(qq).max()
        pos = g[[0, 4, 8, 12]]
        assert np.abs(pos.sum(axis=0)).max() <= 1e-13 * np.abs(g).max()
        assert np.abs(np.cross(qq, g).sum(axis=0)).max() <= 1e-12 * scale


# ------------------------------------------------------------ Hessian
@pytest.mark.parametrize("k", [0, 1])
def test_hessian_matches_complex_step_of_gradient(k):
    s, q, qb = _patch_cases()[k]
    H = O.patch_hessian(s, q, qb)
    hstep = 1e-30
    Hcs = np.array([O.patch_gradient_cs(s, q, hstep * np.eye(48)[i], qb)[1] / hstep for i in range(48)]).T
    assert np.abs(H - Hcs).max() <= 1e-11 * np.abs(Hcs).max()
    assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()


def test_hessian_matches_central_differences():
    s, q, qb = _patch_cases()[1]
    H = O.patch_hessian(s, q, qb)
    fd = np.zeros((48, 48))
    for i in range(48):
        e = np.zeros(48)
        e[i] = 1e-6
        fd[:, i] = (O.patch_gradient(s, q + e, qb) - O.patch_gradient(s, q - e, qb)) / 2e-6
    assert np.abs(H - fd).max() <= 1e-6 * np.abs(H).max()


def test_pseudo_hessian_equals_exact_at_rest_and_differs_when_bent():
    for s, q, qb in _patch_cases():
        Hr = O.patch_hessian(s, qb, qb, pseudo=False)
        Hp = O.patch_hessian(s, qb, qb, pseudo=True)
        assert np.abs(Hr - Hp).max() <= 1e-14 * np.abs(Hr).max()
        He = O.patch_hessian(s, q, qb, pseudo=False)
        Hq = O.patch_hessian(s, q, qb, pseudo=True)
        assert np.abs(He - Hq).max() > 1e-8 * np.abs(He).max()


def test_translations_in_hessian_null_space():
    for s, q, qb in _patch_cases():
        H = O.patch_hessian(s, q, qb)
        for c in range(3):
            t = np.zeros(48)
            t[[12 * k + c for k in range(4)]] = 1.0
            assert np.abs(H @ t).max() <= 1e-12 * np.abs(H).max()


# --------------------------------------------------------- mass, gravity
def _hermite_mass_1d(L):
    """Textbook consistent mass of a cubic Hermite beam element of length L,
    DOFs (w0, w0', w1, w1'), per unit mass density."""
    return L / 420.0 * np.array([[156, 22 * L, 54, -13 * L],
                                 [22 * L, 4 * L * L, 13 * L, -3 * L * L],
                                 [54, 13 * L, 156, -22 * L],
                                 [-13 * L, -3 * L * L, -22 * L, 4 * L * L]])


def test_patch_mass_is_kronecker_of_hermite_beam_masses():
    d1, d2, rho, h = 0.3, 0.55, 930.0, 2e-3
    s = O.make_shell(1, 1, d1, d2, 1e5, 0.3, h, rho)
    qb = np.concatenate([np.r_[c & 1 and d1 or 0.0, (c >> 1) * d2, 0, 1, 0, 0, 0, 1, 0, 0, 0, 0] for c in range(4)])
    M = O.patch_mass(s, qb)
    m1, m2 = _hermite_mass_1d(d1), _hermite_mass_1d(d2)
    idx = lambda p, r: 2 * p + r          # 1-D DOF order (w0, w0', w1, w1')
    for c in range(4):
        for k in range(4):
            for d in range(4):
                for l in range(4):
                    exact = rho * h * m1[idx(c & 1, k & 1), idx(d & 1, l & 1)] * m2[idx(c >> 1, k >> 1), idx(d >> 1, l >> 1)]
                    blk = M[12 * c + 3 * k:12 * c + 3 * k + 3, 12 * d + 3 * l:12 * d + 3 * l + 3]
                    np.testing.assert_allclose(blk, exact * np.eye(3), atol=1e-15 * rho * h)


def test_total_mass_and_gravity_load():
    case = W.sheet_case(4)
    s = O.shell_from_case(case)
    rows, cols, vals = O.matrix_blocks(s, case.q0, case.ref, "mass")
    # a uniform unit x-translation has kinetic mass 1^T M 1 = rho h area
    pos_total = sum(v[0, 0] for v in vals)
    assert abs(pos_total - case.density * case.thickness * 1.0) < 1e-13
    f = O.gravity(s, case.ref).reshape(-1, 4, 3)
    np.testing.assert_allclose(f[:, 0, :].sum(axis=0), case.density * case.thickness * np.array(case.gravity),
                               rtol=1e-13, atol=1e-15)
