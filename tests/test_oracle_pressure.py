"""Pins of the oracle's pressure load (Sec. 4.3, "External Forces", f = p n),
CPU only.  Reading: the pressure acts per unit current area along
a_1 x a_2, so F_I = p integral Phi^I (a_1 x a_2) dxi1 dxi2; in an implicit
step it is evaluated at the step's start (a dead load within the step).

* Flat sheet: the total force is p A e_z and its moment about the centre 0.
* Virtual work: p times the enclosed-volume functional
  V(q) = (1/3) integral x . (a_1 x a_2) dxi1 dxi2 has, for every DOF of a
  node off the boundary (whose shape functions vanish with their slopes on
  the boundary), the derivative F_I / p.  On a bicubic height field both
  integrands are polynomials the 4x4 Gauss rule integrates exactly, so the
  complex-step derivative of the (independently written) quadrature of V
  equals the oracle's force to rounding.
* Pressurised open cylinder held only against rigid motion (the bottom
  ring's axial positions and two tangential positions): a uniform
  inflation r = lambda R with free axial contraction (zero axial stress:
  Green strains E_zz = -nu E, E = (lambda^2 - 1)/2 the hoop strain, and
  second Piola stress Y E).  Virtual work per unit reference length, hoop
  membrane 2 pi R h Y E lambda dlambda against the pressure on the current
  lateral area 2 pi lambda R s_z (s_z = sqrt(1 + 2 E_zz) the axial stretch)
  moving R dlambda: E = (p R / (Y h)) sqrt(1 - 2 nu E), solved by fixed
  point (bending of order h^2/R^2 smaller).  A pressure per unit reference
  area would give E = p R / (Y h lambda) instead, 1.4e-3 away here."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2312_14839_amd import workloads as W


def test_flat_sheet_total_force_and_moment():
    case = W.sheet_case(4, edges=(), sigma=0.0)
    s = O.shell_from_case(case)
    f = O.pressure_load(s, case.ref, 2.5).reshape(-1, 4, 3)
    F = f[:, 0, :].sum(axis=0)
    np.testing.assert_allclose(F, [0.0, 0.0, 2.5], rtol=0, atol=1e-14)
    # moment about the centre: sum over nodes of (x_I - c) x F_I on positions
    # plus the derivative DOFs' force pairs (x_xi x F_xi terms)
    x = case.ref.reshape(-1, 4, 3)
    c = np.array([0.5, 0.5, 0.0])
    Mo = np.cross(x[:, 0, :] - c, f[:, 0, :]).sum(axis=0) + sum(np.cross(x[:, k, :], f[:, k, :]).sum(axis=0)
                                                                for k in (1, 2, 3))
    np.testing.assert_allclose(Mo, 0.0, atol=1e-14)


def _height_field(n, seed):
    rng = np.random.default_rng(seed)
    cz = rng.normal(0.0, 0.05, size=(4, 4))

    def z(x, y):
        v = sum(cz[i, j] * x ** i * y ** j for i in range(4) for j in range(4))
        zx = sum(i * cz[i, j] * x ** (i - 1) * y ** j for i in range(1, 4) for j in range(4))
        zy = sum(j * cz[i, j] * x ** i * y ** (j - 1) for i in range(4) for j in range(1, 4))
        zxy = sum(i * j * cz[i, j] * x ** (i - 1) * y ** (j - 1) for i in range(1, 4) for j in range(1, 4))
        return v, zx, zy, zxy

    ref = W.height_field_ref(n, n, z)
    return W._scene_case("hf", n, n, 0, 1.0 / n, 1.0 / n, ref)


def _volume(s, q):
    """(1/3) integral x . (a_1 x a_2) dxi1 dxi2 by the 4x4 Gauss rule (complex q allowed)."""
    th, wt = O.gauss4()
    q = q.reshape(-1, 12)
    V = 0.0
    for pj in range(s.n2):
        for pi in range(s.n1):
            nodes = O.patch_nodes(s, pi, pj)
            loc = np.stack([q[nd].reshape(4, 3) for nd in nodes]).reshape(16, 3)
            for g2 in range(4):
                for g1 in range(4):
                    phi = O.shape_functions(th[g1], th[g2], s.dxi1, s.dxi2)
                    x, a1, a2 = phi[0] @ loc, phi[1] @ loc, phi[2] @ loc
                    V = V + wt[g1] * wt[g2] * s.dxi1 * s.dxi2 * (x @ np.cross(a1, a2)) / 3.0
    return V


@pytest.mark.parametrize("seed", [1, 2])
def test_force_is_the_derivative_of_the_enclosed_volume(seed):
    case = _height_field(3, seed)
    s = O.shell_from_case(case)
    p = 1.7
    f = O.pressure_load(s, case.ref, p).reshape(-1)
    cols = case.n1 + 1
    interior = [j * cols + i for j in range(1, case.n2) for i in range(1, case.n1)]
    h = 1e-30
    checked = 0
    for nd in interior:
        for w in range(12):
            qc = case.ref.reshape(-1).astype(complex)
            qc[12 * nd + w] += 1j * h
            dV = _volume(s, qc).imag / h
            assert abs(p * dV - f[12 * nd + w]) <= 1e-13 * max(1.0, abs(f).max()), (nd, w)
            checked += 1
    assert checked == 12 * len(interior) and np.abs(f).max() > 0.1


def _cylinder(n1=16, n2=8, R=0.2, L=0.4):
    """Open cylinder, xi1 around (counter-clockwise), xi2 along; held
    against rigid motion only: axial positions of the bottom ring, x of the
    node at 90 degrees and y of the node at 0 degrees (both compatible with
    a radial expansion)."""
    ref = W.cylinder_ref(n1, n2, R, L)
    fixed = np.zeros_like(ref, dtype=np.uint8)
    fixed[:n1, 2] = 1
    fixed[n1 // 4, 0] = 1
    fixed[0, 1] = 1
    return W.Case("pcyl", n1, n2, 1, 2 * math.pi * R / n1, L / n2, 1e5, 0.3, 1e-3, 200.0, (0.0, 0.0, 0.0), ref, fixed,
                  ref.copy(), np.zeros_like(ref), 1e3)


def inflate(newton, case, p, steps=6):
    """Quasi-static inflation: steps of dt = 1e3 s (inertia negligible) from
    rest, each with the pressure evaluated at its start, until the state
    stops changing; returns the final state."""
    q, v = case.q0.copy(), case.v0.copy()
    for _ in range(steps):
        q1, v1 = newton(q, v)
        q, v = q1, np.zeros_like(v1)
    return q


def test_pressurised_cylinder_hoop_closed_form():
    case = _cylinder()
    s = O.shell_from_case(case)
    p, R = 1.0, 0.2

    def newton(q, v):
        rc, q1, v1, _ = O.newton_step(s, case.ref, case.fixed, case.dt, q, v, pressure=p)
        assert rc == 0
        return q1, v1

    q = inflate(newton, case, p)
    k, e = p * R / (1e5 * 1e-3), 0.0
    for _ in range(50):
        e = k * math.sqrt(1.0 - 2.0 * 0.3 * e)
    lam = math.sqrt(1.0 + 2.0 * e)
    qq = q.reshape(-1, 12)
    # the three mid-length rings (the free ends flare in a short bending layer)
    mid = qq[3 * case.n1:6 * case.n1]
    u, u_exact = np.hypot(mid[:, 0], mid[:, 1]) - R, (lam - 1.0) * R
    assert np.abs(u - u_exact).max() <= 1e-4 * u_exact, (u.min(), u.max(), u_exact)
    # axial contraction: plane stress, E_zz = -nu E_theta
    ezz = ((qq[case.n2 * case.n1, 2] / 0.4) ** 2 - 1.0) / 2.0
    assert abs(ezz + 0.3 * (lam ** 2 - 1.0) / 2.0) <= 1e-3 * abs(ezz), ezz
