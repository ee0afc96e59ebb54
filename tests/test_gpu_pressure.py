"""Pressure loads (Sec. 4.3, f = p n) on the GPU through the C ABI against
the oracle: the nodal load at a deformed state (two shells with different
pressures in one context), implicit steps with the pressure evaluated at
the step's start, the open-cylinder inflation closed form, and removing the
pressure again (the captured launch sequences must follow)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2312_14839_amd import workloads as W

from gpu_util import rel_disp_error
import test_oracle_pressure as TP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def S():
    from paper_2312_14839_amd import shell
    return shell


def test_pressure_load_matches_oracle():
    a, b = W.sheet_case(5, edges=()), W.case_cylinder(9, 4)
    qa, qb = W.random_state(a, 3, 1e-2, 5e-2), W.random_state(b, 4, 1e-2, 5e-2)
    ctx = S().context_for([a, b])
    ctx.set_pressure([2.5, -0.7])
    f = torch.zeros((a.nodes + b.nodes) * 12, dtype=torch.float64, device="cuda")
    ctx.pressure_load(dev(np.concatenate([qa, qb])), f)
    fh = host(f).reshape(-1, 12)
    ctx.close()
    fa = O.pressure_load(O.shell_from_case(a), qa, 2.5)
    fb = O.pressure_load(O.shell_from_case(b), qb, -0.7)
    np.testing.assert_allclose(fh[:a.nodes], fa, rtol=0, atol=1e-13 * np.abs(fa).max())
    np.testing.assert_allclose(fh[a.nodes:], fb, rtol=0, atol=1e-13 * np.abs(fb).max())


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-5)])
def test_pressurised_steps_match_oracle(precision, tol):
    """8x8 sheet clamped along one edge, gravity and an upward pressure,
    three steps in one context, each against the oracle's step from the
    GPU's previous state."""
    sh = S()
    case = W.case_small_sheet()
    s = O.shell_from_case(case)
    ctx = sh.context_for([case], precision=sh.SHELL_MIXED if precision == "mixed" else sh.SHELL_FP64)
    ctx.set_pressure([4.0])
    q, v = case.q0.copy(), case.v0.copy()
    for k in range(3):
        q1d, v1d = torch.empty(q.size, dtype=torch.float64, device="cuda"), torch.empty(q.size, dtype=torch.float64,
                                                                                       device="cuda")
        rc, st = ctx.newton_step(case.dt, dev(q), dev(v), None, q1d, v1d)
        assert rc == 0, st
        rc_o, q1o, _, _ = O.newton_step(s, case.ref, case.fixed, case.dt, q, v, pressure=4.0)
        assert rc_o == 0
        q1, v1 = host(q1d).reshape(-1, 12), host(v1d).reshape(-1, 12)
        assert rel_disp_error(q1, q1o, q) <= tol, (k, rel_disp_error(q1, q1o, q))
        q, v = q1, v1
    # pressure removed: the next step is the unloaded oracle step
    ctx.set_pressure(None)
    q1d, v1d = torch.empty(q.size, dtype=torch.float64, device="cuda"), torch.empty(q.size, dtype=torch.float64,
                                                                                   device="cuda")
    rc, st = ctx.newton_step(case.dt, dev(q), dev(v), None, q1d, v1d)
    assert rc == 0
    rc_o, q1o, _, _ = O.newton_step(s, case.ref, case.fixed, case.dt, q, v)
    assert rel_disp_error(host(q1d).reshape(-1, 12), q1o, q) <= tol
    ctx.close()


def test_inflated_open_cylinder_closed_form():
    sh = S()
    case = TP._cylinder()
    ctx = sh.context_for([case], newton_rtol=1e-12, pcg_rtol=1e-12)
    ctx.set_pressure([1.0])

    def newton(q, v):
        qd = dev(q)
        q1, v1 = torch.empty_like(qd), torch.empty_like(qd)
        rc, st = ctx.newton_step(case.dt, qd, dev(v), None, q1, v1)
        assert rc == 0, st
        return host(q1).reshape(-1, 12), host(v1).reshape(-1, 12)

    q = TP.inflate(newton, case, 1.0)
    ctx.close()
    k, e = 0.2 / (1e5 * 1e-3), 0.0
    for _ in range(50):
        e = k * math.sqrt(1.0 - 2.0 * 0.3 * e)
    u_exact = (math.sqrt(1.0 + 2.0 * e) - 1.0) * 0.2
    mid = q[3 * case.n1:6 * case.n1]
    u = np.hypot(mid[:, 0], mid[:, 1]) - 0.2
    assert np.abs(u - u_exact).max() <= 1e-4 * u_exact, (u.min(), u.max(), u_exact)
