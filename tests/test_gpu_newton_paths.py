"""GPU Newton steps through the branches the converging parity cases never
take, each against the oracle (through the C ABI): the diagonal regulariser,
line-search backtracking with quadratic and cubic steps, the CG iteration
cap (SHELL_E_NOT_CONVERGED with the last iterate written) and a system the
regulariser cannot make definite (SHELL_E_INDEFINITE).  The states are the
ones the oracle's own pins of these branches use (tests/test_oracle_newton.py)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2312_14839_amd import workloads as W

from gpu_util import newton_residual, rel_disp_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def S():
    from paper_2312_14839_amd import shell
    return shell


def gpu_step(case, precision="fp64", **opts):
    sh = S()
    ctx = sh.context_for([case], precision=sh.SHELL_MIXED if precision == "mixed" else sh.SHELL_FP64, **opts)
    qn, vn = dev(case.q0), dev(case.v0)
    q1, v1 = torch.full_like(qn, np.nan), torch.full_like(qn, np.nan)
    rc, st = ctx.newton_step(case.dt, qn, vn, None, q1, v1, allow_fail=True)
    ctx.close()
    return rc, host(q1).reshape(-1, 12), host(v1).reshape(-1, 12), st[0]


def stationary(case, q1, st, factor=10.0):
    res = np.linalg.norm(newton_residual(case, q1, case.q0, case.v0, case.dt))
    return res <= factor * max(1e-10 * st["grad_norm0"], st["grad_floor"]), res


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-5)])
def test_regularised_step_matches_oracle(precision, tol):
    """Pre-compressed sheet, dt = 1 s: the first Newton systems are
    indefinite.  The oracle regularises on a failed LDL^T pivot, the GPU on
    a failed block Cholesky or p^T A p <= 0 in the CG; both must regularise,
    end at a stationary point, and (the regularised systems being the same
    here) at the same point."""
    case = W.case_precompressed()
    s = O.shell_from_case(case)
    rc_o, q_o, _, st_o = O.newton_step(s, case.ref, case.fixed, case.dt, case.q0, case.v0)
    assert rc_o == 0 and st_o["reg_delta"] > 0
    rc, q1, v1, st = gpu_step(case, precision)
    print(f"regularised {precision}: gpu delta {st['reg_delta']:g} its {st['newton_iters']} ls {st['ls_backtracks']}"
          f" | oracle delta {st_o['reg_delta']:g} its {st_o['newton_iters']} ls {st_o['ls_backtracks']}", flush=True)
    assert rc == S().SHELL_OK, st
    assert st["reg_delta"] > 0.0
    ok, res = stationary(case, q1, st, 1e3 if precision == "mixed" else 10.0)
    assert ok, res
    err = rel_disp_error(q1, q_o, case.q0)
    assert err <= tol, err


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-5)])
def test_backtracking_step_matches_oracle(precision, tol):
    """Drooping cantilever (4x4 sheet, 3 cm thick, dt = 1 s): the line search
    backtracks, with cubic steps, in the first iterations.  FP64: the same
    Newton and backtrack counts as the oracle and the same point; mixed: the
    same point to the mixed form's bound."""
    case = W.sheet_case(4, seed=1, dt=1.0, edges=("x0",), thickness=0.03)
    s = O.shell_from_case(case)
    rc_o, q_o, _, st_o = O.newton_step(s, case.ref, case.fixed, case.dt, case.q0, case.v0)
    assert rc_o == 0 and st_o["ls_backtracks"] >= 3
    rc, q1, v1, st = gpu_step(case, precision)
    print(f"backtracking {precision}: gpu its {st['newton_iters']} ls {st['ls_backtracks']} | oracle its "
          f"{st_o['newton_iters']} ls {st_o['ls_backtracks']}", flush=True)
    assert rc == S().SHELL_OK, st
    assert st["ls_backtracks"] > 0 and st["reg_delta"] == 0.0
    if precision == "fp64":
        assert st["ls_backtracks"] == st_o["ls_backtracks"]
        assert st["newton_iters"] == st_o["newton_iters"]
    err = rel_disp_error(q1, q_o, case.q0)
    assert err <= tol, err


def test_cg_cap_reports_not_converged_with_the_last_iterate():
    """One CG iteration per Newton system, three Newton iterations:
    SHELL_E_NOT_CONVERGED, and the outputs hold the third iterate, the
    oracle's (its CG also stops after one iteration)."""
    case = W.case_small_sheet()
    s = O.shell_from_case(case)
    rc_o, q_o, _, st_o = O.newton_step(s, case.ref, case.fixed, case.dt, case.q0, case.v0, solver="pcg",
                                       pcg_maxit=1, newton_maxit=3)
    assert rc_o == 1
    sh = S()
    rc, q1, v1, st = gpu_step(case, pcg_maxit=1, newton_maxit=3)
    assert rc == sh.SHELL_E_NOT_CONVERGED and st["status"] == sh.SHELL_E_NOT_CONVERGED
    assert st["newton_iters"] == 3 and st["pcg_iters_total"] == 3
    assert np.all(np.isfinite(q1)) and np.all(np.isfinite(v1))
    err = rel_disp_error(q1, q_o, case.q0)
    assert err <= 1e-10, err
    np.testing.assert_allclose(v1, (q1 - case.q0) / case.dt, rtol=0, atol=1e-9)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_indefinite_beyond_the_regulariser_cap(precision):
    """Thin pre-compressed sheet, dt = 1 s: negative diagonal entries, which
    the regulariser cannot repair.  SHELL_E_INDEFINITE at delta = 1e2 (the
    oracle: status 3), no step taken: the outputs hold the predicted state."""
    case = W.case_precompressed(strain=0.02, thickness=0.01)
    s = O.shell_from_case(case)
    rc_o, q_o, _, st_o = O.newton_step(s, case.ref, case.fixed, case.dt, case.q0, case.v0)
    assert rc_o == 3 and st_o["reg_delta"] == 1e2
    sh = S()
    rc, q1, v1, st = gpu_step(case, precision)
    assert rc == sh.SHELL_E_INDEFINITE and st["status"] == sh.SHELL_E_INDEFINITE
    assert st["reg_delta"] == pytest.approx(1e2, rel=1e-12) and st["newton_iters"] == 0
    np.testing.assert_array_equal(q1, q_o)
    np.testing.assert_array_equal(v1, np.zeros_like(v1))
