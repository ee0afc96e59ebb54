"""The device-driven Newton iteration (one launch sequence per iteration,
decisions on the device) against the host-driven one, through the C ABI.

Both take the same kernels and the same decisions on the same values (the
control kernels repeat the host's expressions with contraction off), so
every output and statistic must agree exactly: on plain steps, on steps
whose shells the device hands back to the host (the regulariser after a
failed block factorisation or p^T A p <= 0, a line search longer than the
device's two trials, the CG iteration cap), for batches of shells whose
iterations end at different times, over many steps with prescribed DOFs,
and with the captured graph replayed many times.  Parity of these paths with
the oracle is covered by the parity and Newton-branch tests, which run the
device-driven iteration (the default)."""
import numpy as np
import pytest

from paper_2312_14839_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STAT_KEYS = ("status", "newton_iters", "pcg_iters_total", "ls_backtracks", "refine_sweeps", "grad_norm0",
             "grad_norm", "grad_floor", "reg_delta")


def S():
    from paper_2312_14839_amd import shell
    return shell


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def run(cases, precision, device_newton, steps=1, graphs=True, **opts):
    """`steps` steps of every case from its start; returns the final q, v and
    the per-step statistics."""
    sh = S()
    prec = sh.SHELL_MIXED if precision == "mixed" else sh.SHELL_FP64
    ctx = sh.context_for(cases, precision=prec, device_newton=device_newton, graphs=graphs, **opts)
    q = dev(np.concatenate([c.q0 for c in cases]).reshape(-1))
    v = dev(np.concatenate([c.v0 for c in cases]).reshape(-1))
    q1, v1 = torch.full_like(q, np.nan), torch.full_like(q, np.nan)
    rcs, stats = [], []
    for k in range(steps):
        presc = None
        if len(cases) == 1 and cases[0].presc is not None:
            presc = dev(cases[0].presc((k + 1) * cases[0].dt).reshape(-1))
        rc, st = ctx.newton_step(cases[0].dt, q, v, presc, q1, v1, allow_fail=True)
        rcs.append(rc)
        stats.append(st)
        q, q1 = q1, q
        v, v1 = v1, v
    torch.cuda.synchronize()
    ctx.close()
    return rcs, q.cpu().numpy(), v.cpu().numpy(), stats


def assert_same(a, b):
    rc_a, q_a, v_a, st_a = a
    rc_b, q_b, v_b, st_b = b
    assert rc_a == rc_b
    np.testing.assert_array_equal(q_a, q_b)
    np.testing.assert_array_equal(v_a, v_b)
    for k, (sa, sb) in enumerate(zip(st_a, st_b)):
        for s, (x, y) in enumerate(zip(sa, sb)):
            for key in STAT_KEYS:
                assert x[key] == y[key], (k, s, key, x[key], y[key])


CASES = {
    "sheet8": lambda: [W.case_small_sheet()],
    "regularised": lambda: [W.case_precompressed()],
    "backtracking": lambda: [W.sheet_case(4, seed=1, dt=1.0, edges=("x0",), thickness=0.03)],
    "indefinite": lambda: [W.case_precompressed(strain=0.02, thickness=0.01)],
    "batch5": lambda: W.case_batch(5, nmin=4, nmax=12),
    "batch_mixed_branches": lambda: [W.case_small_sheet(), W.case_precompressed(),
                                     W.sheet_case(4, seed=1, dt=1.0, edges=("x0",), thickness=0.03)],
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_device_iteration_equals_host_iteration(name, precision):
    cases = CASES[name]()
    if name == "batch_mixed_branches":
        for c in cases:   # one time step for the whole context
            c.dt = 1.0
    a = run(cases, precision, True)
    b = run(cases, precision, False)
    print(f"{name} {precision}: rc {a[0]}, newton {[s['newton_iters'] for s in a[3][0]]}, "
          f"ls {[s['ls_backtracks'] for s in a[3][0]]}, delta {[s['reg_delta'] for s in a[3][0]]}", flush=True)
    assert_same(a, b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_device_iteration_over_twist_steps(precision):
    """Twenty steps of the 12x12 twisting sheet (prescribed DOFs move every
    step): the captured iteration is replayed every Newton iteration of every
    step, with the host's own work between the replays."""
    cases = [W.case_twist(12)]
    a = run(cases, precision, True, steps=20)
    b = run(cases, precision, False, steps=20)
    assert all(rc == S().SHELL_OK for rc in a[0])
    assert_same(a, b)


def test_handed_over_stages_are_exercised():
    """The equality cases above do reach the host's continuation: the
    regulariser (a block factorisation that fails, or p^T A p <= 0), a line
    search past the device's two trials, and (mixed form at a tolerance
    below what two sweeps reach) refinement sweeps past the device's two."""
    st = run(CASES["regularised"](), "fp64", True)[3][0][0]
    assert st["reg_delta"] > 0
    st = run(CASES["backtracking"](), "fp64", True)[3][0][0]
    assert st["ls_backtracks"] >= 3
    # mixed form below what two sweeps reach: every solve of the 12x12 twist
    # at 1e-13 takes three
    cases = [W.case_twist(12)]
    a = run(cases, "mixed", True, steps=3, pcg_rtol=1e-13)
    sweeps = sum(s[0]["refine_sweeps"] for s in a[3])
    newton = sum(s[0]["newton_iters"] for s in a[3])
    print(f"refinement at 1e-13: {sweeps} sweeps over {newton} Newton iterations", flush=True)
    assert sweeps > 2 * newton
    assert_same(a, run(cases, "mixed", False, steps=3, pcg_rtol=1e-13))


def test_device_iteration_without_graphs_and_at_the_cg_cap():
    """Direct launches instead of the graph give the same result, and the CG
    iteration cap (one CG iteration, three Newton iterations) is reported as
    by the host-driven iteration."""
    cases = [W.case_small_sheet()]
    assert_same(run(cases, "fp64", True, graphs=False), run(cases, "fp64", False))
    a = run(cases, "fp64", True, pcg_maxit=1, newton_maxit=3)
    b = run(cases, "fp64", False, pcg_maxit=1, newton_maxit=3)
    assert a[0][0] == S().SHELL_E_NOT_CONVERGED
    assert_same(a, b)
