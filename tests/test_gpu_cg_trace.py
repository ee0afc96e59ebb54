"""The CG's phase trace (shell_cg_trace_enable / shell_cg_trace_get).

Tracing only adds stores of a clock value by each block's first thread, so
the solution and iteration counts must be bit-identical with tracing on and
off, direct and from a replayed graph.  The stamps themselves obey what the
iteration's structure fixes: within one block and iteration they are in
phase order; one iteration ends before the next starts; the iterations
recorded are the first min(64, iterations) of the launch; and, for a shell
held by several blocks, no block leaves an iteration's reduce-barrier before
the last block of the shell has arrived at it (the clock is one constant
device clock, the same on every compute unit)."""
import numpy as np
import pytest

from paper_2312_14839_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def S():
    from paper_2312_14839_amd import shell
    return shell


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


CASES = {
    "sheet4": lambda: W.sheet_case(4, seed=1),
    "cylinder32": lambda: W.case_cylinder(32, 32),
}


def _solve(case, trace, precision):
    sh = S()
    ctx = sh.context_for([case], precision=precision)
    if trace:
        ctx.cg_trace_enable(True)
    ms = 1.0 / case.dt ** 2
    ctx.assemble(dev(case.q0), mass_scale=ms)
    free = ~case.fixed.reshape(-1).astype(bool)
    b = np.random.default_rng(9).normal(size=free.size) * free
    x = torch.zeros(free.size, dtype=torch.float64, device="cuda")
    rc, its, rel = ctx.pcg_solve(dev(b), x, rtol=1e-10)
    tr = ctx.cg_trace_get()
    ctx.close()
    return its, x.cpu().numpy(), tr


def check_trace(tr, iters):
    nb, nit, six = tr.shape
    assert nit == 64 and six == 6
    t = tr.astype(np.int64)
    reached = min(64, int(iters))
    assert np.all(t[:, :reached, 0] > 0), "an iteration that ran has no record"
    assert np.all(t[:, reached:, :] == 0), "a record past the last iteration"
    r = t[:, :reached, :]
    assert np.all(np.diff(r[:, :, [0, 1, 2, 3, 5]], axis=2) >= 0), "stamps out of phase order"
    assert np.all(r[:, 1:, 0] >= r[:, :-1, 5]), "an iteration starts before the previous one ended"
    if nb == 1:
        assert np.all(r[:, :, 4] == 0), "a single-block shell has no grid barrier"
    else:
        assert np.all((r[:, :, 4] >= r[:, :, 3]) & (r[:, :, 4] <= r[:, :, 5]))
        # the reduce-barrier: every block of the shell has arrived before any leaves
        assert np.all(r[:, :, 4].max(axis=0) <= r[:, :, 5].min(axis=0))
    return r


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_trace_changes_nothing_and_is_consistent(name, precision):
    sh = S()
    prec = sh.SHELL_MIXED if precision == "mixed" else sh.SHELL_FP64
    case = CASES[name]()
    its0, x0, tr0 = _solve(case, False, prec)
    its1, x1, tr1 = _solve(case, True, prec)
    assert np.array_equal(its0, its1)
    np.testing.assert_array_equal(x0, x1)
    assert np.all(tr0 == 0), "tracing off returns zeros"
    if name == "cylinder32":
        assert tr1.shape[0] > 1, "the cylinder should span several CG blocks"
    if precision == "fp64":
        # one CG launch per FP64 solve: the trace covers all of its iterations
        r = check_trace(tr1, its1[0])
    else:
        # the refinement's last launch: its iteration count is not returned
        reached = int(np.count_nonzero(tr1[0, :, 0]))
        assert reached > 0
        r = check_trace(tr1, reached)
    span = (r[:, :, 5] - r[:, :, 0]) * 10.0   # ns at 100 MHz
    print(f"{name} {precision}: {tr1.shape[0]} blocks, {r.shape[1]} iterations traced, "
          f"mean iteration {span.mean() / 1e3:.2f} us", flush=True)


def test_trace_from_replayed_graphs_and_disable():
    """Newton steps replay the captured CG launch: tracing on gives the same
    states as tracing off, the trace holds the step's last CG launch, and
    turning tracing off returns zeros again."""
    sh = S()
    case = W.case_cylinder(32, 32)
    out = []
    for trace in (False, True):
        ctx = sh.context_for([case], precision=sh.SHELL_FP64, graphs=True)
        ctx.cg_trace_enable(trace)
        q, v = dev(case.q0.reshape(-1)), dev(case.v0.reshape(-1))
        q1, v1 = torch.empty_like(q), torch.empty_like(q)
        for k in range(3):
            pr = dev(case.presc((k + 1) * case.dt).reshape(-1))
            ctx.newton_step(case.dt, q, v, pr, q1, v1)
            q, q1 = q1, q
            v, v1 = v1, v
        tr = ctx.cg_trace_get()
        if trace:
            reached = int(np.count_nonzero(tr[0, :, 0]))
            assert reached > 0
            check_trace(tr, reached)
            ctx.cg_trace_enable(False)
            assert np.all(ctx.cg_trace_get() == 0)
        else:
            assert np.all(tr == 0)
        out.append((q.cpu().numpy(), v.cpu().numpy()))
        ctx.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
