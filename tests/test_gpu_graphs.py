"""HIP graphs and the CG layout autotuner of the batched form.

Graph replays run the same kernels in the same order as direct launches, so
every Newton step (several replays of each captured sequence, with the
solver's own eager work and synchronisations between them) must give
bit-identical states.  The autotuner changes the CG row-block layout, which
changes the order of the CG reductions only: results agree to the Newton
tolerance.  A second context of the same shape takes the cached layout."""
import numpy as np
import pytest

from paper_2312_14839_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def S():
    from paper_2312_14839_amd import shell
    return shell


def _run(cases, nsteps, precision, graphs, tune=False):
    sh = S()
    ctx = sh.context_for(cases, precision=precision, graphs=graphs, newton_rtol=1e-10, pcg_rtol=1e-10)
    info = ctx.autotune(60) if tune else None
    q = torch.from_numpy(np.concatenate([c.q0.reshape(-1) for c in cases])).cuda()
    v = torch.zeros_like(q)
    q1, v1 = torch.empty_like(q), torch.empty_like(q)
    states, its = [], []
    for k in range(nsteps):
        pr = torch.from_numpy(np.concatenate([(c.presc((k + 1) * c.dt) if c.presc else c.q0).reshape(-1)
                                              for c in cases])).cuda()
        rc, st = ctx.newton_step(cases[0].dt, q, v, pr, q1, v1)
        its.append([s["pcg_iters_total"] for s in st])
        q, q1 = q1, q
        v, v1 = v1, v
        states.append(q.cpu().numpy().copy())
    ctx.close()
    return states, its, info


@pytest.mark.parametrize("precision", [0, 1])
def test_graphs_bit_identical_single(precision):
    case = [W.case_twist(30)]
    a, ia, _ = _run(case, 4, precision, graphs=False)
    b, ib, _ = _run(case, 4, precision, graphs=True)
    assert ia == ib
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_graphs_bit_identical_batch():
    cases = W.case_batch(12, seed=21, nmin=6, nmax=20)
    a, ia, _ = _run(cases, 3, 0, graphs=False)
    b, ib, _ = _run(cases, 3, 0, graphs=True)
    assert ia == ib
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_autotune_same_result_and_cache():
    cases = W.case_batch(20, seed=22, nmin=8, nmax=40)
    a, _, _ = _run(cases, 2, 0, graphs=True)
    b, _, info = _run(cases, 2, 0, graphs=True, tune=True)
    assert info["candidates"] >= 2 and info["from_cache"] == 0
    assert info["threads"] in (256, 512, 1024) and info["blocks"] >= len(cases)
    assert info["us_per_iter"] > 0
    disp = np.abs(a[-1] - np.concatenate([c.q0.reshape(-1) for c in cases])).max()
    assert np.abs(a[-1] - b[-1]).max() <= 1e-8 * disp
    _, _, info2 = _run(cases, 1, 0, graphs=True, tune=True)
    assert info2["from_cache"] == 1 and info2["candidates"] == 0
    assert (info2["threads"], info2["rows_per_block"]) == (info["threads"], info["rows_per_block"])
