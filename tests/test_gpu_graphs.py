"""HIP graphs and the autotuner of the batched form.

Graph replays run the same kernels in the same order as direct launches, so
every Newton step (several replays of each captured sequence, with the
solver's own eager work and synchronisations between them) must give
bit-identical states.  The autotuner changes the CG row-block layout, which
changes the order of the CG reductions only: results agree to the Newton
tolerance; its patch kernel tiles change nothing.  A second context of the
same shape takes the cached choice."""
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
    assert info["hess_waves"] in (4, 8) and info["energy_patches"] in (4, 8, 16)
    assert info["hess_us"] > 0 and info["energy_us"] > 0
    _, _, info2 = _run(cases, 1, 0, graphs=True, tune=True)
    assert info2["from_cache"] == 1 and info2["candidates"] == 0
    assert (info2["threads"], info2["rows_per_block"]) == (info["threads"], info["rows_per_block"])
    assert (info2["hess_waves"], info2["energy_patches"]) == (info["hess_waves"], info["energy_patches"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_patch_kernel_tiles_do_not_change_results(precision):
    """Every patch is one wavefront's (Hessian) or 16 lanes' (energy) work
    and patches of one colour share no matrix block, so the tiles only move
    work between blocks: energies, gradient and matrix are bit-identical for
    every tile the autotuner may choose."""
    from paper_2312_14839_amd import shell as sh
    case = W.case_twist(12)
    prec = sh.SHELL_MIXED if precision == "mixed" else sh.SHELL_FP64
    q = torch.from_numpy(W.random_state(case, seed=5).reshape(-1)).cuda()
    ref = None
    for waves, patches in ((4, 16), (8, 4), (4, 8), (8, 16)):
        ctx = sh.context_for([case], precision=prec)
        ctx.set_patch_tiles(waves, patches)
        g = torch.empty_like(q)
        e = ctx.energy_grad_hess(q, g, hessian=True)
        rp, ci, vals = ctx.get_bsr(0)
        out = (e, g.cpu().numpy(), vals)
        ctx.close()
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])
            assert np.array_equal(out[2], ref[2]), (waves, patches)
