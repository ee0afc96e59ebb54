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


ASM_CASES = {
    "sheet8": lambda: [W.case_small_sheet()],
    "twist12": lambda: [W.case_twist(12)],
    "cyl7x3_six_colours": lambda: [W.case_cylinder(7, 3)],
    "batch4": lambda: W.case_batch(4, nmin=4, nmax=10),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(ASM_CASES))
def test_single_launch_assembly_equals_colour_launches(name, precision):
    """The single-launch assembly (every patch's local blocks to scratch,
    then each stored block summed in colour order) performs the colour
    launches' additions in their order: the matrix of every shell is
    bit-identical, and so are two Newton steps (graphs replayed)."""
    from paper_2312_14839_amd import shell as sh
    cases = ASM_CASES[name]()
    prec = sh.SHELL_MIXED if precision == "mixed" else sh.SHELL_FP64
    q0 = np.concatenate([W.random_state(c, seed=5).reshape(-1) for c in cases])
    out = []
    for single in (0, 1):
        ctx = sh.context_for(cases, precision=prec)
        ctx.set_assembly(single)
        q = torch.from_numpy(q0.copy()).cuda()
        ctx.assemble(q, mass_scale=1.0 / cases[0].dt ** 2)
        mats = [ctx.get_bsr(s)[2] for s in range(len(cases))]
        qn = torch.from_numpy(np.concatenate([c.q0.reshape(-1) for c in cases])).cuda()
        v = torch.zeros_like(qn)
        q1, v1 = torch.empty_like(qn), torch.empty_like(qn)
        for k in range(2):
            pr = torch.from_numpy(np.concatenate([(c.presc((k + 1) * c.dt) if c.presc else c.q0).reshape(-1)
                                                  for c in cases])).cuda()
            ctx.newton_step(cases[0].dt, qn, v, pr, q1, v1)
            qn, q1 = q1, qn
            v, v1 = v1, v
        out.append((mats, qn.cpu().numpy()))
        ctx.close()
    for s, (a, b) in enumerate(zip(out[0][0], out[1][0])):
        assert np.array_equal(a, b), s
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_single_launch_assembly_needs_resident_patches():
    """A shell whose Hessian blocks do not all fit on the device at once
    keeps the colour launches; asking for the single launch is an error."""
    from paper_2312_14839_amd import shell as sh
    ctx = sh.context_for([W.case_cylinder(128, 128)], precision=sh.SHELL_FP64)
    with pytest.raises(sh.ShellError):
        ctx.set_assembly(1)
    ctx.set_assembly(0)
    ctx.close()
