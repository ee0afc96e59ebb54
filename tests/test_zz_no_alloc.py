"""shell_ray_cast_noalloc (the allocation-free variant of shell_ray_cast,
whose cooperative search hands rays over through the library's fixed device
buffer) against shell_ray_cast through the C ABI: two calls in a row, the
second with a smaller input, each bit-identical to the allocating entry
point on the same inputs (the two share their kernels).  Room for four
candidates on a lane sends most rays to the cooperative search, so the
fixed buffer is used, and the second call runs on what the first left in
it."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import ray_oracle as R
from paper_2312_14839_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
EPS = 1e-10


def _ctrl(cases, refs):
    from paper_2312_14839_amd import shell as S
    ctx = S.context_for(cases)
    ctrl = torch.empty((sum(c.patches for c in cases), 4, 4, 3), dtype=torch.float64, device="cuda")
    ctx.bezier(torch.as_tensor(np.concatenate(refs), device="cuda"), ctrl)
    torch.cuda.synchronize()
    ctx.close()
    return ctrl


def _cast(ctrl, rays, noalloc, **kw):
    from paper_2312_14839_amd import shell as S
    n = rays.shape[0]
    hit = torch.full((n, 3), np.nan, dtype=torch.float64, device="cuda")
    patch = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    pops = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    S.ray_cast(ctrl, rays, hit, patch, pops, noalloc=noalloc, eps=EPS, **kw)
    torch.cuda.synchronize()
    return hit.cpu().numpy(), patch.cpu().numpy(), pops.cpu().numpy()


@pytest.mark.parametrize("newton", [0, 8], ids=["midpoint", "newton"])
def test_noalloc_ray_cast_matches_the_allocating_entry_point(newton):
    ref = W.height_field_ref(6, 6, W._drape, x0=-0.5, y0=-0.5)
    low = ref.copy()
    low[:, 0] += 0.1
    low[:, 2] -= 0.03
    layers = W._scene_case("drape6", 6, 6, 0, 1 / 6, 1 / 6, ref)
    drape = W.render_scene("drape")
    calls = [(_ctrl([layers, layers], [ref, low]), W.camera_rays("drape", 40, 40, 1, seed=35)),
             (_ctrl([drape], [drape.ref]), W.camera_rays("drape", 24, 16, 1, seed=38))]
    for k, (ctrl, rays_h) in enumerate(calls):
        rays = torch.as_tensor(rays_h, device="cuda")
        print(f"noalloc call {k}: {rays.shape[0]} rays, {ctrl.shape[0]} patches, newton {newton}", flush=True)
        hn, pn, on = _cast(ctrl, rays, True, newton_iters=newton, heap_cap=4)
        ha, pa, oa = _cast(ctrl, rays, False, newton_iters=newton, heap_cap=4)
        assert np.array_equal(pn, pa) and np.array_equal(on, oa)
        assert np.array_equal(hn, ha, equal_nan=True)
        assert (pn >= 0).sum() > 100 and (on > 4).sum() > 100   # many rays went through the hand-over
    # the hits of the last call against the oracle (the allocating entry
    # point's own parity is tested with the other ray tests)
    ctrl_o = R.bezier_grid(O.make_shell(10, 10, 0.1, 0.1, 1e5, 0.3, 1e-3, 200.0), drape.ref)
    ok = pn != -2
    ho, po = R.ray_cast(ctrl_o, rays_h[ok], eps=EPS, newton_iters=newton)
    assert np.array_equal(pn[ok] >= 0, po >= 0)
