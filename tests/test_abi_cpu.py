"""The C-ABI library loads on the CPU, exports every symbol its header
declares, and rejects invalid descriptors before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2312_14839_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bhem_shell.h")


def _declared():
    src = open(HEADER).read()
    decl = r"^(?:shell_status|void|const char\s*\*)\s*\**\s*(shell_[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(decl, src, flags=re.M)))


def test_header_symbols_exported():
    from paper_2312_14839_amd import shell as S
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(S.lib, n), n
    assert sorted(S.EXPORTED) == names


def test_default_opts():
    from paper_2312_14839_amd import shell as S
    o = S.default_opts()
    assert o.precision == S.SHELL_FP64 and o.hessian == S.SHELL_HESS_EXACT
    assert o.graphs == 1 and o.cg_resident == 1
    assert o.newton_rtol == 1e-10 and o.pcg_rtol == 1e-10 and o.newton_maxit == 50


@pytest.mark.parametrize("field,value,msg", [
    ("n1", 0, "n1 and n2"),
    ("dxi1", -1.0, "dxi"),
    ("young", 0.0, "young"),
    ("poisson", 0.5, "poisson"),
    ("thickness", 0.0, "thickness"),
    ("periodic1", 1, "periodic"),
])
def test_invalid_descriptor_rejected(field, value, msg):
    from paper_2312_14839_amd import shell as S
    case = W.sheet_case(2)
    descs = (S.shell_desc * 1)()
    d = descs[0]
    ref = np.ascontiguousarray(case.ref)
    d.n1, d.n2, d.periodic1, d.dxi1, d.dxi2 = 2, 2, 0, 0.5, 0.5
    d.ref_host = ref.ctypes.data_as(C.POINTER(C.c_double))
    d.young, d.poisson, d.thickness, d.density = 1e5, 0.3, 1e-3, 200.0
    setattr(d, field, value)
    h = C.c_void_p()
    rc = S.lib.shell_create(descs, 1, None, C.byref(h))
    assert rc == S.SHELL_E_INVAL
    assert h.value is None
    assert msg in S.lib.shell_last_error(None).decode()


def test_nonfinite_reference_rejected():
    from paper_2312_14839_amd import shell as S
    case = W.sheet_case(2)
    case.ref[3, 4] = np.nan
    with pytest.raises(S.ShellError) as e:
        S.ShellContext([case])
    assert e.value.status == S.SHELL_E_INVAL


def test_null_arguments():
    from paper_2312_14839_amd import shell as S
    h = C.c_void_p()
    assert S.lib.shell_create(None, 1, None, C.byref(h)) == S.SHELL_E_INVAL
    S.lib.shell_destroy(None)   # NULL-safe
    assert S.lib.shell_energy_grad_hess(None, None, None, None, 0) == S.SHELL_E_INVAL


def S():
    from paper_2312_14839_amd import shell
    return shell


def test_point_load_is_the_consistent_nodal_load():
    """shell_point_load (host code of the library, no GPU) against the
    oracle's shape functions: f_I = Phi^I(xi) f on the 4 corner nodes of the
    containing patch, and f_nodal . q = f . x(xi) for any state q."""
    import numpy as np
    from oracle import oracle as O
    from paper_2312_14839_amd import workloads as W
    from gpu_util import rect_sheet
    rng = np.random.default_rng(4)
    cases = [rect_sheet(5, 4, 0.93, 0.94), W.case_cylinder(7, 3)]
    for case in cases:
        s = O.shell_from_case(case)
        L1, L2 = case.n1 * case.dxi1, case.n2 * case.dxi2
        for _ in range(5):
            xi1, xi2 = rng.uniform(0, L1), rng.uniform(0, L2)
            f = rng.normal(size=3)
            shift = L1 if case.periodic1 else 0.0          # a periodic shell wraps xi1
            fn = S().point_load(case, xi1 + shift, xi2, f)
            i, j = min(int(xi1 / case.dxi1), case.n1 - 1), min(int(xi2 / case.dxi2), case.n2 - 1)
            t1, t2 = xi1 / case.dxi1 - i, xi2 / case.dxi2 - j
            phi = O.shape_functions(t1, t2, case.dxi1, case.dxi2)[0]
            exp = np.zeros_like(fn)
            for c, node in enumerate(O.patch_nodes(s, i, j)):
                for k in range(4):
                    exp[node, 3 * k:3 * k + 3] += phi[4 * c + k] * f
            np.testing.assert_allclose(fn, exp, rtol=0, atol=1e-13 * np.abs(f).max())   # wrap and formula rounding
            q = case.ref + rng.normal(scale=1e-2, size=case.ref.shape)
            x = sum(phi[4 * c + k] * q[node, 3 * k:3 * k + 3]
                    for c, node in enumerate(O.patch_nodes(s, i, j)) for k in range(4))
            assert abs(np.sum(fn * q) - f @ x) <= 1e-13 * max(1.0, abs(f @ x))
    with pytest.raises(S().ShellError):
        S().point_load(cases[0], -0.1, 0.2, (0, 0, 1))


def test_ray_opts_defaults_and_validation():
    """shell_ray_cast checks sizes, pointers and options on the host and
    returns SHELL_E_INVAL before any device call; no rays is a no-op."""
    s = S()
    o = s.ray_opts()
    assert (o.eps, o.newton_tol, o.hole) == (1e-10, 1e-12, 1e-3)
    assert (o.newton_iters, o.max_depth, o.heap_cap, o.device) == (8, 60, s_heap_max(), 0)
    fake = C.c_void_p(0x1000)     # never dereferenced: validation fails first
    lib = s.lib

    def call(n_patches=1, n_rays=1, ctrl=fake, rays=fake, hit=fake, patch=fake, **kw):
        return lib.shell_ray_cast(ctrl, n_patches, rays, n_rays, C.byref(s.ray_opts(**kw)), hit, patch, None)

    assert lib.shell_ray_cast(fake, 1, fake, 1, None, fake, fake, None) == s.SHELL_E_INVAL
    assert call(n_rays=0, rays=None, hit=None, patch=None) == s.SHELL_OK
    cases = [dict(n_patches=-1), dict(n_patches=1 << 24), dict(n_rays=-1), dict(rays=None), dict(hit=None),
             dict(patch=None), dict(ctrl=None), dict(eps=0.0), dict(eps=float("nan")), dict(newton_tol=0.0),
             dict(hole=0.0), dict(hole=0.5), dict(newton_iters=-1), dict(newton_iters=65), dict(max_depth=0),
             dict(max_depth=61), dict(heap_cap=0), dict(heap_cap=s_heap_max() + 1)]
    for kw in cases:
        assert call(**kw) == s.SHELL_E_INVAL, kw
        assert lib.shell_last_error(None).decode(), kw


def s_heap_max():
    src = open(HEADER).read()
    return int(re.search(r"#define SHELL_RAY_HEAP_MAX (\d+)", src).group(1))


def test_ccd_validation():
    s = S()
    fake = C.c_void_p(0x1000)
    lib = s.lib
    o = s.ray_opts()
    assert lib.shell_ccd(fake, fake, 1, fake, 0, 1.0, C.byref(o), None, None, None) == s.SHELL_OK
    for dt in (0.0, -1.0, float("inf")):
        assert lib.shell_ccd(fake, fake, 1, fake, 1, dt, C.byref(o), fake, fake, None) == s.SHELL_E_INVAL
    assert lib.shell_ccd(fake, None, 1, fake, 1, 1.0, C.byref(o), fake, fake, None) == s.SHELL_E_INVAL
    assert lib.shell_ccd(fake, fake, 1, fake, 1, 1.0, None, fake, fake, None) == s.SHELL_E_INVAL
    assert lib.shell_ccd(fake, fake, 1, fake, 1, 1.0, C.byref(s.ray_opts(eps=0.0)), fake, fake, None) == s.SHELL_E_INVAL


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes mirror of a header struct has the header's field offsets
    and size (a C program built with gcc against the header prints them)."""
    import subprocess
    s = S()
    structs = [s.shell_desc, s.shell_opts, s.shell_step_stats, s.shell_timing, s.shell_tune_result,
               s.shell_ray_opts, s.shell_collider, s.shell_collide_opts, s.shell_collide_stats,
               s.shell_point_constraint, s.shell_alm_opts]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "bhem_shell.h"', 'int main(void) {']
    for st in structs:
        n = st.__name__
        lines.append(f'printf("{n} %zu\\n", sizeof({n}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{n}.{f} %zu\\n", offsetof({n}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for st in structs:
        n = st.__name__
        assert int(got[n]) == C.sizeof(st), n
        for f, _ in st._fields_:
            assert int(got[f"{n}.{f}"]) == getattr(st, f).offset, (n, f)
