"""Pins of the CPU oracle of the warm-start MLP: backward pass against central
finite differences of the FP64 loss, bfloat16 rounding against its
definition, and a step of Adam against its closed form on a quadratic.
CPU only."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_parameter_count():
    assert M.N_PARAMS == 60 * 128 + 128 + 128 * 128 + 128 + 128 * 12 + 12


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = M.init_params(1)
    theta += 0.05 * rng.normal(size=theta.shape)      # non-zero last layer
    x = rng.normal(size=(7, M.N_IN))
    t = rng.normal(size=(7, 12))
    loss, g = M.loss_and_grad(theta, x, t)
    # random entries plus a few of every parameter tensor (all of the small
    # output bias), so a slip in any tensor's gradient shows
    idx = list(rng.choice(theta.size, 60, replace=False))
    off = 0
    for name, shape in M.SHAPES:
        size = int(np.prod(shape))
        idx += list(off + rng.choice(size, min(size, 12), replace=False))
        off += size
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = 1e-6
        fd = (M.loss_and_grad(theta + e, x, t)[0] - M.loss_and_grad(theta - e, x, t)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.1415926, 1e-3, 65504.0])
    r = M.bf16_round(vals)
    # 8 significant bits: 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 -> 1 + 2^-6
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7 and r[3] == 1.0 + 2 ** -6
    assert abs(r[4] - vals[4]) <= 2 ** -8 * abs(vals[4])
    assert np.all(np.abs(r - vals) <= 2 ** -8 * np.abs(vals))


def test_adam_first_step_is_lr_sign():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    th, m, v = M.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(th, theta - 0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)


# planted mistakes in the network oracle, caught by the pins above
_MLP_MUTANTS = [
    ("ReLU mask dropped in the backward pass", "* (z2 > 0)", ""),
    ("W2 not transposed in the backward pass", "@ _r(p[\"W2\"], bf16).T)", "@ _r(p[\"W2\"], bf16))"),
    ("loss gradient without the factor 2", "dy = 2.0 * e / n", "dy = e / n"),
    ("bias gradient as a mean instead of a sum", "g[\"b3\"] = dy.sum(axis=0)", "g[\"b3\"] = dy.mean(axis=0)"),
    ("Adam without bias correction of v", "vh = v / (1 - b2 ** step)", "vh = v"),
    ("bf16 rounding by truncation", "r = ((u + 0x7FFF + lsb) >> 16) << 16", "r = (u >> 16) << 16"),
]


@pytest.mark.parametrize("i", range(len(_MLP_MUTANTS)), ids=[m[0] for m in _MLP_MUTANTS])
def test_planted_mistake_in_network_oracle_is_caught(i):
    import types
    name, old, new = _MLP_MUTANTS[i]
    src = open(M.__file__).read()
    assert old in src
    mod = types.ModuleType("mlp_mutant")
    exec(compile(src.replace(old, new, 1), "mlp_mutant", "exec"), mod.__dict__)
    pins = [test_backward_matches_central_differences, test_bf16_rounding, test_adam_first_step_is_lr_sign]
    original = globals()["M"]
    failed = 0
    for pin in pins:
        globals()["M"] = mod
        try:
            pin()
        except (AssertionError, ValueError, IndexError):
            failed += 1
        finally:
            globals()["M"] = original
    assert failed, f"no pin caught: {name}"
