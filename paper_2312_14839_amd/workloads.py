"""Seeded synthetic inputs for the BHEM thin-shell hot path.

This module only builds inputs: reference geometries sampled into nodal
generalized coordinates, constraint masks, initial states, prescribed values
and material parameters.  It holds none of the method's arithmetic (no basis
functions, quadrature, energies or solvers), so the HIP library and the CPU
oracle can both consume exactly the same arrays.

Nodal arrays are ``[nodes, 12]`` float64, DOF ``3*k + component`` with kind k
(0: x, 1: dx/dxi1, 2: dx/dxi2, 3: d2x/dxi1 dxi2).  Node (i, j) has index
``j * cols + i`` with ``cols = n1 + 1`` (open grid) or ``n1`` when column n1
is merged with column 0 (periodic along xi^1, Sec. 4.2 of the paper).

Sheets: a flat square of side 1 m with xi = physical coordinates, so the
reference is represented exactly.  Cylinder: xi^1 = arc length around the
axis, xi^2 = axial coordinate; the reference DOFs are the exact cylinder's
position and derivatives at the nodes.

The paper evaluates on its own scenes (Table 2); the workloads here reuse
their shapes and material ranges (flat cloth sheets of 30x30 patches, a
twisted sheet, a compressed cylinder) with seeded random perturbations.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

GRAVITY = (0.0, 0.0, -9.81)


@dataclasses.dataclass
class Case:
    """One shell: grid, material, reference DOFs, constraints and state."""
    name: str
    n1: int
    n2: int
    periodic1: int
    dxi1: float
    dxi2: float
    young: float
    poisson: float
    thickness: float
    density: float
    gravity: tuple
    ref: np.ndarray            # [nodes, 12] reference generalized coordinates
    fixed: np.ndarray          # [nodes, 12] uint8, 1 = prescribed DOF
    q0: np.ndarray             # [nodes, 12] state at t = 0
    v0: np.ndarray             # [nodes, 12] velocity at t = 0
    dt: float
    # prescribed values of all DOFs at time t (only fixed entries are used)
    presc: Optional[Callable[[float], np.ndarray]] = None
    damping: float = 0.0       # mass-proportional Rayleigh coefficient [1/s]

    @property
    def cols(self) -> int:
        return self.n1 if self.periodic1 else self.n1 + 1

    @property
    def nodes(self) -> int:
        return self.cols * (self.n2 + 1)

    @property
    def patches(self) -> int:
        return self.n1 * self.n2

    def node(self, i: int, j: int) -> int:
        if self.periodic1:
            i %= self.n1
        return j * self.cols + i


def flat_sheet_ref(n1: int, n2: int, lx: float = 1.0, ly: float = 1.0) -> np.ndarray:
    """Exact flat sheet in the plane z = 0 with xi = (x, y)."""
    cols = n1 + 1
    ref = np.zeros(((n2 + 1) * cols, 12))
    for j in range(n2 + 1):
        for i in range(cols):
            n = j * cols + i
            ref[n, 0:3] = (lx * i / n1, ly * j / n2, 0.0)
            ref[n, 3:6] = (1.0, 0.0, 0.0)
            ref[n, 6:9] = (0.0, 1.0, 0.0)
    return ref


def cylinder_ref(n1: int, n2: int, radius: float, length: float) -> np.ndarray:
    """Cylinder around the z axis, xi^1 = arc length (periodic), xi^2 = z."""
    ref = np.zeros(((n2 + 1) * n1, 12))
    for j in range(n2 + 1):
        for i in range(n1):
            phi = 2.0 * math.pi * i / n1
            n = j * n1 + i
            ref[n, 0:3] = (radius * math.cos(phi), radius * math.sin(phi), length * j / n2)
            ref[n, 3:6] = (-math.sin(phi), math.cos(phi), 0.0)
            ref[n, 6:9] = (0.0, 0.0, 1.0)
    return ref


def _material(young=1e5, poisson=0.3, thickness=1e-3, density=200.0):
    return dict(young=young, poisson=poisson, thickness=thickness, density=density)


def clamp_edges(n1: int, n2: int, edges) -> np.ndarray:
    """All 12 DOFs of every node on the named edges ('x0', 'x1', 'y0', 'y1')."""
    cols = n1 + 1
    fixed = np.zeros(((n2 + 1) * cols, 12), np.uint8)
    for j in range(n2 + 1):
        for i in range(cols):
            on = (("x0" in edges and i == 0) or ("x1" in edges and i == n1)
                  or ("y0" in edges and j == 0) or ("y1" in edges and j == n2))
            if on:
                fixed[j * cols + i, :] = 1
    return fixed


def perturb_positions(ref: np.ndarray, fixed: np.ndarray, sigma: float, rng) -> np.ndarray:
    """Reference plus N(0, sigma^2) on the position DOFs of nodes with no fixed DOF."""
    q = ref.copy()
    free_nodes = ~fixed.any(axis=1)
    q[free_nodes, 0:3] += rng.normal(0.0, sigma, size=(int(free_nodes.sum()), 3))
    return q


# ----------------------------------------------------------------- cases
def sheet_case(n=8, seed=1, dt=1e-3, edges=("x0",), gravity=GRAVITY, sigma=1e-4, name=None, **mat) -> Case:
    """Flat 1x1 m sheet of n x n patches, clamped edges, gravity, perturbed."""
    rng = np.random.default_rng(seed)
    ref = flat_sheet_ref(n, n)
    fixed = clamp_edges(n, n, edges)
    q0 = perturb_positions(ref, fixed, sigma, rng)
    m = _material(**mat)
    return Case(name or f"sheet{n}x{n}", n, n, 0, 1.0 / n, 1.0 / n, m["young"], m["poisson"], m["thickness"],
                m["density"], tuple(gravity), ref, fixed, q0, np.zeros_like(q0), dt)


def case_small_sheet(seed: int = 1) -> Case:
    """8x8 patches (81 nodes, 972 DOF), E=1e5, nu=0.3, h=1e-3, rho=200, edge
    xi1 = 0 clamped, gravity, N(0, 1e-4 m) position perturbation, dt = 1e-3."""
    return sheet_case(8, seed=seed, dt=1e-3, edges=("x0",), name="sheet8x8")


def case_twist(n: int = 30, seed: int = 2, omega: float = 1.0, dt: float = 2e-3, centre=None,
               sigma: float = 1e-4) -> Case:
    """n x n sheet whose centre node has its position held and its first
    derivatives rotated about z at omega rad/s (the paper's twisting cloth
    shape, 30x30 patches); no gravity; N(0, sigma) z-perturbation on free nodes."""
    rng = np.random.default_rng(seed)
    ref = flat_sheet_ref(n, n)
    cols = n + 1
    ci, cj = centre if centre is not None else (n // 2, n // 2)
    c = cj * cols + ci
    fixed = np.zeros_like(ref, dtype=np.uint8)
    fixed[c, 0:9] = 1
    q0 = ref.copy()
    free = np.ones(ref.shape[0], bool)
    free[c] = False
    q0[free, 2] += rng.normal(0.0, sigma, size=int(free.sum()))

    def presc(t: float) -> np.ndarray:
        out = ref.copy()
        a = omega * t
        rot = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])
        out[c, 3:6] = rot @ ref[c, 3:6]
        out[c, 6:9] = rot @ ref[c, 6:9]
        return out

    m = _material()
    return Case(f"twist{n}x{n}", n, n, 0, 1.0 / n, 1.0 / n, m["young"], m["poisson"], m["thickness"], m["density"],
                (0.0, 0.0, 0.0), ref, fixed, q0, np.zeros_like(q0), dt, presc)


def case_cylinder(n1: int = 256, n2: int = 256, seed: int = 4, radius: float = 0.2, length: float = 1.0,
                  dt: float = 1e-3, shorten_per_step: float = 1e-4, sigma: float = 1e-5) -> Case:
    """Periodic cylinder (n1 around, n2 along), both end rings fully clamped,
    the top ring moved down by ``shorten_per_step`` metres each step, gravity,
    seeded N(0, sigma) radial perturbation on free nodes."""
    rng = np.random.default_rng(seed)
    ref = cylinder_ref(n1, n2, radius, length)
    fixed = np.zeros_like(ref, dtype=np.uint8)
    fixed[:n1, :] = 1
    fixed[n2 * n1:, :] = 1
    q0 = ref.copy()
    for j in range(1, n2):
        for i in range(n1):
            phi = 2.0 * math.pi * i / n1
            q0[j * n1 + i, 0:3] += rng.normal(0.0, sigma) * np.array([math.cos(phi), math.sin(phi), 0.0])

    def presc(t: float) -> np.ndarray:
        out = ref.copy()
        steps = t / dt
        out[n2 * n1:, 2] -= shorten_per_step * steps
        return out

    m = _material()
    return Case(f"cylinder{n1}x{n2}", n1, n2, 1, 2.0 * math.pi * radius / n1, length / n2, m["young"],
                m["poisson"], m["thickness"], m["density"], GRAVITY, ref, fixed, q0, np.zeros_like(q0), dt, presc)


def case_batch(count: int = 256, seed: int = 3, nmin: int = 8, nmax: int = 64, dt: float = 1e-3) -> List[Case]:
    """Independent 1x1 m sheets with n1, n2 ~ U{nmin..nmax}, thickness
    log-uniform in [5e-4, 5e-3] m, each edge clamped with probability 1/2
    (redrawn until at least one is), gravity, N(0, 1e-4) perturbation."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n1, n2 = (int(v) for v in rng.integers(nmin, nmax + 1, size=2))
        h = float(math.exp(rng.uniform(math.log(5e-4), math.log(5e-3))))
        while True:
            mask = rng.random(4) < 0.5
            if mask.any():
                break
        edges = [e for e, m in zip(("x0", "x1", "y0", "y1"), mask) if m]
        ref = flat_sheet_ref(n1, n2)
        fixed = clamp_edges(n1, n2, edges)
        q0 = perturb_positions(ref, fixed, 1e-4, rng)
        m = _material(thickness=h)
        out.append(Case(f"batch{s}_{n1}x{n2}", n1, n2, 0, 1.0 / n1, 1.0 / n2, m["young"], m["poisson"],
                        m["thickness"], m["density"], GRAVITY, ref, fixed, q0, np.zeros_like(q0), dt))
    return out


def case_compression(n: int = 64, seed: int = 5, pct_per_100: float = 1.0, dt: float = 2e-3,
                     sigma: float = 1e-4) -> Case:
    """n x n sheet with edge xi1 = 0 clamped and edge xi1 = 1 clamped and
    moved inward along x by pct_per_100 percent of the side every 100 steps;
    no gravity; N(0, sigma) out-of-plane perturbation of free nodes (the
    imperfection that lets the sheet buckle)."""
    rng = np.random.default_rng(seed)
    ref = flat_sheet_ref(n, n)
    fixed = clamp_edges(n, n, ("x0", "x1"))
    q0 = ref.copy()
    free = ~fixed.any(axis=1)
    q0[free, 2] += rng.normal(0.0, sigma, size=int(free.sum()))
    cols = n + 1
    moving = np.array([j * cols + n for j in range(n + 1)])
    speed = pct_per_100 / 100.0 / (100.0 * dt)   # m/s for the 1 m side

    def presc(t: float) -> np.ndarray:
        out = ref.copy()
        out[moving, 0] -= speed * t
        return out

    m = _material()
    return Case(f"compress{n}x{n}", n, n, 0, 1.0 / n, 1.0 / n, m["young"], m["poisson"], m["thickness"],
                m["density"], (0.0, 0.0, 0.0), ref, fixed, q0, np.zeros_like(q0), dt, presc)


def case_precompressed(n: int = 6, strain: float = 0.01, thickness: float = 0.02, dt: float = 1.0, seed: int = 11,
                       sigma: float = 1e-4, young: float = 1e5, gravity=GRAVITY) -> Case:
    """n x n sheet already shortened along x by ``strain`` (positions and
    x-slopes scaled by 1 - strain), edges xi1 = 0 and xi1 = 1 clamped in that
    state, gravity, N(0, sigma) out-of-plane perturbation of free nodes.
    With a large time step the inertia no longer stabilises the compressed
    membrane, so the Newton systems of its first steps are indefinite."""
    rng = np.random.default_rng(seed)
    ref = flat_sheet_ref(n, n)
    q0 = ref.copy()
    q0[:, 0] *= 1.0 - strain
    q0[:, 3] *= 1.0 - strain
    fixed = clamp_edges(n, n, ("x0", "x1"))
    free = ~fixed.any(axis=1)
    q0[free, 2] += rng.normal(0.0, sigma, size=int(free.sum()))
    m = _material(young=young, thickness=thickness)
    return Case(f"precompressed{n}x{n}", n, n, 0, 1.0 / n, 1.0 / n, m["young"], m["poisson"], m["thickness"],
                m["density"], tuple(gravity), ref, fixed, q0, np.zeros_like(q0), dt)


def case_random_load(n: int, seed: int, dt: float = 2e-3) -> Case:
    """The load mix of the learned warm start's evaluation: with probability
    1/2 a twist at omega ~ U[0.5, 2] rad/s about a random interior node,
    else a compression at U[0.5, 2] percent per 100 steps."""
    rng = np.random.default_rng(seed)
    if rng.random() < 0.5:
        ci, cj = (int(v) for v in rng.integers(1, n, size=2))
        c = case_twist(n, seed=seed + 1, omega=float(rng.uniform(0.5, 2.0)), dt=dt, centre=(ci, cj))
    else:
        c = case_compression(n, seed=seed + 1, pct_per_100=float(rng.uniform(0.5, 2.0)), dt=dt)
    c.name = f"{c.name}_s{seed}"
    return c


def random_state(case: Case, seed: int, pos_sigma: float = 1e-3, der_sigma: float = 1e-2) -> np.ndarray:
    """A generic deformed state: reference plus Gaussian noise on every DOF
    (positions pos_sigma, derivative DOFs der_sigma).  For kernel parity."""
    rng = np.random.default_rng(seed)
    q = case.ref.copy()
    q[:, 0:3] += rng.normal(0.0, pos_sigma, size=(case.nodes, 3))
    q[:, 3:12] += rng.normal(0.0, der_sigma, size=(case.nodes, 9))
    return q


# ------------------------------------------------------- ray casting scenes
def height_field_ref(n1: int, n2: int, f, lx: float = 1.0, ly: float = 1.0, x0: float = 0.0,
                     y0: float = 0.0) -> np.ndarray:
    """Open n1 x n2 grid over [x0, x0+lx] x [y0, y0+ly] with xi = (x, y) and
    z = f(x, y); ``f`` returns (z, z_x, z_y, z_xy) so the nodal DOFs are the
    surface's own position and derivatives."""
    cols = n1 + 1
    ref = np.zeros(((n2 + 1) * cols, 12))
    for j in range(n2 + 1):
        for i in range(cols):
            x, y = x0 + lx * i / n1, y0 + ly * j / n2
            z, zx, zy, zxy = f(x, y)
            n = j * cols + i
            ref[n, 0:3] = (x, y, z)
            ref[n, 3:6] = (1.0, 0.0, zx)
            ref[n, 6:9] = (0.0, 1.0, zy)
            ref[n, 9:12] = (0.0, 0.0, zxy)
    return ref


def _saddle(x, y):
    # a bicubic Hermite patch reproduces this polynomial exactly
    return (0.25 * x * y - 0.15 * x * x + 0.1 * y * y, 0.25 * y - 0.3 * x, 0.25 * x + 0.2 * y, 0.25)


def _drape(x, y):
    # a bump with folds: A g(x) g(y) + B sin(k x) y^2, g(t) = exp(-t^2 / s)
    A, s, B, k = 0.35, 0.08, 0.04, 8.0 * math.pi
    gx, gy = math.exp(-x * x / s), math.exp(-y * y / s)
    dgx, dgy = -2.0 * x / s * gx, -2.0 * y / s * gy
    sk, ck = math.sin(k * x), math.cos(k * x)
    return (A * gx * gy + B * sk * y * y, A * dgx * gy + B * k * ck * y * y, A * gx * dgy + 2.0 * B * sk * y,
            A * dgx * dgy + 2.0 * B * k * ck * y)


def _scene_case(name, n1, n2, periodic1, dxi1, dxi2, ref) -> Case:
    m = _material()
    z = np.zeros_like(ref)
    return Case(name, n1, n2, periodic1, dxi1, dxi2, m["young"], m["poisson"], m["thickness"], m["density"],
                GRAVITY, ref, np.zeros_like(ref, dtype=np.uint8), ref.copy(), z, 1e-3)


RENDER_SCENES = ("plane", "cylinder", "drape")


def render_scene(name: str) -> Case:
    """The three scenes of the paper's rendering comparison (Sec. 5.1,
    Table 1): one warped patch ("plane"), a 10x10-patch open cylinder and a
    10x10-patch draped sheet."""
    if name == "plane":
        return _scene_case("plane", 1, 1, 0, 1.0, 1.0, height_field_ref(1, 1, _saddle))
    if name == "cylinder":
        return _scene_case("cylinder", 10, 10, 1, 2.0 * math.pi * 0.3 / 10, 0.1, cylinder_ref(10, 10, 0.3, 1.0))
    if name == "drape":
        return _scene_case("drape", 10, 10, 0, 0.1, 0.1, height_field_ref(10, 10, _drape, x0=-0.5, y0=-0.5))
    raise ValueError(f"unknown scene {name!r}")


# camera (eye, target) per scene: every scene fills most of the frame
_CAMERAS = {
    "plane": ((0.5, -0.35, 0.95), (0.5, 0.5, 0.0)),
    "cylinder": ((1.2, -1.4, 1.0), (0.0, 0.0, 0.5)),
    "drape": ((0.0, -1.05, 1.05), (0.0, 0.02, 0.02)),
}


def camera_rays(scene: str, width: int, height: int, spp: int = 1, seed: int = 8, fov_deg: float = 35.0,
                eye=None, target=None) -> np.ndarray:
    """Pinhole camera rays [height*width*spp, 6] (origin, unit direction),
    pixel-major, ``spp`` samples per pixel jittered uniformly inside the
    pixel with a seeded generator (up = +z)."""
    e, t = _CAMERAS.get(scene, ((0.0, -2.0, 1.0), (0.0, 0.0, 0.0)))
    e = np.asarray(eye if eye is not None else e, dtype=np.float64)
    t = np.asarray(target if target is not None else t, dtype=np.float64)
    fwd = t - e
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, (0.0, 0.0, 1.0))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(fov_deg) / 2.0)
    rng = np.random.default_rng(seed)
    jit = rng.random((height, width, spp, 2))
    px = (np.arange(width)[None, :, None] + jit[..., 0]) / width * 2.0 - 1.0
    py = 1.0 - (np.arange(height)[:, None, None] + jit[..., 1]) / height * 2.0
    d = fwd + (px * th * width / height)[..., None] * right + (py * th)[..., None] * up
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    rays = np.empty((height * width * spp, 6))
    rays[:, 0:3] = e
    rays[:, 3:6] = d.reshape(-1, 3)
    return rays
