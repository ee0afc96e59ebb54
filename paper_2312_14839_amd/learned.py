"""Host driver of the learned Newton warm start.

The paper has no learned component; this is an extension of its Newton
solver (the network, its features and the acceptance of its guess are
described with the ``shell_mlp_*`` declarations of the C header).  This
module only orchestrates: it steps scenes of several shells through one
context, records training samples from the solver's own time steps, trains
the network with the library's kernels, and applies the acceptance gate that
keeps a trained network only if it lowers the CG iteration count on
held-out scenes below that of the same warm start without the network
(extrapolation of the previous correction only).  Every computation runs in libbhem.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

from . import shell as S
from . import workloads as W

LAYERS = [(S.MLP_IN, S.MLP_HIDDEN), (S.MLP_HIDDEN, S.MLP_HIDDEN), (S.MLP_HIDDEN, S.MLP_OUT)]


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases and a zero output layer (the untrained
    network adds no correction).  Layout W1, b1, W2, b2, W3, b3 (row-major)."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (fan_in, fan_out) in enumerate(LAYERS):
        if li == len(LAYERS) - 1:
            parts.append(np.zeros(fan_in * fan_out))
        else:
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, size=fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    th = np.concatenate(parts).astype(np.float32)
    assert th.size == S.MLP_PARAMS
    return th


class Scene:
    """Several shells stepped together in one context (concatenated nodes)."""

    def __init__(self, cases: Sequence[W.Case]):
        self.cases = list(cases)
        dts = {c.dt for c in self.cases}
        assert len(dts) == 1, "shells of one scene share the time step"
        self.dt = dts.pop()
        self.q0 = np.concatenate([c.q0.reshape(-1) for c in self.cases])
        self.v0 = np.concatenate([c.v0.reshape(-1) for c in self.cases])
        self.nodes = sum(c.nodes for c in self.cases)
        self.patches = sum(c.patches for c in self.cases)

    def presc(self, t: float) -> np.ndarray:
        """Prescribed values of every shell at time t (held shells: q0)."""
        return np.concatenate([(c.presc(t) if c.presc is not None else c.q0).reshape(-1) for c in self.cases])


def run(scene: Scene, steps: int, precision=S.SHELL_FP64, theta: Optional[np.ndarray] = None,
        record: Optional[Dict] = None, newton_rtol=1e-10, pcg_rtol=1e-10, stream=None) -> Dict:
    """Step `scene` `steps` times from q0.  theta: network parameters for the
    warm start (None = block-Jacobi from zero).  record: dict(capacity,
    per_shell, seed) to record training samples.  Returns the final state,
    per-step CG iteration totals, Newton iterations, warm starts taken and
    (with record) the recorded device tensors and their count."""
    import torch
    ws = S.SHELL_WS_MLP if theta is not None else S.SHELL_WS_NONE
    ctx = S.context_for(scene.cases, precision=precision, newton_rtol=newton_rtol, pcg_rtol=pcg_rtol,
                        warm_start=ws, stream=stream)
    out: Dict = {"pcg_iters": [], "newton_iters": [], "ws_used": [], "status": []}
    try:
        if theta is not None:
            ctx.mlp_set_params(theta)
        if record is not None:
            cap = int(record["capacity"])
            feat = torch.zeros((max(cap, 1), S.MLP_IN), dtype=torch.float32, device="cuda")
            tgt = torch.zeros((max(cap, 1), S.MLP_OUT), dtype=torch.float32, device="cuda")
            ctx.mlp_record(feat, tgt, cap, int(record["per_shell"]), int(record.get("seed", 0)))
        q = torch.from_numpy(scene.q0.copy()).cuda()
        v = torch.from_numpy(scene.v0.copy()).cuda()
        q1, v1 = torch.empty_like(q), torch.empty_like(q)
        for k in range(steps):
            pr = torch.from_numpy(scene.presc((k + 1) * scene.dt)).cuda()
            rc, st = ctx.newton_step(scene.dt, q, v, pr, q1, v1, allow_fail=True)
            out["status"].append(rc)
            out["pcg_iters"].append(sum(s["pcg_iters_total"] for s in st))
            out["newton_iters"].append(sum(s["newton_iters"] for s in st))
            out["ws_used"].append(sum(s["warm_start_used"] for s in st))
            q, q1 = q1, q
            v, v1 = v1, v
        torch.cuda.synchronize()
        out["q"] = q.cpu().numpy()
        if record is not None:
            out["n_samples"] = ctx.mlp_recorded()
            out["feat"], out["tgt"] = feat, tgt
    finally:
        ctx.close()
    return out


def train(feat, tgt, n_samples: int, schedule=((4000, 1e-3), (2000, 3e-4)), batch: int = 256, seed: int = 0,
          theta0: Optional[np.ndarray] = None):
    """Train on recorded device samples with the library's kernels, Adam
    through the (steps, learning rate) phases of `schedule`; returns
    (parameters, per-step mini-batch losses)."""
    holder = S.context_for([W.sheet_case(1)])
    try:
        holder.mlp_set_params(theta0 if theta0 is not None else init_params(seed))
        losses = [holder.mlp_train(feat, tgt, n_samples, batch, int(st), float(lr), seed + 7919 * i)
                  for i, (st, lr) in enumerate(schedule)]
        theta = holder.mlp_get_params()
    finally:
        holder.close()
    return theta, np.concatenate(losses)


def training_scene(count: int = 12, seed: int = 100, nmin: int = 24, nmax: int = 48, dt: float = 2e-3) -> Scene:
    """Sheets of random size under the random twist / compression loads."""
    rng = np.random.default_rng(seed)
    cases = [W.case_random_load(int(rng.integers(nmin, nmax + 1)), seed=int(rng.integers(1 << 30)), dt=dt)
             for _ in range(count)]
    return Scene(cases)


def record_configs(stream=None, twist_steps: int = 60, batch_steps: int = 3, cylinder_steps: int = 4,
                   seed: int = 7) -> Dict:
    """Training samples recorded from the solver's own converged steps on
    the three workloads of the method: the 30x30 twisting sheet
    (`twist_steps` steps, 512 nodes a step), the 256 batched sheets
    (`batch_steps` steps, 32 nodes per sheet a step) and the 256x256
    compressed cylinder (`cylinder_steps` steps, 4096 nodes a step; FP64
    throughout).  A step records only once its shell has a previous
    correction.  Returns the concatenated device tensors, their count and the
    count per workload."""
    import torch
    plan = [("twist30", Scene([W.case_twist(30)]), twist_steps, 512, 1e-10),
            ("batch256", Scene(W.case_batch(256)), batch_steps, 32, 1e-10),
            ("cylinder256", Scene([W.case_cylinder(256, 256)]), cylinder_steps, 4096, 1e-8)]
    feats, tgts, counts = [], [], {}
    for k, (name, sc, steps, per_shell, pcg_rtol) in enumerate(plan):
        cap = per_shell * len(sc.cases) * steps
        r = run(sc, steps, record=dict(capacity=cap, per_shell=per_shell, seed=seed + k), pcg_rtol=pcg_rtol,
                stream=stream)
        if any(st != S.SHELL_OK for st in r["status"]):
            raise RuntimeError(f"recording on {name}: a step did not converge")
        n = int(r["n_samples"])
        counts[name] = n
        feats.append(r["feat"][:n])
        tgts.append(r["tgt"][:n])
    feat = torch.cat(feats).contiguous()
    tgt = torch.cat(tgts).contiguous()
    return {"feat": feat, "tgt": tgt, "n_samples": int(feat.shape[0]), "per_workload": counts}


def gate(theta: np.ndarray, scenes: Sequence[Scene], steps: int, **kw) -> Dict:
    """Acceptance gate: the network is kept only if, on every held-out scene,
    CG needs strictly fewer iterations with it than with the
    extrapolation-only start (the same warm start with a zero network, i.e.
    everything but the network's own contribution) and every step of both
    converged.  Returns the per-scene CG iteration counts of the plain
    solver, the extrapolation-only start and the learned start, and the
    decision."""
    zero = init_params(0)
    plain, extra, learned, accept = [], [], [], True
    for sc in scenes:
        a = run(sc, steps, **kw)
        e = run(sc, steps, theta=zero, **kw)
        b = run(sc, steps, theta=theta, **kw)
        plain.append(int(np.sum(a["pcg_iters"])))
        extra.append(int(np.sum(e["pcg_iters"])))
        learned.append(int(np.sum(b["pcg_iters"])))
        ok = all(s == S.SHELL_OK for s in a["status"] + e["status"] + b["status"])
        accept = accept and ok and learned[-1] < extra[-1]
    return {"accept": accept, "plain_iters": plain, "extrapolation_iters": extra, "learned_iters": learned}
