#!/usr/bin/env python3
"""Benchmark of the BHEM thin-shell hot path on one MI355X.

A step is one implicit-Euler step (Newton iterations with patch
energy/gradient/Hessian assembly, block-Jacobi CG and line search) of the
chosen synthetic workload; inputs stay resident in HBM.  Prints one JSON line.

  value        patch E/grad/Hess evaluations per second of the plain FP64
               path: patches x Newton iterations (each iteration evaluates
               every patch's energy, gradient and Hessian) / timed seconds
  ms_per_step  FP64 implicit-step wall time
  mixed        the same for the FP32-Hessian/CG + FP64-residual form, with its
               relative displacement error against the FP64 path
  roofline     dominant kernel group of the FP64 run, measured with HIP events
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same workload
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("patch E/grad/Hess evals/s + Newton-step ms at 1e-5 rel err, plain FP64 vs mixed/learned")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# algorithmic matrix-core flops per patch of the Hessian kernel: the
# contraction (3 diagonal component pairs with 96-long reductions incl. the
# mass slot, 3 off-diagonal with 80) and the kinematics (16 Gauss points x 30
# values x 16 basis functions)
HESS_MFMA_FLOPS = 2 * 16 * 16 * (3 * 96 + 3 * 80) + 2 * 16 * 30 * 16


def make_case(name):
    """(case, description, solver tolerances) of a named workload."""
    from paper_2312_14839_amd import workloads as W
    if name == "cylinder":
        return (W.case_cylinder(256, 256), "cylinder 256x256 patches (periodic), R=0.2 m, L=1 m, axial compression",
                dict(newton_rtol=1e-10, pcg_rtol=1e-8))
    if name == "twist":
        return (W.case_twist(30), "sheet 30x30 patches, centre derivatives twisted at 1 rad/s",
                dict(newton_rtol=1e-10, pcg_rtol=1e-10))
    if name == "sheet":
        return (W.case_small_sheet(), "sheet 8x8 patches, one edge clamped, gravity",
                dict(newton_rtol=1e-10, pcg_rtol=1e-10))
    if name == "batch":
        cases = W.case_batch(256)
        return (cases, "256 sheets, patch grids U{8..64}^2, h logU[5e-4,5e-3], random clamped edges, gravity",
                dict(newton_rtol=1e-10, pcg_rtol=1e-10))
    raise SystemExit(f"unknown workload {name}")


class Batch:
    """A list of shells presented as one workload (concatenated node arrays)."""

    def __init__(self, cases):
        self.cases = cases
        self.name = f"batch{len(cases)}"
        self.patches = sum(c.patches for c in cases)
        self.nodes = sum(c.nodes for c in cases)
        self.dt = cases[0].dt
        self.q0 = np.concatenate([c.q0 for c in cases])
        self.v0 = np.concatenate([c.v0 for c in cases])
        self.presc = None
        self.n_shells = len(cases)


def shells_of(case):
    return case.cases if isinstance(case, Batch) else [case]


def presc_on_device(case, nsteps):
    """Prescribed DOF values of steps 1..nsteps, resident in HBM before timing."""
    import torch
    if case.presc is None:
        return [None] * nsteps
    return [torch.from_numpy(case.presc((k + 1) * case.dt).reshape(-1).copy()).cuda() for k in range(nsteps)]


def run_steps(case, precision, steps, warmup, stream, tol, autotune=True):
    """Autotune the CG layout, warm up, time `steps` implicit steps, then
    re-run a few more with the library's per-kernel event timing on.
    Returns (wall s, stats, timing, autotune result)."""
    import torch
    from paper_2312_14839_amd import shell as S
    ctx = S.context_for(shells_of(case), precision=precision, stream=stream, **tol)
    tune = ctx.autotune(100) if autotune else None
    n_timing = max(1, min(steps, 2))
    presc = presc_on_device(case, warmup + steps + n_timing)
    q = torch.from_numpy(case.q0.reshape(-1).copy()).cuda()
    v = torch.from_numpy(case.v0.reshape(-1).copy()).cuda()
    q1, v1 = torch.empty_like(q), torch.empty_like(q)
    k = 0
    stats_all = []

    def one_step():
        nonlocal q, v, q1, v1, k
        rc, st = ctx.newton_step(case.dt, q, v, presc[k], q1, v1, allow_fail=True)
        k += 1
        if rc != S.SHELL_OK:
            bad = [s for s in st if s["status"] != 0][:1]
            raise RuntimeError(f"newton step failed: {S.STATUS_NAMES.get(rc)} {bad}")
        q, q1 = q1, q
        v, v1 = v1, v
        # per step: Newton iterations of the slowest shell, CG iterations summed
        return {"newton_iters": max(s["newton_iters"] for s in st),
                "patch_evals": sum(c.patches * s["newton_iters"] for c, s in zip(shells_of(case), st)),
                "pcg_iters_total": sum(s["pcg_iters_total"] for s in st)}

    for _ in range(warmup):
        one_step()
    ctx.timing_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stats_all.append(one_step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # further steps with per-kernel event timing on (it adds synchronisations)
    ctx.timing_enable(True)
    for _ in range(n_timing):
        one_step()
    timing = ctx.timing_get()
    ctx.timing_enable(False)
    ctx.close()
    return wall, stats_all, timing, tune


def qstate_after(case, precision, nsteps, stream, tol):
    """State after nsteps steps from q0 (for the FP64-vs-mixed comparison)."""
    import torch
    from paper_2312_14839_amd import shell as S
    ctx = S.context_for(shells_of(case), precision=precision, stream=stream, **tol)
    presc = presc_on_device(case, nsteps)
    q = torch.from_numpy(case.q0.reshape(-1).copy()).cuda()
    v = torch.from_numpy(case.v0.reshape(-1).copy()).cuda()
    q1, v1 = torch.empty_like(q), torch.empty_like(q)
    for k in range(nsteps):
        rc, st = ctx.newton_step(case.dt, q, v, presc[k], q1, v1, allow_fail=True)
        if rc != S.SHELL_OK:
            raise RuntimeError(f"newton step failed: {S.STATUS_NAMES.get(rc)}")
        q, q1 = q1, q
        v, v1 = v1, v
    torch.cuda.synchronize()
    out = q.cpu().numpy().reshape(-1, 12)
    ctx.close()
    return out


def cg_resident(layout, fp32):
    """Whether the CG ran its resident instance (its own rows' vectors in
    registers and LDS): blocks of at most 4 (FP64 matrix, <= 512 threads;
    none at 1024) or 2 (FP32) row passes of threads/64 x 10 rows."""
    if not layout:
        return False
    maxp = (4 if layout["threads"] <= 512 else 0) if not fp32 else 2
    return layout["rows_per_block"] <= maxp * (layout["threads"] // 64) * 10


def cg_bytes(case, timing, tm_bytes, tv_bytes, resident):
    """Algorithmic HBM bytes of the CG kernel (single-reduction form).  Per
    iteration: every stored block (the upper-triangle blocks: 144 values, a
    column and a slot index, and the 12-value transposed product written to
    its slot by the product phase and read back by the update phase; the
    diagonal blocks, symmetric: 84 values); per node row its inverse
    diagonal block (symmetric, 84 stored values), the row pointer, slot range
    and free mask (10 bytes) and the passes over 12-vectors: with the
    resident instance 3 (the update reads the old u and writes the new one,
    the product reads it), else 13 (also r, x, p and s read and written, the
    stored part of w written and read)."""
    blocks = timing["cg_iter_blocks"]
    rows = timing["cg_iter_rows"]
    vec = 3 if resident else 13
    return ((blocks - rows) * (144 * tm_bytes + 8 + 24 * tv_bytes)
            + rows * (84 * tm_bytes + 84 * tv_bytes + 10 + vec * 12 * tv_bytes))


def profiled_traffic(case, fp32, kernel):
    """HBM bytes per launch of `kernel` (its FP64 or FP32 instance) from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of this workload (the
    FP64 section's or the mixed section's), or
    None when there is none or the kernel source has changed since it was
    taken."""
    import hashlib
    if case.name != "cylinder256x256":
        return None
    tag = f"{kernel}_fp32" if fp32 else kernel
    here = os.path.dirname(os.path.abspath(__file__))
    name = "cylinder256_mixed_rocprof.txt" if fp32 else "cylinder256_rocprof.txt"
    path = os.path.join(here, "profiles", name)
    src = os.path.join(here, "paper_2312_14839_amd", "csrc", "solver_kernels.hip")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        if line.startswith(f"TRAFFIC {tag} "):
            f = dict(kv.split("=") for kv in line.split()[2:])
            if f.get("solver_kernels_sha256") == digest:
                return float(f["bytes_per_launch"])
    return None


def roofline(case, timing, fp32, layout=None):
    ms = timing["ms"]
    grp = max(ms, key=lambda k: ms[k])
    n = max(timing["launches"][grp], 1)
    per_launch_ms = ms[grp] / n
    if grp == "cg":
        tb = 4 if fp32 else 8
        total = cg_bytes(case, timing, tb, tb, cg_resident(layout, fp32))
        ach = total / (ms[grp] * 1e-3) / 1e9
        traffic = profiled_traffic(case, fp32, "k_cg")
        inst = "single-reduction, r, x, p, s, w resident" if cg_resident(layout, fp32) else "vectors in memory"
        return grp, {"kernel": f"k_cg (persistent block-Jacobi CG, {inst})", "bound": "hbm", "achieved": ach,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "avg_launch_ms": per_launch_ms, "algorithmic_bytes_per_launch": total / n}
    if grp == "hessian":
        flops = timing["patch_evals"] * HESS_MFMA_FLOPS
        ach = flops / (ms[grp] * 1e-3) / 1e12
        peak = FP32_PEAK_TFLOPS if fp32 else FP64_PEAK_TFLOPS
        return grp, {"kernel": "k_hessian (patch Hessian + scatter)", "bound": "mfma", "achieved": ach,
                     "peak": peak, "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                     "avg_launch_ms": per_launch_ms, "algorithmic_flops_per_launch": flops / n}
    return grp, {"kernel": grp, "bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                 "traffic": None, "avg_launch_ms": per_launch_ms}


def spmv_bytes(stored, rows, s):
    """Algorithmic HBM bytes of one stand-alone SpMV (two launches) with the
    symmetric storage: every stored upper-triangle block (144 values of s
    bytes, a column and a slot index, and the 12 FP64 values of its
    transposed product written and read back) and diagonal block (84
    values); per row the row pointer, slot range and free mask (10 bytes),
    x read once, y written, then read and written again by the slot-summing
    launch (4 passes of 12 FP64)."""
    off = stored - rows
    return off * (144 * s + 8 + 2 * 96) + rows * (84 * s + 10 + 4 * 96)


def assembly_bytes(patches, stored, rows, s):
    """Algorithmic HBM bytes of one Hessian assembly: each patch adds its 10
    stored node blocks into the matrix, a read and a write of 84 values for
    each of the 4 diagonal blocks (packed symmetric) and of 144 for each of
    the 6 of the upper triangle, except the first touch of every stored block
    (a write only); the state q and reference q-bar read once per node."""
    off = stored - rows
    return ((2 * 4 * patches - rows) * 84 + (2 * 6 * patches - off) * 144) * s + rows * 2 * 96


def kernels_section(case, stream, reps=20):
    """Stand-alone rooflines on the workload's matrix at its initial state
    (K(q0) + M/dt^2): the SpMV (masked, both launches) against 8 TB/s, the
    Hessian assembly against the MFMA peak of its precision and the
    combined assembly + SpMV bytes against 8 TB/s."""
    import torch
    from paper_2312_14839_amd import shell as S
    out = {}
    for name, prec, s, peak in (("fp64", S.SHELL_FP64, 8, FP64_PEAK_TFLOPS), ("fp32", S.SHELL_MIXED, 4, FP32_PEAK_TFLOPS)):
        ctx = S.context_for(shells_of(case), precision=prec, stream=stream)
        tiles = ctx.autotune(20)
        rows = ctx.total_nodes
        stored = (ctx.nnzb + rows) // 2
        q = torch.from_numpy(case.q0.reshape(-1).copy()).cuda()
        ms = 1.0 / case.dt ** 2
        ctx.assemble(q, mass_scale=ms)
        g = torch.Generator(device="cuda")
        g.manual_seed(5)
        x = torch.randn(q.shape, dtype=q.dtype, device="cuda", generator=g)
        y = torch.empty_like(x)
        for _ in range(3):
            ctx.spmv(x, y, masked=True)
            ctx.assemble(q, mass_scale=ms)
        ctx.timing_enable(True)
        for _ in range(reps):
            ctx.spmv(x, y, masked=True)
        for _ in range(reps // 4):
            ctx.assemble(q, mass_scale=ms)
        t = ctx.timing_get()
        ctx.timing_enable(False)
        ctx.close()
        t_spmv = t["ms"]["spmv"] / reps * 1e-3
        t_asm = t["ms"]["hessian"] / (reps // 4) * 1e-3
        b_spmv = spmv_bytes(stored, rows, s)
        b_asm = assembly_bytes(case.patches, stored, rows, s)
        fl_asm = case.patches * HESS_MFMA_FLOPS
        out[name] = {
            "spmv": {"us": t_spmv * 1e6, "bytes": b_spmv, "GB_s": b_spmv / t_spmv / 1e9,
                     "frac_hbm": b_spmv / t_spmv / 1e9 / HBM_PEAK_GBS},
            "assembly": {"ms": t_asm * 1e3, "mfma_TFLOP_s": fl_asm / t_asm / 1e12,
                         "frac_mfma": fl_asm / t_asm / 1e12 / peak, "bytes": b_asm,
                         "GB_s": b_asm / t_asm / 1e9},
            "assembly_plus_spmv_frac_hbm": (b_spmv + b_asm) / (t_spmv + t_asm) / 1e9 / HBM_PEAK_GBS,
            "tiles": {"hess_patches_per_block": tiles["hess_waves"], "energy_patches_per_block": tiles["energy_patches"],
                      "hess_us": tiles["hess_us"], "hess_us_default_tiles": tiles["hess_us_default"],
                      "energy_us": tiles["energy_us"], "energy_us_default_tiles": tiles["energy_us_default"]},
        }
        print(f"[bench] {name}: SpMV {t_spmv * 1e6:.1f} us ({b_spmv / t_spmv / 1e9:.0f} GB/s), assembly "
              f"{t_asm * 1e3:.3f} ms ({fl_asm / t_asm / 1e12:.1f} TFLOP/s MFMA, {b_asm / t_asm / 1e9:.0f} GB/s)",
              file=sys.stderr, flush=True)
    return out


def hbm_achievable(gib=2, reps=10):
    """What the chip streams for plain kernels (torch's sum and copy over
    `gib` GiB of FP64): the achievable reference beside the 8 TB/s peak."""
    import torch
    n = gib * (1 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    out = {}
    for name, fn, nbytes in (("read", lambda: x.sum(), 8 * n), ("copy", lambda: y.copy_(x), 16 * n)):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / reps * 1e-3
        out[name + "_GB_s"] = nbytes / t / 1e9
    out["bytes_read"] = 8 * n
    del x, y
    torch.cuda.empty_cache()
    print(f"[bench] achievable: read {out['read_GB_s']:.0f} GB/s, copy {out['copy_GB_s']:.0f} GB/s (read + write)",
          file=sys.stderr, flush=True)
    return out


def cg_phases_section(case, stream, first=10):
    """Where a CG iteration's time goes, from the CG's own phase trace (the
    GPU's 100 MHz constant clock, stamped by each block's first thread): one
    solve on K(q0) + M/dt^2 with the autotuned layout, iterations
    `first`..63, means over blocks and iterations in microseconds.  update:
    the own rows' vector and preconditioner phase; neighbour_wait: waiting for
    the blocks whose rows the transposed products reach; product: the block's
    share of the symmetric product; arrival_tail: from the first thread's end
    of the product to the block's arrival at the reduce-barrier (its other
    wavefronts finishing); barrier_wait: from arrival to the barrier's exit;
    arrival_spread: per iteration, latest minus earliest arrival over the
    blocks."""
    import torch
    from paper_2312_14839_amd import shell as S
    out = {}
    for name, prec in (("fp64", S.SHELL_FP64), ("mixed", S.SHELL_MIXED)):
        ctx = S.context_for(shells_of(case), precision=prec, stream=stream)
        ctx.autotune(20)
        ctx.cg_trace_enable(True)
        q = torch.from_numpy(case.q0.reshape(-1).copy()).cuda()
        ctx.assemble(q, mass_scale=1.0 / case.dt ** 2)
        g = torch.Generator(device="cuda")
        g.manual_seed(5)
        b = torch.randn(q.shape, dtype=q.dtype, device="cuda", generator=g)
        x = torch.zeros_like(b)
        ctx.pcg_solve(b, x, rtol=1e-10)
        tr = ctx.cg_trace_get().astype(np.int64)
        ctx.close()
        reached = int(np.count_nonzero(tr[0, :, 0]))
        r = tr[:, first:reached, :] * 1e-2   # us
        if r.shape[1] == 0:
            continue
        solo = bool(np.all(r[:, :, 4] == 0))
        arr = r[:, :, 3] if solo else r[:, :, 4]
        out[name] = {
            "blocks": int(tr.shape[0]), "iterations": [first, reached],
            "update_us": float((r[:, :, 1] - r[:, :, 0]).mean()),
            "neighbour_wait_us": float((r[:, :, 2] - r[:, :, 1]).mean()),
            "product_us": float((r[:, :, 3] - r[:, :, 2]).mean()),
            "arrival_tail_us": float((arr - r[:, :, 3]).mean()),
            "barrier_wait_us": float((r[:, :, 5] - arr).mean()),
            "arrival_spread_us": float((arr.max(axis=0) - arr.min(axis=0)).mean()),
            "iteration_us": float((r[:, 1:, 0] - r[:, :-1, 0]).mean()) if r.shape[1] > 1 else None,
        }
        o = out[name]
        print(f"[bench] CG phases {name}: update {o['update_us']:.2f}, neighbour wait {o['neighbour_wait_us']:.2f}, "
              f"product {o['product_us']:.2f}, arrival tail {o['arrival_tail_us']:.2f}, barrier "
              f"{o['barrier_wait_us']:.2f}, iteration {o['iteration_us']:.2f} us ({o['blocks']} blocks)",
              file=sys.stderr, flush=True)
    return out


def pseudo_hessian_section(stream, steps=3, warmup=1):
    """Exact vs pseudo Hessian (the bending geometric term dropped) on the
    256x256 cylinder, FP64: Newton and CG iterations and time per step."""
    import torch
    from paper_2312_14839_amd import shell as S, workloads as W
    case = W.case_cylinder(256, 256)
    out = {}
    for name, hess in (("exact", S.SHELL_HESS_EXACT), ("pseudo", S.SHELL_HESS_PSEUDO)):
        ctx = S.context_for([case], precision=S.SHELL_FP64, hessian=hess, stream=stream, newton_rtol=1e-10,
                            pcg_rtol=1e-8)
        ctx.autotune(100)
        presc = [torch.from_numpy(case.presc((k + 1) * case.dt).reshape(-1).copy()).cuda()
                 for k in range(warmup + steps)]
        q = torch.from_numpy(case.q0.reshape(-1).copy()).cuda()
        v = torch.zeros_like(q)
        q1, v1 = torch.empty_like(q), torch.empty_like(q)
        stats, t0 = [], 0.0
        for k in range(warmup + steps):
            if k == warmup:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            rc, st = ctx.newton_step(case.dt, q, v, presc[k], q1, v1, allow_fail=True)
            if rc != S.SHELL_OK:
                raise RuntimeError(f"{name} Hessian: step {k + 1} failed: {S.STATUS_NAMES.get(rc)}")
            if k >= warmup:
                stats.append(st[0])
            q, q1 = q1, q
            v, v1 = v1, v
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"ms_per_step": 1e3 * wall / steps,
                     "newton_iters_per_step": sum(s["newton_iters"] for s in stats) / steps,
                     "cg_iters_per_step": sum(s["pcg_iters_total"] for s in stats) / steps,
                     "ls_backtracks_per_step": sum(s["ls_backtracks"] for s in stats) / steps}
        ctx.close()
    print(f"[bench] exact vs pseudo Hessian: {out['exact']['ms_per_step']:.2f} vs {out['pseudo']['ms_per_step']:.2f} "
          f"ms/step", file=sys.stderr, flush=True)
    return out


def twist_section(stream, steps=200):
    """The 30x30-patch twisting sheet (11,532 DOF), `steps` implicit steps of
    2 ms from rest, plain FP64 and mixed: wall time per step, per-step
    assembly (Hessian + block-Jacobi factorisation) and PCG kernel time from
    a second, event-timed run, and the relative displacement error of the
    mixed trajectory against the FP64 one (position DOFs, against the FP64
    displacement from the reference) after every step, reported not gated."""
    import torch
    from paper_2312_14839_amd import shell as S, workloads as W
    case = W.case_twist(30)
    presc = presc_on_device(case, steps)
    out = {}
    traj = {}
    for name, prec in (("fp64", S.SHELL_FP64), ("mixed", S.SHELL_MIXED)):
        ctx = S.context_for([case], precision=prec, stream=stream, newton_rtol=1e-10, pcg_rtol=1e-10)
        ctx.autotune(100)
        res = {}
        for timed in (False, True):
            q = torch.from_numpy(case.q0.reshape(-1).copy()).cuda()
            v = torch.from_numpy(case.v0.reshape(-1).copy()).cuda()
            q1, v1 = torch.empty_like(q), torch.empty_like(q)
            qs, stats = [], []
            ctx.timing_enable(timed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(steps):
                rc, st = ctx.newton_step(case.dt, q, v, presc[k], q1, v1, allow_fail=True)
                if rc != S.SHELL_OK:
                    raise RuntimeError(f"twist {name}: step {k + 1} failed: {S.STATUS_NAMES.get(rc)}")
                stats.append(st[0])
                q, q1 = q1, q
                v, v1 = v1, v
                if not timed:
                    qs.append(q.clone())
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if timed:
                tm = ctx.timing_get()["ms"]
                res["assembly_ms_per_step"] = (tm["hessian"] + tm["bj_factor"]) / steps
                res["pcg_ms_per_step"] = tm["cg"] / steps
            else:
                res["ms_per_step"] = 1e3 * wall / steps
                res["newton_iters_per_step"] = sum(s["newton_iters"] for s in stats) / steps
                res["cg_iters_per_step"] = sum(s["pcg_iters_total"] for s in stats) / steps
                traj[name] = torch.stack(qs).cpu().numpy().reshape(steps, -1, 12)
        ctx.timing_enable(False)
        ctx.close()
        out[name] = res
    ref_pos = case.ref[:, 0:3]
    num = np.linalg.norm((traj["mixed"] - traj["fp64"])[:, :, 0:3], axis=(1, 2))
    den = np.linalg.norm(traj["fp64"][:, :, 0:3] - ref_pos[None], axis=(1, 2))
    err = num / np.maximum(den, 1e-300)
    out["mixed"]["rel_disp_err_vs_fp64_max"] = float(err.max())
    out["mixed"]["rel_disp_err_vs_fp64_last"] = float(err[-1])
    out["steps"] = steps
    out["workload"] = "sheet 30x30 patches, centre derivatives twisted at 1 rad/s, dt 2 ms, from rest"
    print(f"[bench] twist 30x30, {steps} steps: fp64 {out['fp64']['ms_per_step']:.2f} ms/step "
          f"(assembly {out['fp64']['assembly_ms_per_step']:.3f}, PCG {out['fp64']['pcg_ms_per_step']:.3f}), "
          f"mixed {out['mixed']['ms_per_step']:.2f} ms/step, max err {err.max():.2e}", file=sys.stderr, flush=True)
    return out


def post_buckling_section(stream, steps=3, before=300):
    """Newton-step time of the 256x256 cylinder after `before` steps of
    compression (past buckling), FP64, CG layout autotuned, with the exact
    and with the pseudo Hessian from the same state; the steps before are
    not timed."""
    import torch
    from paper_2312_14839_amd import shell as S, workloads as W
    case = W.case_cylinder(256, 256)
    presc = [torch.from_numpy(case.presc((k + 1) * case.dt).reshape(-1).copy()).cuda()
             for k in range(before + steps)]

    def run(ctx, q, v, k0, k1):
        q1, v1 = torch.empty_like(q), torch.empty_like(q)
        stats = []
        for k in range(k0, k1):
            rc, st = ctx.newton_step(case.dt, q, v, presc[k], q1, v1, allow_fail=True)
            if rc != S.SHELL_OK:
                raise RuntimeError(f"post-buckling run: step {k + 1} failed: {S.STATUS_NAMES.get(rc)}")
            stats.append(st[0])
            q, q1 = q1, q
            v, v1 = v1, v
        return q, v, stats

    ctx = S.context_for([case], precision=S.SHELL_FP64, stream=stream, newton_rtol=1e-10, pcg_rtol=1e-8)
    ctx.autotune(100)
    q0 = torch.from_numpy(case.q0.reshape(-1).copy()).cuda()
    qb, vb, _ = run(ctx, q0, torch.zeros_like(q0), 0, before)
    qn = qb.cpu().numpy().reshape(-1, 12)
    out = {"steps_before": before, "steps": steps,
           "max_radial_deviation_m": float(np.abs(np.hypot(qn[:, 0], qn[:, 1]) - 0.2).max())}
    for name, hess in (("exact", S.SHELL_HESS_EXACT), ("pseudo", S.SHELL_HESS_PSEUDO)):
        if hess != S.SHELL_HESS_EXACT:
            ctx.close()
            ctx = S.context_for([case], precision=S.SHELL_FP64, hessian=hess, stream=stream, newton_rtol=1e-10,
                                pcg_rtol=1e-8)
            ctx.autotune(100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, stats = run(ctx, qb.clone(), vb.clone(), before, before + steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"ms_per_step": 1e3 * wall / steps,
                     "newton_iters_per_step": sum(s["newton_iters"] for s in stats) / steps,
                     "cg_iters_per_step": sum(s["pcg_iters_total"] for s in stats) / steps,
                     "ls_backtracks_per_step": sum(s["ls_backtracks"] for s in stats) / steps,
                     "patch_evals_per_s": case.patches * sum(s["newton_iters"] for s in stats) / wall}
    ctx.close()
    print(f"[bench] post-buckling (after {before} steps): exact {out['exact']['ms_per_step']:.2f}, pseudo "
          f"{out['pseudo']['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    return out


def learned_section(stream):
    """The learned Newton warm start on held-out sheets: samples recorded from
    the solver's own steps on the twisting 30x30 sheet, the 256 batched
    sheets and the 256x256 cylinder, the network trained on the GPU, then 12
    steps of two 64x64 and one 128x128 unseen sheet under random twist /
    compression, plain solver vs warm start (and the extrapolation-only
    start, zero network, as the ablation)."""
    import torch
    from paper_2312_14839_amd import learned as L, workloads as W
    t0 = time.perf_counter()
    rec = L.record_configs(stream=stream)
    t_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    theta, losses = L.train(rec["feat"], rec["tgt"], rec["n_samples"], schedule=((8000, 1e-3), (4000, 3e-4)),
                            batch=512, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_samples, per_workload = rec["n_samples"], rec["per_workload"]
    del rec
    scenes = [L.Scene([W.case_random_load(n, seed=sd)]) for n, sd in ((64, 906), (64, 910), (128, 903))]
    res = {"plain": [0, 0.0], "learned": [0, 0.0], "extrapolation_only": [0, 0.0]}
    zero = L.init_params(0)
    steps = 12
    strict = True
    for sc in scenes:
        per = {}
        for key, th in (("plain", None), ("learned", theta), ("extrapolation_only", zero)):
            L.run(sc, 2, theta=th, stream=stream)                      # warm-up (graph capture, caches)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = L.run(sc, steps, theta=th, stream=stream)
            torch.cuda.synchronize()
            per[key] = int(np.sum(r["pcg_iters"]))
            res[key][0] += per[key]
            res[key][1] += time.perf_counter() - t0
        strict = strict and per["learned"] < per["extrapolation_only"]
    nsteps = steps * len(scenes)
    out = {k: {"cg_iters_per_step": v[0] / nsteps, "ms_per_step": 1e3 * v[1] / nsteps} for k, v in res.items()}
    # the gate's rule: the network counts only if it beats the same start
    # without it (extrapolation of the previous correction) on every scene
    out["network_accepted"] = bool(strict)
    out.update({"train_samples": int(n_samples), "train_samples_per_workload": per_workload,
                "train_steps": int(losses.size), "train_loss_first": float(np.mean(losses[:20])),
                "train_loss_last": float(np.mean(losses[-100:])), "record_s": t_rec, "train_s": t_train,
                "eval": "twist/compression 64x64 (seeds 906, 910) and 128x128 (seed 903), 12 steps each, dt 2e-3"})
    print(f"[bench] learned: CG its/step plain {out['plain']['cg_iters_per_step']:.1f} learned "
          f"{out['learned']['cg_iters_per_step']:.1f} extrapolation {out['extrapolation_only']['cg_iters_per_step']:.1f}",
          file=sys.stderr, flush=True)
    return out


def collision_section(stream, steps=40):
    """Collision handling (Sec. 6.2) against a sphere: a 64x64-patch sheet
    clamped along one edge falls under gravity onto it, each step an
    implicit Newton step and then the collision pass (s = 3 samples a side,
    36,864 samples; rollback, impulses, push-out); wall time of both per
    step.  Then the sampled detection alone at the cylinder's scale: 589,824
    samples of the 256x256 cylinder's first step against a sphere inside it
    (no contact), per call."""
    import torch
    from paper_2312_14839_amd import shell as S, workloads as W
    case = W.sheet_case(64, edges=("y0",), sigma=0.0, dt=5e-3)
    sphere = [("sphere", (0.5, 0.7, -0.32), 0.3)]
    ctx = S.context_for([case], stream=stream)
    q = torch.from_numpy(case.q0.reshape(-1).copy()).cuda()
    v = torch.zeros_like(q)
    q1, v1, qo, vo = (torch.empty_like(q) for _ in range(4))
    t_newton = t_coll = 0.0
    contacts = steps_with_contact = 0
    sim_time = 0.0
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = ctx.newton_step(case.dt, q, v, None, q1, v1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cs = ctx.collide(case.dt, q, q1, v1, sphere, qo, vo)
        t2 = time.perf_counter()
        if rc != S.SHELL_OK:
            raise RuntimeError(f"collision run: step {k + 1} failed: {S.STATUS_NAMES.get(rc)}")
        if k >= 2:
            t_newton += t1 - t0
            t_coll += t2 - t1
        contacts += cs["contacts"]
        steps_with_contact += cs["contacts"] > 0
        sim_time += cs["t_contact"] if cs["contacts"] else case.dt
        q, qo = qo, q
        v, vo = vo, v
    ctx.close()
    out = {"workload": "sheet 64x64 patches clamped along one edge, falling onto a sphere (R 0.3 m), dt 5 ms, "
                       f"{steps} steps, 3x3 samples per patch",
           "newton_ms_per_step": 1e3 * t_newton / (steps - 2), "collide_ms_per_step": 1e3 * t_coll / (steps - 2),
           "steps_with_contact": steps_with_contact, "contacts_per_step": contacts / steps,
           "simulated_time_s": sim_time}
    cyl = W.case_cylinder(256, 256)
    ctx = S.context_for([cyl], stream=stream)
    q0 = torch.from_numpy(cyl.q0.reshape(-1).copy()).cuda()
    v0 = torch.zeros_like(q0)
    q1, v1, qo, vo = (torch.empty_like(q0) for _ in range(4))
    ctx.newton_step(cyl.dt, q0, v0, torch.from_numpy(cyl.presc(cyl.dt).reshape(-1).copy()).cuda(), q1, v1)
    inner = [("sphere", (0.0, 0.0, 0.5), 0.19)]
    ctx.collide(cyl.dt, q0, q1, v1, inner, qo, vo)
    reps = 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.collide(cyl.dt, q0, q1, v1, inner, qo, vo)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    ctx.close()
    nsamp = cyl.patches * 9
    out["detection_cylinder256"] = {"samples": nsamp, "ms_per_call": ms, "samples_per_s": nsamp / (ms * 1e-3)}
    print(f"[bench] collision: newton {out['newton_ms_per_step']:.2f} ms + collide {out['collide_ms_per_step']:.2f} ms "
          f"per step, {out['contacts_per_step']:.1f} contacts/step; detection {ms:.3f} ms for {nsamp} samples",
          file=sys.stderr, flush=True)
    return out


def batch_section(stream, steps=3, warmup=1):
    """The 256-sheet batch in one context (a14): 256 flat sheets with patch
    grids U{8..64}^2, one persistent CG launch for all of them per Newton
    iteration; FP64, the CG layout autotuned; wall time per step and patch
    evaluations per second (each Newton iteration of a shell evaluates all
    of its patches)."""
    case_list, desc, tol = make_case("batch")
    case = Batch(case_list)
    wall, st, tm, tune = run_steps(case, 0, steps, warmup, stream, tol, True)
    cg_its = sum(s["pcg_iters_total"] for s in st) / steps
    out = {"workload": desc, "shells": len(case_list), "patches": case.patches, "dof": 12 * case.nodes,
           "ms_per_step": 1e3 * wall / steps, "patch_evals_per_s": sum(s["patch_evals"] for s in st) / wall,
           "newton_iters_per_step_slowest_shell": sum(s["newton_iters"] for s in st) / steps,
           "cg_iters_per_step_summed": cg_its, "cg_layout": tune, "kernel_ms_event_timed_steps": tm["ms"],
           "cg_launches_event_timed_steps": tm["launches"]["cg"]}
    print(f"[bench] batch: {out['ms_per_step']:.1f} ms/step, {out['patch_evals_per_s'] / 1e6:.2f} M patch evals/s",
          file=sys.stderr, flush=True)
    return out


def loads_section(stream, steps=3):
    """Follower pressure (Sec. 4.3) and point constraints imposed by the
    augmented Lagrangian method (Sec. 4.2, 6.1) at scale.  (a) The 256x256
    cylinder of the main workload with an internal pressure of 5 Pa, its
    load evaluated at each step's start, against the same steps without it.
    (b) A 64x64-patch sheet under gravity clamped along its edge y = 0
    (nodal constraints), alone and with three points inside patches also
    held at their reference positions (point constraints, penalty 1e3)."""
    import torch
    from paper_2312_14839_amd import shell as S, workloads as W
    out = {}
    cyl = W.case_cylinder(256, 256)
    presc = presc_on_device(cyl, steps + 1)
    for label, p in (("no_pressure", None), ("pressure_5Pa", [5.0])):
        ctx = S.context_for([cyl], stream=stream, newton_rtol=1e-10, pcg_rtol=1e-8)
        if p is not None:
            ctx.set_pressure(p)
        q = torch.from_numpy(cyl.q0.reshape(-1).copy()).cuda()
        v = torch.zeros_like(q)
        q1, v1 = torch.empty_like(q), torch.empty_like(q)
        ctx.newton_step(cyl.dt, q, v, presc[0], q1, v1)   # warm-up (graph capture)
        q, q1, v, v1 = q1, q, v1, v
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = cg = 0
        for k in range(steps):
            rc, st = ctx.newton_step(cyl.dt, q, v, presc[k + 1], q1, v1)
            its += st[0]["newton_iters"]
            cg += st[0]["pcg_iters_total"]
            q, q1, v, v1 = q1, q, v1, v
        torch.cuda.synchronize()
        out[label] = {"ms_per_step": 1e3 * (time.perf_counter() - t0) / steps, "newton_iters_per_step": its / steps,
                      "cg_iters_per_step": cg / steps}
        ctx.close()
    n = 64
    clamped = W.sheet_case(n, edges=("y0",), sigma=0.0, dt=5e-3)
    # three points inside patches held at their reference positions (a
    # sheet tacked to a frame at three spots besides its clamped edge)
    pts = [(0, 0, x, y, (x, y, 0.0)) for x, y in ((0.3 + 0.3 / n, 0.5 + 0.4 / n), (0.5 + 0.3 / n, 0.75 + 0.4 / n),
                                                  (0.7 + 0.3 / n, 0.5 + 0.4 / n))]
    for label, case, cons in (("nodal_clamp", clamped, None), ("clamp_and_point_constraints", clamped, pts)):
        ctx = S.context_for([case], stream=stream)
        if cons:
            ctx.set_point_constraints(cons, penalty=1e3, tol=1e-9)
        q = torch.from_numpy(case.q0.reshape(-1).copy()).cuda()
        v = torch.zeros_like(q)
        q1, v1 = torch.empty_like(q), torch.empty_like(q)
        rc, st = ctx.newton_step(case.dt, q, v, None, q1, v1)
        q, q1, v, v1 = q1, q, v1, v
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = cg = outer = 0
        res = 0.0
        for k in range(steps):
            rc, st = ctx.newton_step(case.dt, q, v, None, q1, v1)
            its += st[0]["newton_iters"]
            cg += st[0]["pcg_iters_total"]
            outer += st[0]["alm_outer"]
            res = max(res, st[0]["alm_residual"])
            q, q1, v, v1 = q1, q, v1, v
        torch.cuda.synchronize()
        out[label] = {"ms_per_step": 1e3 * (time.perf_counter() - t0) / steps, "newton_iters_per_step": its / steps,
                      "cg_iters_per_step": cg / steps}
        if cons:
            out[label].update(multiplier_updates_per_step=outer / steps, max_constraint_residual=res,
                              constraints=len(cons))
        ctx.close()
    out["workload"] = ("cylinder 256x256 with and without 5 Pa internal pressure (steps 2-4); sheet 64x64, "
                       "gravity, dt 5 ms, edge y=0 clamped, alone and with three interior points held "
                       "(penalty 1e3, tol 1e-9), steps 2-4")
    print(f"[bench] loads: cylinder {out['no_pressure']['ms_per_step']:.1f} -> {out['pressure_5Pa']['ms_per_step']:.1f} "
          f"ms/step with pressure; sheet clamp {out['nodal_clamp']['ms_per_step']:.1f} ms/step, with point constraints "
          f"{out['clamp_and_point_constraints']['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# Table 1 of the paper: seconds to render each scene on a desktop CPU (16
# samples per pixel, image size not stated, shading included), for the
# midpoint subdivision and for the Newton-accelerated form.  Context only.
PAPER_RENDER_S = {"plane": (58.3, 4.5), "cylinder": (91.6, 9.7), "drape": (86.0, 14.8)}


def render_section(stream, width=512, height=512, spp=16, reps=3, eps=1e-10):
    """Static ray--patch intersection (Sec. 5.1) on the paper's three render
    scenes (one warped patch, a 10x10-patch cylinder, a 10x10-patch draped
    sheet): Bezier control points from the shell state on the device, then
    one pinhole-camera frame of width x height pixels x spp jittered samples,
    midpoint subdivision and Newton-accelerated forms.  Kernel time from HIP
    events around `reps` launches; pops = candidate surfaces examined per
    ray.  The oracle's rate on a seeded sample of the same rays (all host
    threads) is reported with the CPU baseline.  The cylinder and the drape
    also run the dynamic intersection of Sec. 5.2 (`ccd_frame`) on the same
    number of moving points."""
    import torch
    from paper_2312_14839_amd import shell as S, workloads as W
    out = {"workload": f"{width}x{height} pixels x {spp} samples per scene, eps {eps:g}, hole 1e-3, "
                       f"8 Newton steps", "rays_per_frame": width * height * spp}
    for sc in W.RENDER_SCENES:
        case = W.render_scene(sc)
        ctx = S.context_for([case], stream=stream)
        ctrl = torch.empty((case.patches, 4, 4, 3), dtype=torch.float64, device="cuda")
        ctx.bezier(torch.as_tensor(case.ref, device="cuda"), ctrl)
        rays_h = W.camera_rays(sc, width, height, spp)
        rays = torch.as_tensor(rays_h, device="cuda")
        n = rays.shape[0]
        hit = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        patch = torch.empty(n, dtype=torch.int32, device="cuda")
        pops = torch.empty(n, dtype=torch.int32, device="cuda")
        res = {"patches": case.patches}
        for mode, ni in (("midpoint", 0), ("newton", 8)):
            S.ray_cast(ctrl, rays, hit, patch, pops, stream=stream, newton_iters=ni, eps=eps)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                S.ray_cast(ctrl, rays, hit, patch, pops, stream=stream, newton_iters=ni, eps=eps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            p, pp = patch.cpu().numpy(), pops.cpu().numpy()
            res[mode] = {"ms_per_frame": ms, "rays_per_s": n / (ms * 1e-3), "hit_fraction": float(np.mean(p >= 0)),
                         "no_result": int(np.sum(p < -1)), "pops_mean": float(pp.mean()),
                         "pops_p99": float(np.percentile(pp, 99)), "pops_max": int(pp.max()),
                         "paper_table1_s": PAPER_RENDER_S[sc][0 if ni == 0 else 1]}
            print(f"[bench] render {sc} {mode}: {ms:.2f} ms/frame, {n / ms / 1e3:.1f} M rays/s, "
                  f"pops mean {pp.mean():.2f} max {pp.max()}", file=sys.stderr, flush=True)
        if sc != "plane":
            res["ccd"] = ccd_frame(ctx, case, ctrl, stream, width, height, spp, reps, eps)
        ctx.close()
        out[sc] = res
    return out


def rigid_velocity(case, V=(0.0, 0.0, -0.5), w=(0.3, -0.2, 0.5)):
    """Nodal velocities of the rigid motion V + w x x (derivative DOFs: w x)."""
    q = case.ref.reshape(-1, 4, 3)
    out = np.cross(np.asarray(w), q)
    out[:, 0] += np.asarray(V)
    return out.reshape(-1, 12)


def ccd_points(scene, width, height, spp):
    """Points starting 1 m along the scene's camera rays, moving along them
    at 3 m/s (one step of 0.5 s)."""
    from paper_2312_14839_amd import workloads as W
    pts = W.camera_rays(scene, width, height, spp)
    pts[:, :3] += pts[:, 3:]
    pts[:, 3:] *= 3.0
    return pts


def ccd_frame(ctx, case, ctrl, stream, width, height, spp, reps, eps, dt=0.5):
    """Dynamic intersection (Sec. 5.2): the scene moving rigidly (0.5 m/s
    down, rotating at |w| = 0.62 rad/s) against the moving points of
    ccd_points over one step; control-point velocities from the nodal ones
    with shell_bezier."""
    import torch
    from paper_2312_14839_amd import shell as S
    vel = torch.empty_like(ctrl)
    ctx.bezier(torch.as_tensor(rigid_velocity(case), device="cuda"), vel)
    pts = torch.as_tensor(ccd_points(case.name, width, height, spp), device="cuda")
    n = pts.shape[0]
    hit = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    patch = torch.empty(n, dtype=torch.int32, device="cuda")
    pops = torch.empty(n, dtype=torch.int32, device="cuda")
    res = {}
    for mode, ni in (("midpoint", 0), ("newton", 8)):
        S.ccd(ctrl, vel, pts, dt, hit, patch, pops, stream=stream, newton_iters=ni, eps=eps)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            S.ccd(ctrl, vel, pts, dt, hit, patch, pops, stream=stream, newton_iters=ni, eps=eps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        p, pp = patch.cpu().numpy(), pops.cpu().numpy()
        res[mode] = {"ms": ms, "points_per_s": n / (ms * 1e-3), "contact_fraction": float(np.mean(p >= 0)),
                     "no_result": int(np.sum(p < -1)), "pops_mean": float(pp.mean()), "pops_max": int(pp.max())}
        print(f"[bench] ccd {case.name} {mode}: {ms:.2f} ms, {n / ms / 1e3:.1f} M points/s, "
              f"pops mean {pp.mean():.2f} max {pp.max()}", file=sys.stderr, flush=True)
    return res


def render_cpu_baseline(width=512, height=512, spp=16, eps=1e-10, sample=200_000):
    """The oracle's ray casting rate (all host threads) on a seeded sample of
    the render section's rays, per scene and form."""
    from oracle import oracle as O, ray_oracle as R
    from paper_2312_14839_amd import workloads as W
    out = {"unit": "rays/s", "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
           "kind": "oracle", "sample": f"{sample} of the {width * height * spp} rays of each frame"}
    for sc in W.RENDER_SCENES:
        case = W.render_scene(sc)
        ctrl = R.bezier_grid(O.make_shell(case.n1, case.n2, case.dxi1, case.dxi2, case.young, case.poisson,
                                          case.thickness, case.density, periodic1=case.periodic1), case.ref)
        rays = W.camera_rays(sc, width, height, spp)
        idx = np.random.default_rng(41).choice(len(rays), min(sample, len(rays)), replace=False)
        for mode, ni in (("midpoint", 0), ("newton", 8)):
            t0 = time.perf_counter()
            R.ray_cast(ctrl, rays[idx], eps=eps, newton_iters=ni)
            out[f"{sc}_{mode}"] = len(idx) / (time.perf_counter() - t0)
        if sc != "plane":
            vel = R.bezier_grid(O.make_shell(case.n1, case.n2, case.dxi1, case.dxi2, case.young, case.poisson,
                                             case.thickness, case.density, periodic1=case.periodic1),
                                rigid_velocity(case))
            pts = ccd_points(sc, width, height, spp)[idx]
            for mode, ni in (("midpoint", 0), ("newton", 8)):
                t0 = time.perf_counter()
                R.ccd(ctrl, vel, pts, 0.5, eps=eps, newton_iters=ni)
                out[f"ccd_{sc}_{mode}"] = len(idx) / (time.perf_counter() - t0)
    return out


def cpu_baseline(budget_s=12.0, budget_1t=8.0):
    """Oracle patch energy + gradient + Hessian evaluations per second on a
    32x32-patch cylinder section (1024 patches): all host threads (the
    reported value), then one thread (OpenMP thread count set through the
    runtime the oracle library links)."""
    import ctypes
    from oracle import oracle as O
    from paper_2312_14839_amd import workloads as W
    c = W.case_cylinder(32, 32)
    s = O.shell_from_case(c)
    q = W.random_state(c, 1, 1e-4, 1e-3)

    def rate(budget, max_reps):
        reps, t0 = 0, time.perf_counter()
        while True:
            O.energy(s, q, c.ref)
            O.gradient(s, q, c.ref)
            O.matrix_blocks(s, q, c.ref, "hessian")
            reps += 1
            el = time.perf_counter() - t0
            if el > budget or reps >= max_reps:
                return reps, el

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    reps, el = rate(budget_s, 400)
    out = {"value": reps * c.patches / el, "unit": "patch E/grad/Hess evals/s", "cores": cores, "kind": "oracle",
           "sample": f"E+grad+Hess of the {c.patches} patches of a 32x32-patch cylinder section, {reps} reps, "
                     f"{el:.1f} s", "cpu_model": _cpu_model()}
    try:
        omp = ctypes.CDLL("libgomp.so.1")
        omp.omp_set_num_threads(1)
        r1, e1 = rate(budget_1t, 100)
        omp.omp_set_num_threads(cores)
        out["value_1thread"] = r1 * c.patches / e1
        out["sample_1thread"] = f"{r1} reps, {e1:.1f} s on one thread"
    except OSError:
        out["value_1thread"] = None
    return out


def oracle_newton_baseline(gpu_step1=None, cyl=True):
    """The oracle's implicit Newton step, timed on the host: the banded
    LDL^T Newton (the paper's solver class) on the 8x8 sheet and on step 1
    of the 30x30 twist, on all host threads and on one; the oracle's own
    block-Jacobi CG Newton on step 1 of the 256x256 cylinder (all threads
    only: about a minute), and the relative displacement error of the GPU's
    step-1 states (gpu_step1: {form: state}) against it."""
    import ctypes
    from oracle import oracle as O
    from paper_2312_14839_amd import workloads as W
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    try:
        omp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        omp = None
    out = {"unit": "ms per implicit step", "cores": cores, "kind": "oracle"}

    def step(case, solver, tol, threads):
        if omp is not None:
            omp.omp_set_num_threads(threads)
        s = O.shell_from_case(case)
        qp = case.presc(case.dt) if case.presc is not None else None
        t0 = time.perf_counter()
        rc, q1, _, st = O.newton_step(s, case.ref, case.fixed, case.dt, case.q0, case.v0, qp, solver=solver, **tol)
        ms = 1e3 * (time.perf_counter() - t0)
        if omp is not None:
            omp.omp_set_num_threads(cores)
        return rc, q1, st, ms

    for name, case, solver, tol in (
            ("sheet8x8_ldlt", W.case_small_sheet(), "ldlt", dict(newton_rtol=1e-10)),
            ("twist30x30_step1_ldlt", W.case_twist(30), "ldlt", dict(newton_rtol=1e-10))):
        rc, _, st, ms_all = step(case, solver, tol, cores)
        _, _, _, ms_one = step(case, solver, tol, 1) if omp is not None else (None, None, None, None)
        out[name] = {"ms": ms_all, "ms_1thread": ms_one, "status": rc, "newton_iters": st["newton_iters"]}
        print(f"[bench] oracle {name}: {ms_all:.0f} ms ({cores} threads), {ms_one} ms (1 thread)",
              file=sys.stderr, flush=True)
    if cyl:
        case = W.case_cylinder(256, 256)
        rc, q1, st, ms = step(case, "pcg", dict(newton_rtol=1e-10, pcg_rtol=1e-8), cores)
        res = {"ms": ms, "status": rc, "newton_iters": st["newton_iters"], "cg_iters": st["pcg_iters_total"]}
        for form, q in (gpu_step1 or {}).items():
            num = np.linalg.norm((q - q1)[:, 0:3])
            den = np.linalg.norm((q1 - case.q0)[:, 0:3])
            res[f"rel_disp_err_{form}_vs_oracle"] = float(num / den)
        out["cylinder256_step1_pcg"] = res
        print(f"[bench] oracle cylinder step 1 (PCG): {ms / 1e3:.1f} s, errors "
              f"{ {k: v for k, v in res.items() if k.startswith('rel_')} }", file=sys.stderr, flush=True)
    return out


def teardown():
    """Finish device work and release what the process holds on the
    device before the interpreter exits: contexts still referenced (closed
    by their finaliser), then torch's cached device memory."""
    import gc
    import torch
    torch.cuda.synchronize()
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cylinder", choices=["cylinder", "twist", "sheet", "batch"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-post-buckling", action="store_true")
    ap.add_argument("--no-pseudo", action="store_true")
    ap.add_argument("--no-kernels", action="store_true")
    ap.add_argument("--no-twist", action="store_true", help="skip the 200-step 30x30 twist section")
    ap.add_argument("--no-render", action="store_true", help="skip the ray--patch intersection section")
    ap.add_argument("--no-collision", action="store_true", help="skip the collision-handling section")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-sheet batch section")
    ap.add_argument("--no-loads", action="store_true", help="skip the pressure / point-constraint section")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="first run a plain device copy of MB megabytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU (asked for {args.gpus}); "
              "sharding across GPUs is designed but not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2312_14839_amd import shell as S
    if args.copy_probe:
        a = torch.ones(args.copy_probe * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    case, desc, tol = make_case(args.workload)
    if isinstance(case, list):
        case = Batch(case)
    stream = torch.cuda.current_stream().cuda_stream
    print(f"[bench] workload {case.name}: {case.patches} patches, {12 * case.nodes} DOF", file=sys.stderr, flush=True)
    wall, st64, tm64, tune64 = run_steps(case, S.SHELL_FP64, args.steps, args.warmup, stream, tol,
                                         not args.no_autotune)
    newton64 = sum(s["newton_iters"] for s in st64)
    # each Newton iteration of a shell evaluates every patch of that shell
    value = sum(s["patch_evals"] for s in st64) / wall
    ms_step = 1e3 * wall / args.steps
    print(f"[bench] fp64: {ms_step:.2f} ms/step, {newton64} Newton its, "
          f"{sum(s['pcg_iters_total'] for s in st64)} CG its", file=sys.stderr, flush=True)
    grp, roof = roofline(case, tm64, False, tune64)
    out = {
        "metric": METRIC, "value": value, "unit": "patch E/grad/Hess evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "patches": case.patches, "dof": 12 * case.nodes, "dt": case.dt,
                   "precision": "fp64", **tol},
        "newton_iters_per_step": newton64 / args.steps,
        "cg_iters_per_step": sum(s["pcg_iters_total"] for s in st64) / args.steps,
        "kernel_ms_fp64": {k: v for k, v in tm64["ms"].items()},
        "kernel_launches_fp64": tm64["launches"],
        "cg_layout": tune64,
        "roofline": roof,
    }
    if not args.no_mixed:
        wallm, stm, tmm, tunem = run_steps(case, S.SHELL_MIXED, args.steps, args.warmup, stream, tol,
                                           not args.no_autotune)
        newtonm = sum(s["newton_iters"] for s in stm)
        evalsm = sum(s["patch_evals"] for s in stm)
        nst = args.warmup + args.steps
        qa = qstate_after(case, S.SHELL_FP64, nst, stream, tol)
        qb = qstate_after(case, S.SHELL_MIXED, nst, stream, tol)
        ref = case.q0.reshape(-1, 12)
        err = np.linalg.norm((qb - qa)[:, 0:3]) / max(np.linalg.norm((qa - ref)[:, 0:3]), 1e-300)
        _, roofm = roofline(case, tmm, True, tunem)
        out["mixed"] = {"value": evalsm / wallm, "ms_per_step": 1e3 * wallm / args.steps,
                        "dtype": "f32 Hessian/CG + f64 residual", "rel_disp_err_vs_fp64": float(err),
                        "err_steps": nst, "newton_iters_per_step": newtonm / args.steps,
                        "cg_iters_per_step": sum(s["pcg_iters_total"] for s in stm) / args.steps,
                        "kernel_ms": tmm["ms"], "kernel_launches": tmm["launches"], "roofline": roofm}
        print(f"[bench] mixed: {1e3 * wallm / args.steps:.2f} ms/step, err {err:.2e}", file=sys.stderr, flush=True)
    if not args.no_kernels:
        out["kernels"] = kernels_section(case, stream)
        out["cg_phases"] = cg_phases_section(case, stream)
        out["hbm_achievable"] = hbm_achievable()
    if args.workload == "cylinder" and not args.no_post_buckling:
        out["post_buckling"] = post_buckling_section(stream)
    if args.workload == "cylinder" and not args.no_pseudo:
        out["hessian_variants"] = pseudo_hessian_section(stream)
    if args.workload == "cylinder" and not args.no_twist:
        out["twist"] = twist_section(stream)
    if args.workload == "cylinder" and not args.no_render:
        out["render"] = render_section(stream)
    if args.workload == "cylinder" and not args.no_collision:
        out["collision"] = collision_section(stream)
    if args.workload == "cylinder" and not args.no_loads:
        out["loads"] = loads_section(stream)
    if args.workload == "cylinder" and not args.no_batch:
        out["batch"] = batch_section(stream)
    if not args.no_learned:
        out["learned"] = learned_section(stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        gpu_step1 = None
        if args.workload == "cylinder":
            gpu_step1 = {"fp64": qstate_after(case, S.SHELL_FP64, 1, stream, tol)}
            if not args.no_mixed:
                gpu_step1["mixed"] = qstate_after(case, S.SHELL_MIXED, 1, stream, tol)
        out["cpu_baseline"]["newton_step"] = oracle_newton_baseline(gpu_step1, cyl=args.workload == "cylinder")
        if "render" in out:
            out["cpu_baseline"]["render"] = render_cpu_baseline()
    teardown()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
