"""Benchmark of the HOME-LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the 256^3 fully periodic decaying-turbulence configuration (seeded
divergence-free random field on |k| <= 8, max |u| = 0.1 cs, rho = 1,
tau = 0.51), advanced in both storage formats: the paper's 16-bit moments
(the headline value) and FP32 moments.  A step is one fluid pass over every
cell plus the boundary pass (empty here: no solids, all faces periodic).
Inputs are resident in HBM before the timed region; K steps are timed between
two device synchronisations with events on the stream the kernels run on.

Prints one JSON line: MLUPS (whole job), the roofline of the dominant kernel
(the fluid pass: algorithmic bytes per launch / mean launch time from HIP
events, against the 8 TB/s HBM peak; measured HBM traffic from rocprofv3
counters when a summary for the current kernel source is committed), its
VALU-issue roofline (measured wave instructions per launch / launch time,
against 614.4 G/s; the 16-bit pass is bound by it), the adjoint/forward
ratio, the obstacle channel and the 128-domain batch, and the CPU oracle timed
on the host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import faulthandler
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM peak, fp32 vs 16-bit moments; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
N = 256
TAU = 0.51
# fluid-pass tile height of the 256^3 legs and the channel: 0 lets each
# context time the heights (the default); a profiling run pins one so that its
# counters are taken on a known kernel
TILE_ROWS = 0
BYTES_PER_CELL = {"q16": 40, "fp32": 80}   # one state read + one state written
KERNEL_SOURCES = ["paper_2602_05295_amd/csrc/lbm_fluid.hip", "paper_2602_05295_amd/csrc/lbm_device.h",
                  "paper_2602_05295_amd/csrc/lbm_codec.h", "paper_2602_05295_amd/csrc/lbm_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fluid_256cubed_traffic.json")
VALU_FILE = os.path.join(ROOT, "profiles", "fluid_256cubed_valu.json")
VALU_PEAK_G = 256 * 4 * 2.4 / 4  # G wave64 VALU instructions per second


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profiled_rows(kernel_name: str) -> int:
    """Tile height of a profiled fluid-kernel name, fluid_kernel<FMT, ROWS, ...>."""
    m = re.search(r"fluid_kernel<\d+, (\d+),", kernel_name)
    return int(m.group(1)) if m else 0


def _hash_checked(path: str, fmt: str, key: str, rows: int):
    """The committed counter summary's `key` for `fmt`, or None when the file
    is missing, was taken on a different kernel source or on another tile
    height than the `rows` the timed context used."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or fmt not in t.get("formats", {}):
        return None
    f = t["formats"][fmt]
    if _profiled_rows(f.get("kernel", "")) != rows:
        return None
    return f[key]


def valu_roofline(fmt: str, kernel_ms: float, rows: int):
    """VALU-issue roofline of the fluid pass: measured wave instructions per
    launch (rocprofv3 SQ_INSTS_VALU) / mean launch time, against 256 CUs x 4
    SIMDs x 2.4 GHz / 4 cycles per wave64 VALU instruction (packed FP32 off)."""
    n = _hash_checked(VALU_FILE, fmt, "valu_instructions_per_launch", rows)
    if n is None:
        return None
    achieved = n / (kernel_ms * 1e-3) / 1e9
    return {"bound": "alu", "achieved": round(achieved, 1), "peak": VALU_PEAK_G, "unit": "G wave-instructions/s",
            "frac": round(achieved / VALU_PEAK_G, 4), "instructions_per_launch": n}


def measured_traffic(fmt: str, rows: int):
    """HBM bytes per fluid launch from the committed rocprofv3 counter summary,
    or None when it is missing or was taken on a different kernel source or
    tile height."""
    return _hash_checked(TRAFFIC_FILE, fmt, "hbm_bytes_per_launch", rows)


def copy_ceiling(nbytes=1 << 30, seconds=0.5):
    """The practical HBM ceiling: a plain device-to-device copy (torch's copy
    kernel) of nbytes, repeated for about `seconds`; bandwidth = bytes read +
    written / mean time of the last 50 copies, timed with events on the
    current stream."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        reps += 10
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(50):
        dst.copy_(src)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 50
    del src, dst
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    return {"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_copy": nbytes,
            "kernel": "torch copy_ (device to device)", "warm_copies": reps}


def workload():
    from paper_2602_05295_amd import workloads as W
    u = W.random_solenoidal(N, N, N, 8.0, 0.1 * W.CS, seed=0).astype(np.float32)
    rho = np.ones((N, N, N), np.float32)
    return rho, u


def open_format(fmt, rho_d, u_d, steps, warmup):
    """A 256^3 context of one format, set up for its timed leg: the field,
    the tile height timed, and the step sequences that the warm-up and the
    timed call replay captured.  The legs' contexts are all opened before
    any of them is timed, so that the timed legs follow one another with no
    host-side set-up in between (the GPU's clocks drop while the host works
    and take about 100 steps to come back)."""
    import torch
    from paper_2602_05295_amd.homelbm import HomeLBM
    stream = torch.cuda.current_stream()
    s = HomeLBM((N, N, N), TAU, fmt=fmt, stream=stream.cuda_stream)
    s.set_options(check_health=False, dither_mode=1, seed=0, tile_rows=TILE_ROWS)
    s.set_equilibrium(rho_d, u_d)
    s.prepare(warmup)
    s.prepare(steps)
    return s


def run_format(s, fmt, steps, warmup):
    """The timed leg on a context from open_format (left open: the caller
    closes it once every leg has run)."""
    import torch
    stream = torch.cuda.current_stream()
    s.step(warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    s.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    bad = s.check()
    # per-launch kernel time of the fluid pass (events around each launch)
    prof = s.profile_steps(min(steps, 200))
    state_bytes, _ = s.memory_bytes()
    rows = s.tile_rows
    cells = N ** 3
    fluid_ms = prof["fluid_ms"] / max(prof["fluid_launches"], 1)
    achieved = cells * BYTES_PER_CELL[fmt] / (fluid_ms * 1e-3) / 1e9
    return {
        "mlups": cells * steps / (ms * 1e-3) / 1e6,
        "ms_per_step": ms / steps,
        "wall_s": wall,
        "fluid_kernel_ms": fluid_ms,
        "achieved_GBs": achieved,
        "hbm_frac": achieved / HBM_PEAK_GBS,
        "state_bytes": state_bytes,
        "tile_rows": rows,
        "unhealthy_values": int(bad),
    }


def adjoint_ratio(n=128, steps=400, every=20):
    """(recompute + adjoint) / forward wall time of a checkpointed rollout on
    the 128^3 box with ~5% sphere obstacles (FP32, tau = 0.6); loss = L2 of
    the final velocity against a second seeded field."""
    import torch
    from paper_2602_05295_amd import workloads as W
    from paper_2602_05295_amd.adjoint import rollout
    from paper_2602_05295_amd.homelbm import HomeLBM
    mask = W.sphere_mask(n, n, n, phi=0.05, rmin=4.0, rmax=12.0, seed=0)
    u0 = torch.tensor(W.random_solenoidal(n, n, n, 4.0, 0.05, seed=0), dtype=torch.float32, device="cuda")
    tgt = torch.tensor(W.random_solenoidal(n, n, n, 4.0, 0.05, seed=1), dtype=torch.float32, device="cuda")
    fl = torch.tensor(mask == 0, dtype=torch.float32, device="cuda")
    with HomeLBM((n, n, n), 0.6, mask=mask) as s:
        s.set_options(check_health=False)
        u = u0.clone().requires_grad_(True)
        for rep in range(2):  # the first pass warms up
            u.grad = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = rollout(s, u, steps, every)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            vel = out[1:4] / out[0]
            loss = 0.5 * (((vel - tgt) ** 2).sum(0) * fl).sum()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            loss.backward()
            torch.cuda.synchronize()
            t3 = time.perf_counter()
        fwd, bwd = t1 - t0, t3 - t2
        # the forward alone, without checkpoint copies
        s.set_equilibrium(torch.ones((n, n, n), device="cuda"), u0)
        s.prepare(steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        plain = time.perf_counter() - t0
    return {"config": f"{n}^3 box, {float(mask.mean()):.3f} solid, FP32, tau 0.6, {steps} steps, checkpoint every {every}",
            "forward_s": round(fwd, 4), "backward_s": round(bwd, 4), "forward_plain_s": round(plain, 4),
            "ratio": round(bwd / plain, 3), "grad_finite": bool(torch.isfinite(u.grad).all())}


def channel(steps=20):
    """The 1000x400x400 obstacle channel in 16-bit moments: fluid + boundary
    passes per step (MLUPS over all cells) and the two kernels' times.  The
    fluid starts at rest and the inflow face (u = 0.08) drives it: an
    impulsive start at u = 0.08 everywhere takes the density behind the
    obstacles to 0.76 within 50 steps (FP32), below the 16-bit range."""
    import torch
    from paper_2602_05295_amd import workloads as W
    from paper_2602_05295_amd.homelbm import HomeLBM
    nx, ny, nz = 1000, 400, 400
    mask = W.channel_mask(nx, ny, nz, seed=0)
    u = torch.zeros((3, nz, ny, nx), dtype=torch.float32, device="cuda")
    rho = torch.ones((nz, ny, nx), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    with HomeLBM((nx, ny, nz), 0.52, mask=mask, fmt="q16", stream=stream.cuda_stream) as s:
        s.set_options(check_health=False, inflow=True, u_in=(0.08, 0.0, 0.0), tile_rows=TILE_ROWS)
        s.set_equilibrium(rho, u)
        del u, rho
        s.prepare(5)
        s.prepare(steps)
        s.step(5)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        s.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        prof = s.profile_steps(steps)
        nf, ns = s.boundary_counts()
        rows = s.tile_rows
        bad = s.check()
        # the same scene in the paper's mixed-precision pipeline (Sec. 5.3):
        # stream pass into FP32, link corrections with atomicAdd, requantize
        s.set_options(pipeline=1)
        s.step(3)
        torch.cuda.synchronize()
        ev0.record(stream)
        s.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_mixed = ev0.elapsed_time(ev1) / steps
        st = s.profile_stages(steps)
        mixed = {"ms_per_step": round(ms_mixed, 4),
                 "mlups": round(nx * ny * nz / (ms_mixed * 1e-3) / 1e6, 1),
                 "fluid_update_ms": round(st["fluid_ms"] / steps, 4),
                 "solid_correction_ms": round(st["boundary_ms"] / steps, 4),
                 "requantize_ms": round(st["requantize_ms"] / steps, 4),
                 "unhealthy_values": int(s.check())}
    cells = nx * ny * nz
    return {"config": "1000x400x400 channel, 16-bit, tau 0.52, inflow 0.08 into fluid at rest, 300 obstacles",
            "solid_fraction": round(float(mask.mean()), 4), "boundary_fluid_cells": nf, "boundary_solid_cells": ns,
            "mlups": round(cells / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "fluid_kernel_ms": round(prof["fluid_ms"] / prof["fluid_launches"], 4), "tile_rows": rows,
            "boundary_kernel_ms": round(prof["boundary_ms"] / max(prof["boundary_launches"], 1), 4),
            # the fluid pass's algorithmic bytes (one 16-bit state read and written, 40 B per cell)
            "fluid_GBs": round(cells * 40 / (prof["fluid_ms"] / prof["fluid_launches"] * 1e-3) / 1e9, 1),
            "fluid_hbm_frac": round(cells * 40 / (prof["fluid_ms"] / prof["fluid_launches"] * 1e-3) / 1e9
                                    / HBM_PEAK_GBS, 4),
            "unhealthy_values": int(bad),
            "paper_mixed_pipeline": mixed}


def channel_triangles(steps=10):
    """The paper's solid correction both ways on the obstacle channel built
    from triangle meshes (its ellipsoids and boxes tessellated, about 2.9 M
    triangles, the mask the lattice points inside them), 16-bit mixed
    pipeline, obstacles at rest (so both give the same step): per-link
    corrections over the voxel links (wall rule 1) against one thread per
    triangle sweeping its bounding box with link-triangle tests (wall rule 2,
    Alg. 3).  Stage times per step, and the one-off nearest-hit pass."""
    import torch
    from paper_2602_05295_amd import workloads as W
    from paper_2602_05295_amd.homelbm import HomeLBM
    nx, ny, nz = 1000, 400, 400
    mask, tris, ids = W.channel_mesh(nx, ny, nz, seed=0)
    stream = torch.cuda.current_stream()
    out = {"triangles": int(tris.shape[0]), "solid_fraction": round(float((mask != 0).mean()), 4)}
    with HomeLBM((nx, ny, nz), 0.52, mask=mask, fmt="q16", stream=stream.cuda_stream) as s:
        s.set_triangles(tris, ids)
        u = torch.zeros((3, nz, ny, nx), dtype=torch.float32, device="cuda")
        s.set_options(check_health=False, inflow=True, u_in=(0.08, 0.0, 0.0), pipeline=1, wall_rule=1)
        s.set_equilibrium(torch.ones((nz, ny, nx), dtype=torch.float32, device="cuda"), u)
        del u
        for rule in (1, 2):
            s.set_options(wall_rule=rule)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(1)  # rule 2: builds the nearest-hit table first
            torch.cuda.synchronize()
            first = time.perf_counter() - t0
            st = s.profile_stages(steps)
            out["per_link" if rule == 1 else "per_triangle"] = {
                "ms_per_step": round((st["fluid_ms"] + st["boundary_ms"] + st["requantize_ms"]) / steps, 4),
                "fluid_update_ms": round(st["fluid_ms"] / steps, 4),
                "solid_correction_ms": round(st["boundary_ms"] / steps, 4),
                "requantize_ms": round(st["requantize_ms"] / steps, 4),
                "first_step_s": round(first, 3)}
        out["unhealthy_values"] = int(s.check())
    return out


def bit_allocation(steps=2000, n=(128, 128, 32), tau=0.55):
    """The b_rho_u / b_S study on a 3D double shear layer (the paper's
    double-layer vortex, made three-dimensional by a z modulation of the
    perturbation): the same run in FP32, 16-bit and each packed allocation;
    relative L2 error of the velocity field against the FP32 run after
    `steps` steps, bytes per cell, and the fluid pass's time per launch on
    the 256^3 decaying-turbulence field for each format."""
    import torch
    from paper_2602_05295_amd import workloads as W
    from paper_2602_05295_amd.homelbm import HomeLBM, BITS, FORMATS, raw_planes
    nx, ny, nz = n
    rho, u = W.double_shear_layer(nx, ny, nz, seed=0)
    rho_d = torch.from_numpy(rho.astype(np.float32)).cuda()
    u_d = torch.from_numpy(u.astype(np.float32)).cuda()
    names = ["fp32", "q16", "p16_15", "p15_14", "p14_13", "p13_12", "p12_11"]
    seeds = (0, 1, 2, 3)

    def velocity(name, seed):
        with HomeLBM((nx, ny, nz), tau, fmt=name) as s:
            s.set_options(check_health=False, dither_mode=1, seed=seed)
            s.set_equilibrium(rho_d, u_d)
            s.step(steps)
            m = s.get_moments()
        return m[1:4] / m[0]

    ref = velocity("fp32", 0)
    errs = {name: [float(np.linalg.norm(velocity(name, sd) - ref) / np.linalg.norm(ref)) for sd in seeds]
            for name in names[1:]}
    rows = {}
    rho2, u2 = workload()
    r2 = torch.from_numpy(rho2).cuda()
    v2 = torch.from_numpy(u2).cuda()
    for name in names:
        fmt = FORMATS[name]
        with HomeLBM((N, N, N), TAU, fmt=name) as s:
            s.set_options(check_health=False, dither_mode=1, seed=0)
            s.set_equilibrium(r2, v2)
            s.step(10)
            prof = s.profile_steps(50)
        e = errs.get(name, [0.0])
        rows[name] = {"bits": None if name == "fp32" else "%d/%d" % BITS[fmt],
                      "bytes_per_cell": 4 * raw_planes(fmt), "l2_rel_error_vs_fp32": round(float(np.mean(e)), 7),
                      "l2_rel_error_min_max": [round(min(e), 7), round(max(e), 7)],
                      "fluid_kernel_ms_256cubed": round(prof["fluid_ms"] / prof["fluid_launches"], 4)}
    return {"config": "double shear layer %dx%dx%d, U0 0.04, tau %g, %d steps, error = mean over dither seeds %s "
                      "of the relative L2 velocity difference from the FP32 run; kernel times on 256^3"
                      % (nx, ny, nz, tau, steps, list(seeds)),
            "formats": rows}


def batched(steps=200):
    """128 periodic domains of seeded sizes 24^3..96^3 with sphere obstacles
    (0-10% solid) and tau in [0.52, 0.8], 16-bit moments: the autotuned work
    split, then `steps` steps replayed from one captured HIP graph."""
    import torch
    from paper_2602_05295_amd import workloads as W
    from paper_2602_05295_amd.homelbm import HomeLBMBatch
    doms = W.batched_domains(128, seed=0)
    fields = [W.batched_domain_fields(d) for d in doms]
    dims = [d["dims"] for d in doms]
    stream = torch.cuda.current_stream()
    with HomeLBMBatch(dims, [d["tau"] for d in doms], [f[0] for f in fields], fmt="q16",
                      stream=stream.cuda_stream) as b:
        b.set_options(check_health=False)
        for k, (mask, u) in enumerate(fields):
            b.set_equilibrium(k, np.ones(mask.shape, np.float32), u.astype(np.float32))
        tuning = b.tune()
        b.step(steps)  # captures the graph and warms up
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        b.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        prof = b.profile_steps(20)
        nf, ns = b.boundary_counts()
        bad = b.check()
        cells = b.cells()
    fl = prof["fluid_ms"] / prof["steps"]
    return {"config": "128 domains 24..96 per axis, 0-10% spheres, tau 0.52-0.8, 16-bit, one graph of "
                      f"{steps} steps", "cells": int(cells), "boundary_fluid_cells": nf, "boundary_solid_cells": ns,
            "mlups": round(cells / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "fluid_kernel_ms": round(fl, 4), "boundary_kernel_ms": round(prof["boundary_ms"] / prof["steps"], 4),
            "fluid_GBs": round(cells * 40 / (fl * 1e-3) / 1e9, 1),
            "tuning": {k: tuning[k] for k in ("block", "wg_per_cu", "workgroups", "segments", "balance")},
            "unhealthy_values": int(bad)}


def host_threads() -> int:
    """Host threads the oracle may use: OMP_NUM_THREADS when set (the share of
    the host given to this process), else the CPUs this process may run on."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    if n <= 0:
        try:
            n = len(os.sched_getaffinity(0))
        except (AttributeError, OSError):
            n = os.cpu_count() or 1
    return max(1, n)


def physical_cores() -> int | None:
    """Physical cores of the host (sockets x cores per socket), from lscpu."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    vals = {}
    for line in out.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    try:
        return int(vals["Socket(s)"]) * int(vals["Core(s) per socket"])
    except (KeyError, ValueError):
        return None


def _timed(fn, cells_per_call, calls):
    t0 = time.perf_counter()
    for _ in range(calls):
        fn()
    dt = time.perf_counter() - t0
    return {"mlups": round(cells_per_call * calls / dt / 1e6, 3), "seconds": round(dt, 2)}


def cpu_baseline(u, gpu=None, channel_mask=None):
    """The FP64 oracle on the host, untuned, on every configuration: the
    headline (16-bit step of the 256^3 field) on all host threads the process
    may use and on one thread, and per configuration a bounded sample on both
    (about 30 s of host time in all).  gpu: the GPU's MLUPS per configuration,
    for the ratios."""
    import oracle
    from paper_2602_05295_amd import workloads as W
    gpu = gpu or {}
    nt = host_threads()
    per = {}

    def note(what):
        print(f"[bench] oracle: {what}", file=sys.stderr, flush=True)

    # 256^3 decaying turbulence, 16-bit (the headline): 3 steps on nt threads;
    # one thread: one step of a 256 x 256 x 16 slab of the same field
    m = oracle.equilibrium_moments(np.ones((N, N, N)), u.astype(np.float64))
    P = oracle.make_params((N, N, N), TAU)
    w = oracle.q16_encode(m, t=0, seed=0, mode=1)
    del m
    head = _timed(lambda: oracle.q16_step(P, w, t=1, seed=0, mode=1, nthreads=nt), N ** 3, 3)
    slab = np.ascontiguousarray(w[:, :16])
    Ps = oracle.make_params((N, N, 16), TAU)
    one = _timed(lambda: oracle.q16_step(Ps, slab, t=1, seed=0, mode=1, nthreads=1), N * N * 16, 1)
    note("turbulence_256_q16")
    per["turbulence_256_q16"] = {"threads": nt, "mlups": head["mlups"], "mlups_1_thread": one["mlups"],
                                 "sample": "3 steps of 256^3; 1 thread: 1 step of a 256x256x16 slab",
                                 "gpu_mlups": gpu.get("q16")}
    # FP32-format step of the same field (FP64 arithmetic either way)
    m = oracle.equilibrium_moments(np.ones((N, N, N)), u.astype(np.float64))
    f64 = _timed(lambda: oracle.step(P, m, nthreads=nt), N ** 3, 2)
    ms = np.ascontiguousarray(m[:, :16])
    f1 = _timed(lambda: oracle.step(Ps, ms, nthreads=1), N * N * 16, 1)
    del m, ms
    note("turbulence_256_fp32")
    per["turbulence_256_fp32"] = {"threads": nt, "mlups": f64["mlups"], "mlups_1_thread": f1["mlups"],
                                  "sample": "2 steps of 256^3; 1 thread: 1 step of a 256x256x16 slab",
                                  "gpu_mlups": gpu.get("fp32")}
    # 32^3 Taylor-Green, FP64 moments: 100 steps / 20 steps on one thread
    rho, uu = W.taylor_green_2d(32, 32, 32, 0.05)[:2]
    mt = oracle.equilibrium_moments(rho, uu)
    Pt = oracle.make_params((32, 32, 32), 0.6)
    a = _timed(lambda: oracle.step(Pt, mt, nthreads=nt), 32 ** 3, 100)
    b = _timed(lambda: oracle.step(Pt, mt, nthreads=1), 32 ** 3, 20)
    note("taylor_green_32")
    per["taylor_green_32"] = {"threads": nt, "mlups": a["mlups"], "mlups_1_thread": b["mlups"],
                              "sample": "100 steps; 1 thread: 20 steps", "gpu_mlups": None}
    # 1000x400x400 channel, 16-bit with faces and obstacles: a 1000x100x50
    # block of the real obstacle mask (y, z periodic within the block)
    if channel_mask is None:
        channel_mask = W.channel_mask(1000, 400, 400, seed=0)
    blk = np.ascontiguousarray(channel_mask[:50, :100, :])
    blk[:, :, :3] = 0
    blk[:, :, -3:] = 0
    nb = blk.size
    mc = oracle.equilibrium_moments(np.ones(blk.shape), np.zeros((3,) + blk.shape))
    Pc = oracle.make_params((1000, 100, 50), 0.52, inflow=True, u_in=(0.08, 0.0, 0.0))
    wc = oracle.q16_encode(mc, blk, t=0, seed=0, mode=1)
    a = _timed(lambda: oracle.q16_step(Pc, wc, blk, t=1, seed=0, mode=1, nthreads=nt), nb, 2)
    wc1 = np.ascontiguousarray(wc[:, :10])
    Pc1 = oracle.make_params((1000, 100, 10), 0.52, inflow=True, u_in=(0.08, 0.0, 0.0))
    b = _timed(lambda: oracle.q16_step(Pc1, wc1, np.ascontiguousarray(blk[:10]), t=1, seed=0, mode=1, nthreads=1),
               wc1[0].size, 1)
    note("channel_1000x400x400")
    per["channel_1000x400x400"] = {"threads": nt, "mlups": a["mlups"], "mlups_1_thread": b["mlups"],
                                   "sample": "2 steps of a 1000x100x50 block of the obstacle mask; "
                                             "1 thread: 1 step of 1000x100x10", "gpu_mlups": gpu.get("channel")}
    # 128-domain batch: one 16-bit step of every domain / of the first 8 on one thread
    doms = W.batched_domains(128, seed=0)
    cells = 0
    t_all = 0.0
    t_one = 0.0
    cells_one = 0
    for k, d in enumerate(doms):
        mk, uk = W.batched_domain_fields(d)
        mm = oracle.equilibrium_moments(np.ones(mk.shape), uk.astype(np.float64))
        Pk = oracle.make_params(d["dims"], d["tau"])
        wk = oracle.q16_encode(mm, mk, t=0, seed=0, mode=1)
        r = _timed(lambda: oracle.q16_step(Pk, wk, mk, t=1, seed=0, mode=1, nthreads=nt), mk.size, 1)
        t_all += r["seconds"]
        cells += mk.size
        if k < 8:
            r1 = _timed(lambda: oracle.q16_step(Pk, wk, mk, t=1, seed=0, mode=1, nthreads=1), mk.size, 1)
            t_one += r1["seconds"]
            cells_one += mk.size
    note("batched_128_domains")
    per["batched_128_domains"] = {"threads": nt, "mlups": round(cells / t_all / 1e6, 3),
                                  "mlups_1_thread": round(cells_one / t_one / 1e6, 3),
                                  "sample": "1 step of all 128 domains; 1 thread: 1 step of the first 8",
                                  "gpu_mlups": gpu.get("batched")}
    # 128^3 adjoint box: forward and adjoint steps (FP64)
    n5 = 128
    mask5 = W.sphere_mask(n5, n5, n5, phi=0.05, rmin=4.0, rmax=12.0, seed=0)
    u5 = W.random_solenoidal(n5, n5, n5, 4.0, 0.05, seed=0)
    m5 = oracle.equilibrium_moments(np.ones((n5, n5, n5)), u5)
    P5 = oracle.make_params((n5, n5, n5), 0.6)
    lam = np.random.default_rng(0).standard_normal(m5.shape)
    fwd = _timed(lambda: oracle.step(P5, m5, mask5, nthreads=nt), n5 ** 3, 2)
    adj = _timed(lambda: oracle.adjoint_step(P5, m5, lam, mask5), n5 ** 3, 1)
    note("adjoint_128")
    per["adjoint_128"] = {"threads": nt, "forward_mlups": fwd["mlups"], "adjoint_mlups": adj["mlups"],
                          "sample": "2 forward steps and 1 adjoint step of the 128^3 box",
                          "gpu_forward_mlups": gpu.get("adjoint_forward")}
    for v in per.values():
        g = v.get("gpu_mlups")
        if g:
            v["gpu_over_oracle"] = round(g / v["mlups"], 1)
    return {"value": head["mlups"], "unit": "MLUPS", "cores": nt, "kind": "oracle",
            "sample": f"3 FP64-oracle 16-bit steps (decode, step, encode) of the full {N}^3 field, "
                      f"{head['seconds']:.1f} s on {nt} host threads",
            "single_thread": {"value": one["mlups"], "unit": "MLUPS",
                              "sample": "1 step of a 256x256x16 slab of the same field on 1 thread"},
            "cpu": host_cpu(), "physical_cores": physical_cores(), "logical_cpus": os.cpu_count(),
            "per_config": per}


def host_cpu() -> str:
    """The host's CPU model, as /proc/cpuinfo names it."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    faulthandler.enable()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--formats", default="q16,fp32", help="storage formats to run (the headline value is q16)")
    ap.add_argument("--no-extras", action="store_true", help="skip the adjoint ratio and the channel run")
    ap.add_argument("--only", choices=["adjoint", "channel", "triangles", "batched", "bits"], default=None,
                    help="run only this extra workload and print its JSON object (for profiling)")
    ap.add_argument("--extra-steps", type=int, default=None, help="steps of the --only workload")
    ap.add_argument("--no-copy-ceiling", action="store_true",
                    help="skip the plain-copy ceiling (and its device warm-up) before the timed legs")
    ap.add_argument("--tile-rows", type=int, default=0, choices=[0, 8, 10, 12, 13],
                    help="fluid-pass tile height of the 256^3 legs and the channel (0: timed per context)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB three times (the reference kernel that "
                         "scales hardware byte counters)")
    args = ap.parse_args()
    global TILE_ROWS
    TILE_ROWS = args.tile_rows
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 copies of {nbytes} bytes", file=sys.stderr, flush=True)
        del src, dst
    if args.only is not None:
        fn = {"adjoint": adjoint_ratio, "channel": channel, "triangles": channel_triangles, "batched": batched,
              "bits": bit_allocation}[args.only]
        kw = {} if args.extra_steps is None else {"steps": args.extra_steps}
        print(json.dumps(fn(**kw)), flush=True)
        return
    print(f"[bench] device {torch.cuda.get_device_name(0)}; building the {N}^3 field", file=sys.stderr, flush=True)
    rho, u = workload()
    rho_d = torch.from_numpy(rho).cuda()
    u_d = torch.from_numpy(u).cuda()
    extras = {}
    if not args.no_extras:
        print("[bench] adjoint/forward ratio (128^3, 400 steps)", file=sys.stderr, flush=True)
        extras["adjoint"] = adjoint_ratio()
        print(f"[bench] {extras['adjoint']}", file=sys.stderr, flush=True)
    # the headline format runs last; every format's context is set up first
    fmts = args.formats.split(",")
    fmts = [f for f in fmts if f != "q16"] + [f for f in fmts if f == "q16"]
    print("[bench] setting up the 256^3 contexts", file=sys.stderr, flush=True)
    ctxs = {fmt: open_format(fmt, rho_d, u_d, args.steps, args.warmup) for fmt in fmts}
    # the plain-copy ceiling: the practical HBM bound, reported beside the
    # roofline; it also keeps the GPU busy up to the first timed leg
    print("[bench] plain device copy", file=sys.stderr, flush=True)
    ceiling = None if args.no_copy_ceiling else copy_ceiling()
    if ceiling:
        print(f"[bench] copy: {ceiling['GBs']:.0f} GB/s", file=sys.stderr, flush=True)
    res = {}
    for fmt in fmts:
        res[fmt] = run_format(ctxs[fmt], fmt, args.steps, args.warmup)
        print(f"[bench] {fmt}: {res[fmt]['mlups']:.0f} MLUPS, fluid kernel {res[fmt]['fluid_kernel_ms']:.4f} ms, "
              f"{res[fmt]['achieved_GBs']:.0f} GB/s", file=sys.stderr, flush=True)
    for c in ctxs.values():
        c.close()
    if not args.no_extras:
        print("[bench] 1000x400x400 channel", file=sys.stderr, flush=True)
        extras["channel"] = channel()
        print(f"[bench] {extras['channel']}", file=sys.stderr, flush=True)
        print("[bench] channel with triangle meshes: per-link and per-triangle solid correction",
              file=sys.stderr, flush=True)
        extras["triangles"] = channel_triangles()
        print(f"[bench] {extras['triangles']}", file=sys.stderr, flush=True)
        print("[bench] 128-domain batch", file=sys.stderr, flush=True)
        extras["batched"] = batched()
        print(f"[bench] {extras['batched']}", file=sys.stderr, flush=True)
        print("[bench] bit allocation (double shear layer)", file=sys.stderr, flush=True)
        extras["bits"] = bit_allocation()
        print(f"[bench] {extras['bits']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
    gpu_rates = {k: round(v["mlups"], 1) for k, v in res.items()}
    if "channel" in extras:
        gpu_rates["channel"] = extras["channel"]["mlups"]
    if "batched" in extras:
        gpu_rates["batched"] = extras["batched"]["mlups"]
    if "adjoint" in extras:
        gpu_rates["adjoint_forward"] = round(128 ** 3 * 400 / extras["adjoint"]["forward_plain_s"] / 1e6, 1)
    cpu = None if args.no_cpu_baseline else cpu_baseline(u, gpu_rates)
    if "q16" not in res or "fp32" not in res:
        print(json.dumps({k: v for k, v in res.items()}), flush=True)
        return
    q = res["q16"]
    traffic = measured_traffic("q16", q["tile_rows"])
    traffic32 = measured_traffic("fp32", res["fp32"]["tile_rows"])
    line = {
        "metric": METRIC,
        "value": round(q["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(q["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "decaying turbulence 256^3 periodic, D3Q27 HOME-LBM, 16-bit moments",
                   "grid": [N, N, N], "tau": TAU, "moments": "q16", "field": "solenoidal |k|<=8, max|u|=0.1cs",
                   "dither": "per step"},
        "roofline": {"bound": "hbm", "achieved": round(q["achieved_GBs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(q["hbm_frac"], 4),
                     "traffic": None if traffic is None else round(traffic / (q["fluid_kernel_ms"] * 1e-3) / 1e9, 1),
                     "traffic_bytes_per_launch": traffic, "algorithmic_bytes_per_launch": N ** 3 * BYTES_PER_CELL["q16"],
                     "kernel": f"fluid_kernel<Q16, {q['tile_rows']} rows>", "bytes_per_cell": BYTES_PER_CELL["q16"]},
        "roofline_valu": valu_roofline("q16", q["fluid_kernel_ms"], q["tile_rows"]),
        "copy_ceiling": None if ceiling is None else dict(ceiling, fluid_frac_of_copy=round(q["achieved_GBs"] / ceiling["GBs"], 4)),
        "fp32": {"value": round(res["fp32"]["mlups"], 1), "unit": "MLUPS",
                 "ms_per_step": round(res["fp32"]["ms_per_step"], 5),
                 "roofline": {"bound": "hbm", "achieved": round(res["fp32"]["achieved_GBs"], 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(res["fp32"]["hbm_frac"], 4),
                              "traffic": None if traffic32 is None else
                              round(traffic32 / (res["fp32"]["fluid_kernel_ms"] * 1e-3) / 1e9, 1),
                              "traffic_bytes_per_launch": traffic32,
                              "kernel": f"fluid_kernel<F32, {res['fp32']['tile_rows']} rows>",
                              "bytes_per_cell": BYTES_PER_CELL["fp32"]},
                 "roofline_valu": valu_roofline("fp32", res["fp32"]["fluid_kernel_ms"], res["fp32"]["tile_rows"])},
        "memory_ratio_q16_fp32": res["q16"]["state_bytes"] / res["fp32"]["state_bytes"],
        "adjoint_forward_ratio": extras.get("adjoint", {}).get("ratio"),
        "adjoint": extras.get("adjoint"),
        "channel_1000x400x400": extras.get("channel"),
        "solid_correction_channel_meshes": extras.get("triangles"),
        "batched_128_domains": extras.get("batched"),
        "bit_allocation": extras.get("bits"),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
