"""Throughput of the granule hot path on one MI355X.

One step = one sand sub-step (Alg. 2) through the C ABI (gic_step): cell
sort, reorder, G2P, drag, contact, integration and P2G, on the c3 workload
(dam-break column, 4,194,304 granules, 256x128x128 grid), FP32 form; the
plain FP64 GPU path is timed the same way.  Inputs are resident in HBM
before timing.

Prints ONE JSON line (rank 0, N=1):
  value         granule-steps/s of the FP32 form (whole step)
  fp64_value    granule-steps/s of the plain FP64 path
  roofline      dominant kernel: algorithmic bytes per launch / its average
                duration from HIP events recorded between the step's stages on
                the step's own stream, vs 8 TB/s
  fp32_error    the FP32 form's error against the plain FP64 path, per output
  c2, c5        the polydisperse moving bed (262,144 granules, 100 steps) and
                the large bed (16,777,216 granules, 20 steps), per-stage GB/s
  cpu_baseline  the FP64 CPU oracle on this host's cores, bounded sample,
                one thread and all threads

    python bench.py [--steps K] [--warmup W] [--workload c3] [--no-cpu] ...
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-coupled", action="store_true")
    ap.add_argument("--no-capillary", action="store_true")
    ap.add_argument("--no-idp", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (read 1 GiB, write 1 GiB) three times, "
                         "to scale the HBM byte counters of a profiler pass")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes per granule (and per touched grid node) of each kernel of
# the step: the arrays the method itself must read and write once, neighbour
# re-reads and scratch excluded.  B = size of the real type.
def stage_bytes(stage, n, nodes, real_bytes, G=0, assembled=False, tile_bytes=0):
    B = real_bytes
    if stage == "assemble":
        # the stored tiles read once, and each node that holds a value written
        # once (four int64 channels); the zeros elsewhere stay from the step
        # before
        return tile_bytes + 32 * nodes
    per = {
        "sort": 24 + 4 + 4,                          # read x, write key, write order
        "gather_g2p_drag": 4 + 2 * (24 + 24 + 8 + 4) + 3 * B,  # order; gather + write x, v, r, id; write F_d
        "contact": 24 + 24 + 8 + 3 * B,              # read x, v, r; write F_c
        "integrate_p2g": 8 + 3 * B + 3 * B + 2 * (24 + 24),  # read r, F_c, F_d; read + write x, v
    }[stage]
    # node reads / writes; with assembled grids the tile kernel writes no grid
    grid = {"gather_g2p_drag": 3 * B + 8, "integrate_p2g": 0 if assembled else 8 + 24}.get(stage, 0)
    return per * n + grid * nodes


# The remaining interphase forces: the fluid gather also reads grad p and the
# fluid acceleration at each node; the exchange deposit reads x, r, F_c, F_fluid
# per granule and adds three int64 components per touched node.
def coupled_bytes(stage, n, nodes, real_bytes):
    B = real_bytes
    if stage == "gather_g2p_fluid":
        return (4 + 2 * (24 + 24 + 8 + 4) + 3 * B) * n + (3 * B + 8 + 6 * B) * nodes
    if stage == "exchange_p2g":
        return (24 + 8 + 3 * B + 3 * B) * n + 24 * nodes
    return stage_bytes(stage, n, nodes, real_bytes)


# Contact with liquid bridges (FP32 form): the dry contact's x, v, r and F_c
# plus the moisture ratio and the held water (wet mass) of each granule.
CAPILLARY_BYTES_PER_GRANULE = 24 + 24 + 8 + 3 * 4 + 4 + 8


def time_steps(sim, steps, warmup):
    """K whole steps (gic_step) between two HIP events on the step's stream,
    after W warm-up steps; also the neighbour-list builds during the K."""
    import torch
    for _ in range(warmup):
        sim.step()
    torch.cuda.synchronize()
    b0 = sim.ctx.neighbour_builds()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    sim.step(steps)
    end.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return start.elapsed_time(end) / 1e3, t1 - t0, sim.ctx.neighbour_builds() - b0


STAGE_KEYS = {"sort": "sort", "gather": "gather_g2p_drag", "contact": "contact", "exchange": "exchange_p2g",
              "grid_clear": "grid_clear", "integrate_p2g": "integrate_p2g", "assemble": "assemble"}


def time_stages(sim, steps, sand_dt=None, **sand):
    """Per-stage times of the step itself: the library records HIP events on
    the step's stream between its stages (gic_stage_timing) over `steps`
    further steps (or sand steps of length sand_dt); mean seconds per
    (sub-)step of each stage."""
    ctx = sim.ctx
    ctx.stage_timing(steps * 64)
    for _ in range(steps):
        if sand_dt is None:
            sim.step()
        else:
            sim.sand_step(sand_dt, **sand)
    ms, k = ctx.stage_times()
    ctx.stage_timing(0)
    out = {STAGE_KEYS[key]: v / 1e3 / max(k, 1) for key, v in ms.items()}
    if sand_dt is None:
        out.pop("exchange_p2g")
    else:
        out["gather_g2p_fluid"] = out.pop("gather_g2p_drag")
    return out, k


# Kernels whose time is one launch of one kernel per (sub-)step (the sort is
# a sequence of kernels; the contact stage is the neighbour-list kernel plus
# the list build, which returns at once when the list is kept; the assembly
# of the grids from the brick tiles is followed by the small deposit of the
# granules whose stencil left their tile, so it is priced beside them but
# not taken as the dominant kernel).
SINGLE_KERNEL_STAGES = ("gather_g2p_drag", "contact", "integrate_p2g")


def dominant_roofline(stages, n, nodes, real_bytes, workload, G):
    dom = max(SINGLE_KERNEL_STAGES, key=lambda k: stages[k])
    abytes = stage_bytes(dom, n, nodes, real_bytes, G, stages.get("assemble", 0.0) > 0.0)
    ach = abytes / stages[dom] / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": stored_traffic(dom, workload), "algorithmic_bytes": abytes}


def stored_tile_bytes(d):
    """Bytes of the stored P2G tiles of the bed d (its initial positions):
    one tile of four int64 channels per occupied brick of 4x4x4 cells, E
    nodes an edge (4 cell / dx + 2 when that is an integer, else its ceiling
    + 3)."""
    p = d["params"]
    m4 = 4.0 * p["cell"] / p["dx"]
    E = int(round(m4)) + 2 if abs(m4 - round(m4)) < 1e-9 * max(round(m4), 1.0) else int(np.ceil(m4)) + 3
    nc = np.array(p["nc"], dtype=np.int64)
    c = np.clip(np.floor(d["x"] / p["cell"]).astype(np.int64), 0, (nc - 1)[:, None])
    b = c // 4
    nb = (nc + 3) // 4
    occupied = np.unique((b[2] * nb[1] + b[1]) * nb[0] + b[0]).size
    return occupied * 4 * E ** 3 * 8


def stage_rooflines(stages, n, nodes, real_bytes, G, tile_bytes=0):
    """Algorithmic GB/s and fraction of the HBM peak of each single-kernel
    stage, and of the grid assembly when the step has one."""
    out = {}
    assembled = stages.get("assemble", 0.0) > 0.0
    for k in SINGLE_KERNEL_STAGES + (("assemble",) if assembled else ()):
        ab = stage_bytes(k, n, nodes, real_bytes, G, assembled, tile_bytes)
        out[k] = {"ms": round(stages[k] * 1e3, 4), "algorithmic_bytes": ab,
                  "GB_s": round(ab / stages[k] / 1e9, 1), "frac": round(ab / stages[k] / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def fp32_error(d, rmax):
    """Error of the FP32 form against the plain FP64 path (itself within
    1e-12 of the FP64 oracle in the parity tests) after one step from the
    same state, per output and per granule: max and 99th percentile of
      F_c  |dF_c| / (|F_c| + m |g|)     F_d  |dF_d| / (beta (|u_at| + |v|))
      u_at |du| / (|u_at| + max|u|)     alpha_f |d alpha_f| (a fraction)
      v    |dv| / (|v| + dt (|F_c| + |F_d| + m |g|) / m)
      x    |dx| / (dt times the v scale)
    with the FP64 values on the right."""
    import torch
    from paper_2504_00745_amd import gic
    cfg = d["params"]
    outs = {}
    for prec in ("fp32", "fp64"):
        sim = gic.Simulator(cfg, d["x"], d["v"], d["r"], d["u"], prec, r_max=rmax)
        gic.gic_step(sim.ctx, sim.cur, sim.nxt, sim.u, sim.alpha, sim.mom, sim.scratch)
        s = sim.scratch
        ids = sim.nxt["id"].long()
        n = ids.numel()

        def unsort(t, comps):
            o = torch.empty(comps, n, dtype=torch.float64, device="cuda")
            o[:, ids] = t.view(comps, n).double()
            return o
        outs[prec] = dict(Fc=unsort(s["f_contact"], 3), Fd=unsort(s["f_drag"], 3), uat=unsort(s["u_at"], 3),
                          af=unsort(s["alpha_f"], 1)[0], v=unsort(sim.nxt["v"], 3), x=unsort(sim.nxt["x"], 3))
        del sim
        torch.cuda.empty_cache()
    a, b = outs["fp32"], outs["fp64"]
    r = torch.as_tensor(d["r"], device="cuda")
    v0 = torch.as_tensor(d["v"], device="cuda")
    m = cfg["rho_s"] * (4.0 / 3.0) * np.pi * r ** 3
    g = float(np.linalg.norm(cfg["g"]))
    beta = cfg["c_drag"] * 6.0 * np.pi * cfg["eta_f"] * r
    nrm = lambda t: torch.linalg.norm(t, dim=0)
    umax = float(np.abs(d["u"]).max())
    vscale = nrm(b["v"]) + cfg["dt"] * (nrm(b["Fc"]) + nrm(b["Fd"]) + m * g) / m
    rel = {"F_c": nrm(a["Fc"] - b["Fc"]) / (nrm(b["Fc"]) + m * g + 1e-300),
           "F_d": nrm(a["Fd"] - b["Fd"]) / (beta * (nrm(b["uat"]) + nrm(v0)) + 1e-300),
           "u_at": nrm(a["uat"] - b["uat"]) / (nrm(b["uat"]) + umax + 1e-300),
           "alpha_f": (a["af"] - b["af"]).abs(),
           "v": nrm(a["v"] - b["v"]) / (vscale + 1e-300),
           "x": nrm(a["x"] - b["x"]) / (cfg["dt"] * vscale + 1e-300)}
    return {k: {"max": float(t.max()), "p99": float(torch.quantile(t[::max(1, t.numel() // 1000000)], 0.99))}
            for k, t in rel.items()}


def run_leg(name, steps, warmup, with_fp64=False):
    """Another workload as its own leg: whole FP32 steps (and FP64 if asked)
    timed with events, the stage times and each single-kernel stage's
    algorithmic GB/s."""
    import torch
    from paper_2504_00745_amd import gic, workloads as wl
    d = wl.make(name)
    n = d["x"].shape[1]
    rmax = float(d["r"].max())
    res = {"workload": WORKLOAD_TEXT[name](d), "granules": n, "steps": steps}
    for prec in (["fp32", "fp64"] if with_fp64 else ["fp32"]):
        sim = gic.Simulator(d["params"], d["x"], d["v"], d["r"], d["u"], prec, r_max=rmax)
        t, _, builds = time_steps(sim, steps, warmup)
        stages, k = time_stages(sim, min(steps, 10))
        nodes = touched_nodes(sim)
        code, idx = sim.ctx.error()
        B = 4 if prec == "fp32" else 8
        r = {"value": n * steps / t, "unit": "granule-steps/s", "ms_per_step": t / steps * 1e3,
             "neighbour_builds": builds, "stages_ms": {k_: round(v * 1e3, 4) for k_, v in stages.items()},
             "stage_rooflines": stage_rooflines(stages, n, nodes, B, int(np.prod(d["params"]["n"])),
                                               stored_tile_bytes(d)),
             "error": [code, idx]}
        res[prec] = r
        del sim
        torch.cuda.empty_cache()
    return res


WORKLOAD_TEXT = {
    "c2": lambda d: (f"c2: {d['x'].shape[1]} granules, log-normal radii (median 5 mm, sigma 0.2, clipped to "
                     f"[3, 10] mm), random sequential addition at solid fraction 0.30, gravity, 128^3 grid "
                     f"dx=0.01, 16 Fourier modes A=0.2, dt=5e-6, FP32 form"),
    "c3": lambda d: (f"c3: dam-break column, {d['x'].shape[1]} granules r=1 mm, {d['params']['n']} grid "
                     f"dx={d['params']['dx']}, dt={d['params']['dt']}"),
    "c5": lambda d: (f"c5: {d['x'].shape[1]} granules, radii U[0.75, 1.5] mm on a jittered lattice, "
                     f"{d['params']['n']} grid dx=0.003, shear flow plus 32 modes, gravity, dt=1e-6, FP32 form"),
}


def time_adjoint(reps=3):
    """Forward and backward of the differentiable rollout on the c4 workload
    (65,536 bidisperse granules, 20 steps, checkpoint every 5), FP64: each
    pass replayed as a recorded HIP graph (recorded in the untimed first
    repetition), and run directly for comparison."""
    import torch
    from paper_2504_00745_amd import workloads as wl
    from paper_2504_00745_amd.rollout import GICRollout, Rollout
    d = wl.make("c4")
    cfg = d["params"]
    x0 = torch.as_tensor(d["x"]).cuda()
    v0d = torch.as_tensor(d["v"]).cuda()

    def timed(sim):
        fw, bw = [], []
        for it in range(reps + 1):
            v0 = v0d.clone().requires_grad_(True)
            mu = torch.tensor(cfg["mu"], dtype=torch.float64, requires_grad=True)
            cd = torch.tensor(cfg["c_drag"], dtype=torch.float64, requires_grad=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L = GICRollout.apply(x0, v0, mu, cd, sim)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if it:
                fw.append(t1 - t0)
                bw.append(t2 - t1)
        return float(np.median(fw)) * 1e3, float(np.median(bw)) * 1e3

    rm = float(d["r"].max())
    f, b = timed(Rollout(cfg, d["r"], d["u"], 20, ckpt=5, r_max=rm, graph=True))
    fd, bd = timed(Rollout(cfg, d["r"], d["u"], 20, ckpt=5, r_max=rm))
    return {"workload": "c4: 65,536 bidisperse granules, 64^3 grid, 20 steps, checkpoint every 5, FP64",
            "forward_ms": f, "backward_ms": b, "ratio": b / f, "reps": reps, "graph": True,
            "direct": {"forward_ms": fd, "backward_ms": bd, "ratio": bd / fd}}


COPY_BYTES = 1 << 30


def copy_calibration():
    """Three launches of a plain elementwise copy of 1 GiB (torch's neg: reads
    1 GiB, writes 1 GiB): a known-size kernel for scaling HBM byte counters."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


# Source files whose change invalidates a stored HBM traffic measurement.
TRAFFIC_SOURCES = {
    "contact": ["contact.hip", "gic_device.hpp", "gic_launch.hpp"],
    "assemble": ["transfer.hip", "gic_device.hpp", "gic_launch.hpp"],
    "integrate_p2g": ["transfer.hip", "gic_device.hpp", "gic_launch.hpp"],
    "gather_g2p_drag": ["step.hip", "gic_device.hpp", "gic_launch.hpp"],
    "gather_g2p_fluid": ["step.hip", "gic_device.hpp", "gic_launch.hpp"],
    "exchange_p2g": ["transfer.hip", "gic_device.hpp", "gic_launch.hpp"],
}


def source_digest(stage):
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2504_00745_amd", "csrc")
    for f in TRAFFIC_SOURCES.get(stage, []):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(stage, workload):
    """HBM bytes per launch of a stage's kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same
    counter's reading for the 1 GiB copy), or None when there is none or the
    kernel's sources have changed since it was taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"hbm_traffic_{stage}_{workload}.txt")
    if stage not in TRAFFIC_SOURCES or not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_digest(stage):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_coupled(d, wl_name, substeps=4, sand_steps=8):
    """The workload with the remaining interphase forces on (Sec. 3.3 Eq.
    5a-5c, Sec. 5.2 Eq. 9) in sand steps of `substeps` sub-steps (Alg. 2),
    FP32 form: a hydrostatic pressure gradient rho_f g plus a seeded
    perturbation, a seeded fluid-acceleration field, virtual mass and the
    exchange-momentum deposit.  Whole sand steps timed with HIP events, then
    the stages of each sub-step from the events the library records between
    them."""
    import torch
    from paper_2504_00745_amd import gic
    cfg = dict(d["params"], rho_f=1000.0, vmass=1, f_unit=1e-8)
    n = d["x"].shape[1]
    Gn = int(np.prod(cfg["n"]))
    rng = np.random.Generator(np.random.PCG64(12))
    gp = (np.array(cfg["g"])[:, None] * 1000.0 + rng.normal(0.0, 50.0, (3, Gn))).reshape(-1)
    af = rng.normal(0.0, 0.1, 3 * Gn)
    sim = gic.Simulator(cfg, d["x"], d["v"], d["r"], d["u"], "fp32", r_max=float(d["r"].max()))
    GP = torch.as_tensor(gp, dtype=torch.float32, device="cuda")
    AF = torch.as_tensor(af, dtype=torch.float32, device="cuda")
    FS = torch.zeros(3 * Gn, dtype=torch.int64, device="cuda")
    Dt = substeps * cfg["dt"]
    sim.sand_step(Dt, grad_p=GP, acc_f=AF, fs=FS)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    N = 0
    for _ in range(sand_steps):
        N += sim.sand_step(Dt, grad_p=GP, acc_f=AF, fs=FS)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    code, idx = sim.ctx.error()
    # per stage, from the events the library records between the stages of
    # each sub-step
    st, k = time_stages(sim, 4, sand_dt=Dt, grad_p=GP, acc_f=AF, fs=FS)
    acc = {key: st[key] for key in ("sort", "gather_g2p_fluid", "contact", "exchange_p2g", "integrate_p2g",
                                    "assemble")}
    nodes = touched_nodes(sim)
    xb = coupled_bytes("exchange_p2g", n, nodes, 4)
    ach = xb / acc["exchange_p2g"] / 1e9
    return {"workload": f"same bed with grad p, fluid acceleration, virtual mass (rho_f = 1000) and the "
                        f"exchange deposit, sand steps of {substeps} sub-steps, FP32",
            "ms_per_substep": t / N * 1e3, "value": n * N / t, "unit": "granule-substeps/s",
            "substeps": N, "stages_ms": {k: round(v * 1e3, 4) for k, v in acc.items()},
            "exchange_roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes": xb,
                                  "traffic": stored_traffic("exchange_p2g", wl_name)},
            "error": [code, idx]}


def time_capillary(d, wl_name, reps=10):
    """The workload as a wet bed (Sec. 5.3-5.4): the moisture ratio of every
    granule from its sampled fluid fraction and a seeded held-water ratio,
    contact plus liquid-bridge forces with the wet masses of Eq. 19 in the
    damping, and the wet integrate + P2G, FP32 form, on the sorted state of a
    step; the dry contact and dry integrate + P2G timed on the same state
    beside them (the state is restored before every integrate call)."""
    import torch
    from paper_2504_00745_amd import gic
    cfg = dict(d["params"], sigma=0.072, vbridge=1e-4, sr_peak=0.3, rho_f=1000.0)
    n = d["x"].shape[1]
    sim = gic.Simulator(cfg, d["x"], d["v"], d["r"], d["u"], "fp32", r_max=float(d["r"].max()))
    sim.step()
    ctx, s = sim.ctx, sim.scratch
    cur, nxt = sim.cur, sim.nxt
    gic.gic_sort_cells(ctx, cur["x"], s["key"], s["order"], s["cell_begin"], s["cell_end"])
    uat = torch.empty(3 * n, dtype=torch.float32, device="cuda")
    af = torch.empty(n, dtype=torch.float32, device="cuda")
    gic.gic_gather_g2p_drag(ctx, s["order"], cur["x"], cur["v"], cur["r"], cur["id"], nxt["x"], nxt["v"], nxt["r"],
                            nxt["id"], sim.u, sim.alpha, s["cell_begin"], s["cell_end"], s["f_drag"], u_at=uat,
                            alpha_f=af)
    rng = np.random.Generator(np.random.PCG64(14))
    held = torch.as_tensor(rng.uniform(0.0, 0.2, n), dtype=torch.float64, device="cuda")
    sr = torch.empty(n, dtype=torch.float32, device="cuda")
    F, Fd = s["f_contact"], s["f_drag"]
    cb_, ce_ = s["cell_begin"], s["cell_end"]
    args = (nxt["x"], nxt["v"], nxt["r"])
    x0, v0 = nxt["x"].clone(), nxt["v"].clone()
    X, V = torch.empty_like(x0), torch.empty_like(v0)
    gic.gic_moisture_ratio(ctx, held, af, sr)
    gic.gic_contact_capillary_forces(ctx, *args, sr, cb_, ce_, F, held=held)  # warm-up
    torch.cuda.synchronize()
    K = 6
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * K * reps)]
    for i in range(reps):
        e = ev[2 * K * i:2 * K * (i + 1)]
        e[0].record()
        gic.gic_moisture_ratio(ctx, held, af, sr)
        e[1].record()
        e[2].record()
        gic.gic_contact_capillary_forces(ctx, *args, sr, cb_, ce_, F, held=held)
        e[3].record()
        e[4].record()
        gic.gic_contact_forces(ctx, *args, cb_, ce_, F)
        e[5].record()
        X.copy_(x0)
        V.copy_(v0)
        e[6].record()
        gic.gic_integrate_p2g_wet(ctx, X, V, nxt["r"], held, F, Fd, cb_, ce_, sim.alpha, sim.mom)
        e[7].record()
        X.copy_(x0)
        V.copy_(v0)
        e[8].record()
        gic.gic_integrate_p2g(ctx, X, V, nxt["r"], F, Fd, cb_, ce_, sim.alpha, sim.mom)
        e[9].record()
        e[10].record()
        e[11].record()
    torch.cuda.synchronize()
    t = [sum(ev[2 * K * i + 2 * k].elapsed_time(ev[2 * K * i + 2 * k + 1]) for i in range(reps)) / reps / 1e3
         for k in range(5)]
    code, idx = ctx.error()
    cb = n * CAPILLARY_BYTES_PER_GRANULE
    ach = cb / t[1] / 1e9
    srv = sr.cpu().numpy()
    return {"workload": "same bed wet (sigma = 0.072 N/m, bridge volume 1e-4 of the granule volume, Gamma peak "
                        "at sr = 0.3; held water U(0, 0.2) per granule volume, rho_f = 1000), FP32",
            "moisture_ratio_ms": round(t[0] * 1e3, 4), "contact_capillary_ms": round(t[1] * 1e3, 4),
            "contact_dry_ms": round(t[2] * 1e3, 4), "integrate_p2g_wet_ms": round(t[3] * 1e3, 4),
            "integrate_p2g_dry_ms": round(t[4] * 1e3, 4), "value": n / t[1],
            "unit": "granules/s (contact + bridges, wet masses)", "sr_median": float(np.median(srv)),
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes": cb, "traffic": None},
            "error": [code, idx]}


# One conjugate-gradient iteration of the density projection reads and writes,
# per cell (ac: the signed coefficient that carries alpha_f' and the label):
# w = L d (d, ac; w: 24), the update (d, w, 1/diag, q, r; q, r: 56) and the new
# direction (r, 1/diag, d; d: 32).
IDP_BYTES_PER_CELL_ITER = 24 + 56 + 32
# With the multigrid V-cycle: w = L d (24), the update without r.z (d, w, q, r;
# q, r: 48), the new direction (z, d; d: 24) and per fine cell the
# restriction (b, 1/diag, ac: 24 plus 1/8 of a coarse write), the coarse
# correction (b, 1/diag, ac, 1/8 of the coarse e and ac; u: 34) and the
# post-sweep (u, ac, 1/diag, b; e: 40), on every level of at least 2^18
# cells (the finest two here: 1 + 1/8); smaller levels correct and sweep in
# one pass (b, 1/diag, ac, coarse e and ac; e: 34), 1/64 + 1/512 + ... = 1/56.
IDP_MG_BYTES_PER_CELL_ITER = 24 + 48 + 24 + (25 + 34 + 40) * (1 + 1 / 8.0) + (25 + 34) / 56.0


def time_idp(reps=3, tol=1e-6):
    """Density projection (Sec. 5.1, Eq. 12b-13) on the dam-break grid
    (256 x 128 x 128 cells), cold start, relative residual 1e-6: whole
    projections with the multigrid preconditioner (state checked every 8
    iterations) and with the Jacobi one (every 32), timed with events; then
    each solver's iterations alone (a fixed count with a tolerance never met)
    for the per-iteration rate and its roofline."""
    import torch
    from paper_2504_00745_amd import gic, workloads as wl
    d = wl.idp_case("c3")
    ctx = gic.Context(d["params"], 1, "fp64", r_max=0.25 * d["params"]["dx"])
    G = ctx.G
    nx, ny, nz = d["params"]["n"]
    afx = torch.as_tensor(d["alpha_fx"]).to("cuda")
    ast = torch.as_tensor(d["alpha_star"]).to("cuda")
    lab = torch.as_tensor(d["label"]).to("cuda")
    q = torch.zeros(G, dtype=torch.float64, device="cuda")
    fx = torch.empty((nx + 1) * ny * nz, dtype=torch.float64, device="cuda")
    fy = torch.empty(nx * (ny + 1) * nz, dtype=torch.float64, device="cuda")
    fz = torch.empty(nx * ny * (nz + 1), dtype=torch.float64, device="cuda")
    work = gic.idp_workspace(ctx)
    at = torch.empty(G, dtype=torch.float64, device="cuda")
    s = torch.empty_like(at)
    gic.gic_idp_setup(ctx, afx, ast, lab, at, s)
    out = {}
    for pc, name, chk, fixed in ((1, "multigrid", 8, 16), (0, "jacobi", 32, 64)):
        q.zero_()
        gic.gic_density_projection(ctx, afx, ast, lab, q, fx, fy, fz, work, max_iter=5000, tol=tol,
                                   check_every=chk, precond=pc)  # warm-up
        ts = []
        for _ in range(reps):
            q.zero_()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            it, rel = gic.gic_density_projection(ctx, afx, ast, lab, q, fx, fy, fz, work, max_iter=5000, tol=tol,
                                                 check_every=chk, precond=pc)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        q.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gic.gic_idp_solve(ctx, at, lab, s, q, work, max_iter=fixed, tol=0.0, check_every=fixed, precond=pc)
        e1.record()
        torch.cuda.synchronize()
        t_it = e0.elapsed_time(e1) / 1e3 / fixed
        per = IDP_MG_BYTES_PER_CELL_ITER if pc else IDP_BYTES_PER_CELL_ITER
        ach = per * G / t_it / 1e9
        out[name] = {"ms_per_projection": round(float(np.median(ts)) * 1e3, 3), "iterations": int(it),
                     "relres": rel, "us_per_iteration": round(t_it * 1e6, 2),
                     "roofline": {"bound": "hbm", "kernel": f"PCG iteration ({name})", "achieved": ach,
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                  "algorithmic_bytes": per * G, "traffic": None}}
    t = out["multigrid"]["ms_per_projection"] / 1e3
    return {"workload": "dam-break grid 256 x 128 x 128 cells (dx = 0.004): sand column of the c3 bed, fluid to "
                        "3/4 height, air above, a submerged solid block, fluid fraction perturbed 8 % and "
                        "compressed 1.8x in a ball; PCG from zero to relative residual 1e-6",
            "value": G / t, "unit": "cells/s (whole projection, multigrid)", **out}


def touched_nodes(sim):
    import torch
    return int((sim.alpha != 0).sum().item())


def cpu_info():
    """Host cores visible to this process and the CPU model (lscpu)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(d, steps):
    """The FP64 oracle as it stands, on this host's cores: `steps` full steps
    of the workload with all threads, and one step of a slab of a quarter of
    its granules (the quarter with the smallest x) on one thread."""
    import oracle
    cfg = d["params"]
    x, v, r, u = d["x"], d["v"], d["r"], d["u"]
    n = x.shape[1]
    all_threads = oracle.num_threads()
    res = {"kind": "oracle", "unit": "granule-steps/s", **cpu_info()}

    def run(xx, vv, rr, k):
        a0, _ = oracle.p2g_fixed(cfg, xx, vv, rr)
        t0 = time.perf_counter()
        for _ in range(k):
            st = oracle.step(cfg, xx, vv, rr, u, a0)
            xx, vv, a0 = st["x"], st["v"], st["alpha"]
        return time.perf_counter() - t0

    oracle.set_num_threads(all_threads)
    t = run(x, v, r, steps)
    res.update(value=n * steps / t, cores=all_threads, seconds=round(t, 3),
               sample=f"{steps} full steps of the {d['name']} workload ({n} granules), FP64 C oracle, "
                      f"{all_threads} OpenMP threads")
    m = n // 4
    sel = np.argsort(x[0], kind="stable")[:m]
    xs, vs, rs = np.ascontiguousarray(x[:, sel]), np.ascontiguousarray(v[:, sel]), r[sel]
    oracle.set_num_threads(1)
    t1 = run(xs, vs, rs, 1)
    oracle.set_num_threads(all_threads)
    res["single_thread"] = {"value": m / t1, "cores": 1, "seconds": round(t1, 3),
                            "sample": f"1 step of the {m} granules with the smallest x of the {d['name']} workload"}
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported: the path runs on one GPU "
              "and its sharding across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2504_00745_amd import gic, workloads as wl
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if a.copy_calibration:
        log("[bench] copy calibration: 3 x 1 GiB")
        copy_calibration()
    log(f"[bench] generating {a.workload}")
    d = wl.make(a.workload)
    n = d["x"].shape[1]
    G = int(np.prod(d["params"]["n"]))
    rmax = float(d["r"].max())
    out = {}
    for prec in (["fp32"] if a.no_fp64 else ["fp32", "fp64"]):
        log(f"[bench] {prec}: building state")
        sim = gic.Simulator(d["params"], d["x"], d["v"], d["r"], d["u"], prec, r_max=rmax)
        log(f"[bench] {prec}: timing {a.steps} steps after {a.warmup} warmup")
        t_ev, t_wall, builds = time_steps(sim, a.steps, a.warmup)
        code, idx = sim.ctx.error()
        if code:
            log(f"[bench] {prec}: kernel error latched: code {code} index {idx}")
        stages, _ = time_stages(sim, max(3, min(a.steps, 10)))
        nodes = touched_nodes(sim)
        out[prec] = dict(t=t_ev, wall=t_wall, stages=stages, nodes=nodes, err=code, builds=builds)
        log(f"[bench] {prec}: {t_ev / a.steps * 1e3:.3f} ms/step  stages(ms) " +
            " ".join(f"{k}={v * 1e3:.3f}" for k, v in stages.items()) + f"  list builds {builds}")
        del sim
        torch.cuda.empty_cache()
    r32 = out["fp32"]
    value = n * a.steps / r32["t"]
    st = r32["stages"]
    line = {
        "metric": "granule-steps/s FP32 vs plain FP64 GPU path at 4M granules; bwd/fwd time",
        "value": value,
        "unit": "granule-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r32["t"] / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 forces / f64 state / i64 grids",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[a.workload](d) if a.workload in WORKLOAD_TEXT else a.workload,
                   "granules": n, "grid_nodes": G, "parallelism": "single GPU"},
        "stages_ms": {k: round(v * 1e3, 4) for k, v in st.items()},
        "neighbour_builds": r32["builds"],
        "roofline": dominant_roofline(st, n, r32["nodes"], 4, a.workload, G),
        "stage_rooflines": stage_rooflines(st, n, r32["nodes"], 4, G, stored_tile_bytes(d)),
    }
    if "fp64" in out:
        r64 = out["fp64"]
        line["fp64_value"] = n * a.steps / r64["t"]
        line["fp32_over_fp64"] = line["value"] / line["fp64_value"]
        line["fp64_stages_ms"] = {k: round(v * 1e3, 4) for k, v in r64["stages"].items()}
    if not a.no_error:
        log("[bench] FP32 form against the plain FP64 path, per output")
        line["fp32_error"] = {a.workload: fp32_error(d, rmax)}
        if not a.no_c2:
            d2 = wl.make("c2")
            line["fp32_error"]["c2"] = fp32_error(d2, float(d2["r"].max()))
            del d2
        torch.cuda.empty_cache()
    if not a.no_c2:
        log("[bench] c2: polydisperse moving bed, 100 steps")
        line["c2"] = run_leg("c2", 100, 3, with_fp64=True)
    if not a.no_c5:
        log("[bench] c5: large bed, 20 steps")
        line["c5"] = run_leg("c5", 20, 2)
    if not a.no_coupled:
        log("[bench] coupled: remaining interphase forces and exchange, sand steps of 4 sub-steps")
        line["coupled"] = time_coupled(d, a.workload)
        torch.cuda.empty_cache()
    if not a.no_capillary:
        log("[bench] capillary: wet bed, moisture ratio and contact plus liquid-bridge forces")
        line["capillary"] = time_capillary(d, a.workload)
        torch.cuda.empty_cache()
    if not a.no_idp:
        log("[bench] density projection on the dam-break grid")
        line["idp"] = time_idp()
        torch.cuda.empty_cache()
    if not a.no_adjoint:
        log("[bench] adjoint: forward and backward of the c4 rollout")
        line["bwd_fwd"] = time_adjoint()
    if not a.no_cpu:
        log(f"[bench] cpu baseline: {a.cpu_steps} oracle steps, all threads; a quarter slab on one thread")
        line["cpu_baseline"] = cpu_baseline(d, a.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
