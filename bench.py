"""Benchmark of the mechanical-interaction step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64]
                    [--neighbors 12] [--no-cpu] [--no-extras]

A step is one pass of the whole hot path over the population: uniform-grid
build (bounds, binning, counts, scan, stable scatter), 27-box gather with the
Eq. 1 force and the displacement rule, and the position update.  The headline
workload is 2,097,152 agents uniform in a cube sized for ~12 neighbours within
the interaction radius 12, diameters U[8, 12], FP32.  Inputs are resident in
device memory before timing starts.  The timed region replays a HIP graph of
one step K times.

One JSON line is printed with, besides the headline value:
  roofline      the force step's algorithmic flops per call (9 per 27-box
                candidate + 25 per contact, the measured candidate and contact
                counts of the workload) over its mean duration from HIP events
                around every ms_mech_step call of an eager K-step pass (the
                gather kernel k_force and the record split k_soa), against the
                FP32 vector peak; traffic (HBM bytes of both kernels from
                rocprofv3 counters) is filled from the committed profile summary
                when it was taken on the current sources.
  cpu_baseline  the FP64 oracle (single thread) on the same population.
  variants      other densities / FP64, fwd+bwd and the batched workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "agent-steps/s mech step @2M agents: plain vs batched vs fwd+bwd; % HBM peak"
HBM_PEAK = 8.0e12            # B/s
FP32_PEAK = 157.3e12         # flop/s, published FP32 vector peak
FP64_PEAK = 78.6e12
PARAMS = dict(kappa=2.0, gamma=1.0, dt=0.01, max_disp=3.0, adherence=0.0)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_alg(n, n_boxes, S):
    """Algorithmic bytes of a whole step: 22S + 16 per agent and 20 per box."""
    return (22 * S + 16) * n + 20 * n_boxes


def force_bytes(n, n_boxes, S):
    """Force kernel: payload 4S + perm 4 read, 3S written per agent; start 4 per box."""
    return (7 * S + 4) * n + 4 * n_boxes


def workload_stats(ms, ws, n):
    """Mean 27-box candidates C, contacts K, neighbours within the radius and
    occupancy, from the exported grid and neighbour lists."""
    import torch
    g = ms.grid_get(ws)
    info = g["info"][0]
    nx, ny, nz = info["dims"]
    start = g["start"].cpu().numpy().astype(np.int64)
    cnt = np.diff(start).reshape(nz, ny, nx)
    pad = np.pad(cnt, 1)
    box27 = np.zeros_like(cnt)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                box27 += pad[dz:dz + nz, dy:dy + ny, dx:dx + nx]
    C = float(np.sum(cnt * (box27 - 1)) / n)
    counts, offsets, lst = ms.neighbors(ws)
    return dict(candidates=C, neighbors=float(counts.double().mean().item()),
                n_boxes=int(info["n_boxes"]), occupancy=n / max(int(info["n_boxes"]), 1),
                dims=list(info["dims"]), edge=info["edge"], lists=(counts, offsets, lst))


def contacts_per_agent(x, y, z, d, counts, lst):
    import torch
    i = torch.repeat_interleave(torch.arange(counts.numel(), device=counts.device), counts.long())
    j = lst.long()
    X, Y, Z, D = (t.double() for t in (x, y, z, d))
    l = torch.sqrt((X[i] - X[j]) ** 2 + (Y[i] - Y[j]) ** 2 + (Z[i] - Z[j]) ** 2)
    K = ((D[i] + D[j]) / 2 - l > 0).sum().item()
    return K / counts.numel()


def time_plain(ms, torch, arrs, dtype, steps, warmup, graph=True, events=False, backward=False):
    """Returns (seconds for `steps` steps, mean force-kernel ms or None)."""
    n = arrs[0].size
    # The differentiated step keeps the forward's forces for the backward of
    # the same build and parameters, as the autograd rollout does.
    ws = ms.Workspace(n, dtype=dtype, keep_forces=backward)
    in_t = torch.float32 if dtype == "f32" else torch.float64
    t = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda", in_t) for a in arrs]
    x0 = [a.clone() for a in t[:3]]
    out = tuple(torch.empty(n, dtype=ws.out_dtype, device="cuda") for _ in range(3))
    gout = tuple(torch.empty(n, dtype=ws.out_dtype, device="cuda") for _ in range(4))
    gkg = torch.empty(2, dtype=torch.float64, device="cuda")
    gin = tuple(torch.full((n,), 1e-3, dtype=ws.out_dtype, device="cuda") for _ in range(3))
    # contact-list length of the gather picked on this workload, outside the timed region
    from paper_2105_00039_amd import autotune
    ms.grid_build(ws, *t)
    ws.tuning = autotune.tune(ws, lambda: ms.mech_step(ws, PARAMS, out=out))

    def one(ev=None):
        ms.grid_build(ws, *t)
        if ev is not None:
            # roofline pass: events around the displacement step alone
            ev[0].record()
            ms.mech_step(ws, PARAMS, out=out)
            ev[1].record()
        else:
            # rollout step: displacements written and added to the positions
            ms.mech_step_integrate(ws, PARAMS, *t[:3], out=out)
        if backward:
            ms.mech_step_backward(ws, PARAMS, *gin, out=gout, g_params=gkg)
        if ev is not None:
            ms.integrate(*t[:3], *out)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    ms.device_status(ws)
    force_ms = None
    if events:
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for k in range(steps):
            one(evs[k])
        b.record()
        torch.cuda.synchronize()
        force_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
        total = a.elapsed_time(b) / 1e3
    elif graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            one()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            one()
        for _ in range(max(warmup, 1)):
            gr.replay()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            gr.replay()
        b.record()
        torch.cuda.synchronize()
        total = a.elapsed_time(b) / 1e3
    else:
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            one()
        b.record()
        torch.cuda.synchronize()
        total = a.elapsed_time(b) / 1e3
    ms.device_status(ws)
    for a_, b_ in zip(t[:3], x0):
        a_.copy_(b_)
    return total, force_ms, ws, t


def time_sorted_state(ms, torch, arrs, dtype, steps, warmup, reps=10):
    """Steps on the same population renumbered into the slot order of its
    first build (box-sorted state, as a rollout that reorders its state
    keeps it), and the time to reorder the four state arrays once: from the
    random input order (first_reorder_us) and from the sorted state after one
    step of motion (reorder_us, what a rollout pays per reorder)."""
    n = arrs[0].size
    in_t = torch.float32 if dtype == "f32" else torch.float64
    ws = ms.Workspace(n, dtype=dtype)
    t = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda", in_t) for a in arrs]
    out = [torch.empty_like(a) for a in t]

    def reorder_us():
        for a, o in zip(t, out):
            ms.reorder(ws, a, out=o)
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a0.record()
        for _ in range(reps):
            for a, o in zip(t, out):
                ms.reorder(ws, a, out=o)
        a1.record()
        torch.cuda.synchronize()
        ms.device_status(ws)
        return a0.elapsed_time(a1) / reps * 1e3

    ms.grid_build(ws, *t)
    first_us = reorder_us()
    sarrs = [o.cpu().numpy() for o in out]
    # one step of motion on the sorted state, then the reorder a rollout does
    for a, o in zip(t, out):
        a.copy_(o)
    disp = tuple(torch.empty(n, dtype=ws.out_dtype, device="cuda") for _ in range(3))
    ms.grid_build(ws, *t)
    ms.mech_step(ws, PARAMS, out=disp)
    ms.integrate(*t[:3], *disp)
    ms.grid_build(ws, *t)
    steady_us = reorder_us()
    del ws, t, out, disp
    sec, _, _, _ = time_plain(ms, torch, sarrs, dtype, steps, warmup, graph=True)
    return dict(value=n * steps / sec, unit="agent-steps/s", ms_per_step=sec / steps * 1e3,
                reorder_us=steady_us, first_reorder_us=first_us,
                what="graph-replayed steps on the box-sorted state (ms_reorder of x, y, z, d "
                     "into the slot order of the first build); reorder_us: one reorder of the "
                     "four arrays of a sorted state after a step of motion; first_reorder_us: "
                     "the same from the random input order")


def time_host_state(ms, torch, arrs, steps, warmup):
    """Host co-processing: the state (x, y, z, d) lives in pinned host memory,
    as in the paper's deployment, and every step copies it to the GPU, builds
    the grid, steps and integrates there, and copies the positions back.
    (a) one simulation, copies and compute in sequence; (b) the population
    split into two independent simulations on two streams of default priority,
    so one's copies overlap the other's compute.  Rates count all agents."""
    n = arrs[0].size
    host = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in arrs]

    def sim(lo, hi):
        m = hi - lo
        ws = ms.Workspace(m, dtype="f32")
        dev = [torch.empty(m, dtype=torch.float32, device="cuda") for _ in range(4)]
        return ws, dev, [h[lo:hi] for h in host]

    def one(ws, dev, hs):
        for dv, h in zip(dev, hs):
            dv.copy_(h, non_blocking=True)
        ms.grid_build(ws, *dev)
        ms.mech_step_integrate(ws, PARAMS, *dev[:3])
        for dv, h in zip(dev[:3], hs[:3]):
            h.copy_(dv, non_blocking=True)

    def run(sims, streams, k):
        for _ in range(k):
            for sm, st in zip(sims, streams):
                with torch.cuda.stream(st):
                    one(*sm)
        torch.cuda.synchronize()

    out = {}
    for label, sims in (("one_sim", [sim(0, n)]), ("two_sims_overlapped", [sim(0, n // 2), sim(n // 2, n)])):
        streams = [torch.cuda.Stream() for _ in sims]
        run(sims, streams, warmup)
        t0 = time.perf_counter()
        run(sims, streams, steps)
        sec = time.perf_counter() - t0
        for ws, _, _ in sims:
            ms.device_status(ws)
        out[label] = n * steps / sec
        out[label + "_ms_per_step"] = sec / steps * 1e3
        del sims
    out.update(unit="agent-steps/s", bytes_per_step=n * 16 + n * 12,
               what="pinned host state (x, y, z, d) copied in and positions copied out every "
                    "step around build + step + integrate; PCIe-inclusive, host-clock timed")
    return out


def time_growing(ms, torch, steps, seed=0, n0=1_048_576, growth=1.04):
    """Variable population: a 1,048,576-agent uniform population (n≈12) grows by
    the synthetic division rule of workloads.grow_and_divide (done here on the
    device with torch ops: d *= growth, agents above 12 split into two
    half-volume daughters) and is stepped on one workspace sized for the final
    count.  Timed with events: grid build + step + integrate of every step;
    the rate is sum(N_t) / sum(time_t)."""
    from paper_2105_00039_amd import workloads
    pop = workloads.uniform(n0, mean_neighbors=12.0, seed=seed)
    t = [torch.from_numpy(a.astype(np.float32)).cuda() for a in pop.arrays()]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed + 77)
    ws = ms.Workspace(4 * n0, dtype="f32")
    ev = []
    sizes = []
    for _ in range(steps):
        x, y, z, d = t
        d = d * growth
        div = torch.nonzero(d > 12.0).squeeze(1)
        if div.numel():
            u = torch.randn(div.numel(), 3, device="cuda", generator=gen, dtype=torch.float32)
            u = u / u.norm(dim=1, keepdim=True)
            off = (d[div] / 4.0)[:, None] * u
            dd = d[div] / 2.0 ** (1.0 / 3.0)
            px, py, pz = x[div], y[div], z[div]
            x = x.clone(); y = y.clone(); z = z.clone()
            x[div] = px + off[:, 0]; y[div] = py + off[:, 1]; z[div] = pz + off[:, 2]; d[div] = dd
            x = torch.cat([x, px - off[:, 0]]); y = torch.cat([y, py - off[:, 1]])
            z = torch.cat([z, pz - off[:, 2]]); d = torch.cat([d, dd])
        t = [x.contiguous(), y.contiguous(), z.contiguous(), d.contiguous()]
        if t[0].numel() > 4 * n0:
            break
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ms.grid_build(ws, *t)
        ms.mech_step_integrate(ws, PARAMS, *t[:3])
        e1.record()
        ev.append((e0, e1))
        sizes.append(t[0].numel())
    torch.cuda.synchronize()
    ms.device_status(ws)
    times = [a.elapsed_time(b) / 1e3 for a, b in ev]
    return dict(value=sum(sizes) / sum(times), unit="agent-steps/s", steps=len(sizes),
                n_first=sizes[0], n_last=sizes[-1], ms_per_step_first=times[0] * 1e3,
                ms_per_step_last=times[-1] * 1e3,
                what="growing population (synthetic division rule), eager build + fused step "
                     "per step on one workspace, events around each step")


def time_batched(ms, torch, steps, warmup, seed=0):
    from paper_2105_00039_amd import workloads
    b = workloads.batched(seed=seed)
    n = b.n
    ws = ms.Workspace(n, max_sims=b.n_sims, dtype="f32_pos64")
    t = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in b.arrays(np.float64)]
    spec = ms.BatchSpec(b.offsets)
    P = ms.params_tensor([dict(PARAMS, kappa=float(k), gamma=float(g)) for k, g in zip(b.kappa, b.gamma)],
                         "cuda")
    out = tuple(torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3))
    from paper_2105_00039_amd import autotune
    ms.grid_build_batched(ws, *t, spec)
    tuning = autotune.tune(ws, lambda: ms.mech_step_batched(ws, P, out=out))

    def one():
        ms.grid_build_batched(ws, *t, spec)
        ms.mech_step_batched_integrate(ws, P, *t[:3], out=out)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    ms.device_status(ws)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        one()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        one()
    gr.replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        gr.replay()
    e.record()
    torch.cuda.synchronize()
    ms.device_status(ws)
    sec = a.elapsed_time(e) / 1e3
    return dict(value=n * steps / sec, unit="agent-steps/s", n_sims=b.n_sims, n_agents=n, steps=steps,
                ms_per_step=sec / steps * 1e3, dtype="f32 force, f64 positions",
                gather_list=tuning["choice"],
                workload="batched256: sizes 10^U(3,5), 4-30 neighbours, kappa U[1,4], gamma U[0.5,2]")


def cpu_baseline(arrs, budget_s=12.0, max_steps=3):
    import oracle
    a64 = [np.asarray(a, dtype=np.float64) for a in arrs]
    n = a64[0].size
    done = 0
    t0 = time.perf_counter()
    while done < max_steps:
        oracle.step(*a64, PARAMS)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    sec = time.perf_counter() - t0
    return dict(value=n * done / sec, unit="agent-steps/s", cores=1, kind="oracle",
                sample=f"{done} full step(s) (grid + force + displacement) of the same {n}-agent "
                       f"population, FP64, single thread, {sec:.1f} s")


FORCE_SOURCES = ("paper_2105_00039_amd/csrc/force.hip", "paper_2105_00039_amd/csrc/gather.hpp",
                 "paper_2105_00039_amd/csrc/common.hpp")


def force_source_hash():
    """Hash of the force kernel's sources: a traffic figure measured on other
    sources is stale and reported as null."""
    import hashlib
    h = hashlib.sha256()
    for rel in FORCE_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_values(name):
    """The `- key: value` lines of a committed profile summary, or None when
    the summary is missing or was taken on other force sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("force_source_hash") != force_source_hash():
        return None
    return vals


def traffic_from_profiles(workload):
    """HBM bytes per ms_mech_step call from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy probe), if it was taken on the
    current force sources."""
    vals = profile_values(f"k_force_{workload}_traffic.md")
    try:
        return float(vals["hbm_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def issue_from_profiles(workload):
    """Issue-side utilisation of the force kernel from the committed counter
    summary (VALU issue share of the SIMD cycles, texture address/data unit
    busy), if it was taken on the current force sources."""
    vals = profile_values(f"k_force_{workload}_counters.md")
    if not vals:
        return None
    try:
        return {k: float(vals[k]) for k in ("valu_issue_frac", "ta_busy_frac", "td_busy_frac",
                                            "valu_insts_per_wave")}
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--neighbors", type=float, default=12.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the eager K-step pass (for rocprofv3 runs)")
    ap.add_argument("--workload", default="uniform2M", choices=["uniform2M", "clusters16M", "batched256"],
                    help="with --profile-only: the population of the eager pass (clusters16M: "
                         "16,777,216 agents in 64 Gaussian clusters, FP32; batched256: the "
                         "batched line's 256 simulations, graph-replayed steps)")
    ap.add_argument("--backward", action="store_true",
                    help="with --profile-only: eager steps with the backward step as well")
    ap.add_argument("--probe-copy", type=int, default=0, metavar="MIB",
                    help="with --profile-only: also run the copy probe once on MIB MiB "
                         "(the known-size kernel that scales rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the step runs on a single GPU).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2105_00039_amd as ms
    from paper_2105_00039_amd import workloads
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    N = workloads.FULL_N
    pop = workloads.uniform(N, mean_neighbors=args.neighbors, seed=args.seed)
    np_in = np.float32 if args.dtype == "f32" else np.float64
    arrs = [a.astype(np_in) for a in pop.arrays()]
    S = 4 if args.dtype == "f32" else 8
    name = f"uniform2M_n{args.neighbors:g}"
    log(f"workload {name} {args.dtype}: {N} agents, cube side {pop.meta['side']:.1f}")

    if args.profile_only:
        if args.workload == "batched256":
            del pop, arrs
            b = time_batched(ms, torch, args.steps, args.warmup)
            log(f"batched {b['n_sims']} simulations, {b['n_agents']} agents: {b['ms_per_step']:.3f} ms/step, "
                f"{b['value']:.3e} agent-steps/s, list {b['gather_list']}")
            return
        if args.workload == "clusters16M":
            del pop, arrs
            cl = workloads.workload("clusters16M", seed=args.seed)
            arrs = [a.astype(np.float32) for a in cl.arrays()]
            args.dtype = "f32"
            log(f"workload clusters16M f32: {arrs[0].size} agents")
        sec, fms, ws, _ = time_plain(ms, torch, arrs, args.dtype, args.steps, args.warmup, events=True,
                                     backward=args.backward)
        log(f"eager {args.steps} steps: {sec * 1e3 / args.steps:.3f} ms/step, force {fms * 1e3:.1f} us")
        if args.probe_copy:
            nbytes = args.probe_copy << 20
            src = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            ms.copy_probe(dst, src)
            torch.cuda.synchronize()
            log(f"copy probe: {nbytes} bytes read, {nbytes} bytes written; force sources "
                f"{force_source_hash()}")
        return

    # headline: graph-replayed steps
    sec, _, ws, t = time_plain(ms, torch, arrs, args.dtype, args.steps, args.warmup, graph=True)
    head_tuning = ws.tuning
    value = N * args.steps / sec
    log(f"graph {args.steps} steps: {sec * 1e3 / args.steps:.3f} ms/step, {value:.3e} agent-steps/s")
    # roofline of the force kernel: eager pass with events around each launch
    sec_e, force_ms, ws, t = time_plain(ms, torch, arrs, args.dtype, args.steps, args.warmup, events=True)
    log(f"eager {args.steps} steps: {sec_e * 1e3 / args.steps:.3f} ms/step, force kernel {force_ms * 1e3:.1f} us")
    ms.grid_build(ws, *t)
    st = workload_stats(ms, ws, N)
    counts, offsets, lst = st.pop("lists")
    K = contacts_per_agent(*t, counts, lst)
    del counts, offsets, lst
    flops_agent = 9 * st["candidates"] + 25 * K
    flops = flops_agent * N
    peak = FP32_PEAK if args.dtype == "f32" else FP64_PEAK
    achieved = flops / (force_ms * 1e-3)
    fb = force_bytes(N, st["n_boxes"], S)
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=peak / 1e12, unit="TFLOP/s",
                    frac=achieved / peak, traffic=traffic_from_profiles(f"{name}_{args.dtype}"),
                    kernel="ms_mech_step = k_force + k_soa (the timed rollout step runs k_soa_integrate)", flops_per_agent=flops_agent,
                    force_us=force_ms * 1e3,
                    force_alg_bytes=fb, force_alg_GBps=fb / (force_ms * 1e-3) / 1e9,
                    issue=issue_from_profiles(f"{name}_{args.dtype}"))
    balg = bytes_alg(N, st["n_boxes"], S)
    hbm = dict(step_alg_bytes=balg, step_alg_GBps=balg * args.steps / sec / 1e9,
               frac_of_peak=balg * args.steps / sec / HBM_PEAK)
    log(f"C={st['candidates']:.1f} K={K:.2f} nbrs={st['neighbors']:.2f} boxes={st['n_boxes']} "
        f"force {achieved / 1e12:.1f} TF/s; step {hbm['step_alg_GBps']:.0f} GB/s alg")

    extras = {}
    if not args.no_extras:
        other = "f64" if args.dtype == "f32" else "f32"
        oarrs = [a.astype(np.float32 if other == "f32" else np.float64) for a in pop.arrays()]
        s2, _, w2, _ = time_plain(ms, torch, oarrs, other, args.steps, args.warmup, graph=True)
        extras[f"plain_{other}_n{args.neighbors:g}"] = N * args.steps / s2
        extras[f"plain_{other}_n{args.neighbors:g}_gather_list"] = w2.tuning["choice"]
        for nb in (4.0, 30.0):
            p2 = workloads.uniform(N, mean_neighbors=nb, seed=args.seed)
            a2 = [a.astype(np_in) for a in p2.arrays()]
            s3, _, w3, _ = time_plain(ms, torch, a2, args.dtype, args.steps, args.warmup, graph=True)
            extras[f"plain_{args.dtype}_n{nb:g}"] = N * args.steps / s3
            extras[f"plain_{args.dtype}_n{nb:g}_gather_list"] = w3.tuning["choice"]
        # clustered workload: 16,777,216 agents in 64 Gaussian clusters, FP32
        cl = workloads.workload("clusters16M", seed=args.seed)
        carrs = [a.astype(np.float32) for a in cl.arrays()]
        del cl
        s5, _, w5, _ = time_plain(ms, torch, carrs, "f32", args.steps, args.warmup, graph=True)
        extras["clusters16M_f32"] = carrs[0].size * args.steps / s5
        extras["clusters16M_f32_gather_list"] = w5.tuning["choice"]
        del w5
        extras["clusters16M_f32_ms_per_step"] = s5 / args.steps * 1e3
        del carrs
        torch.cuda.empty_cache()
        sorted_state = time_sorted_state(ms, torch, arrs, args.dtype, args.steps, args.warmup)
        host_state = time_host_state(ms, torch, arrs, args.steps, args.warmup) \
            if args.dtype == "f32" else None
        growing = time_growing(ms, torch, args.steps, seed=args.seed)
        s4, _, _, _ = time_plain(ms, torch, arrs, args.dtype, args.steps, args.warmup, graph=True,
                                 backward=True)
        fwd_bwd = dict(value=N * args.steps / s4, unit="agent-steps/s", ms_per_step=s4 / args.steps * 1e3,
                       what="grid build + forward + backward + integrate, same workload")
        batched = time_batched(ms, torch, max(args.steps // 2, 2), args.warmup)
        log(f"variants {extras}; fwd+bwd {fwd_bwd['value']:.3e}; batched {batched['value']:.3e}; "
            f"sorted state {sorted_state['value']:.3e} (reorder {sorted_state['reorder_us']:.1f} us); "
            f"host state {host_state}; growing {growing}")
    else:
        fwd_bwd = batched = sorted_state = host_state = growing = None

    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline ...")
        cpu = cpu_baseline(arrs)
        log(f"oracle {cpu['value']:.3e} agent-steps/s")

    rec = {
        "metric": METRIC, "value": value, "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": name, "n_agents": N, "mean_neighbors_target": args.neighbors,
                   "measured_neighbors": st["neighbors"], "contacts_per_agent": K,
                   "candidates_per_agent": st["candidates"], "n_boxes": st["n_boxes"],
                   "diameters": "U[8,12]", "params": PARAMS, "graph": True,
                   "gather_list": head_tuning["choice"], "gather_list_ms": head_tuning["ms"]},
        "roofline": roofline, "hbm": hbm, "cpu_baseline": cpu,
        "variants": extras, "fwd_bwd": fwd_bwd, "batched": batched, "sorted_state": sorted_state,
        "host_state": host_state, "growing_population": growing,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
