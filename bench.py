"""Benchmark of the mechanical-interaction step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64]
                    [--neighbors 12] [--order sorted|caller] [--no-cpu] [--no-extras]

A step is one pass of the whole hot path over the population: uniform-grid
build (bounds, binning, counts, scan, stable scatter), 27-box gather with the
Eq. 1 force and the displacement rule, and the position update.  The headline
workload is 2,097,152 agents uniform in a cube sized for ~12 neighbours within
the interaction radius 12, diameters U[8, 12], FP32, stepped as a rollout
whose state is kept in the box-sorted slot order of each build (the agent
sorting of the paper's Section IV-D: ms_mech_step_integrate_sorted writes the
state after the step renumbered into the other of two buffers, so every
store is coalesced).  Inputs are resident in device memory before timing
starts.  The timed region replays HIP graphs of one step, K times.

One JSON line is printed with, besides the headline value:
  roofline      the force kernel's algorithmic flops per launch (9 per 27-box
                candidate + 25 per contact, the measured candidate and contact
                counts of the workload) over its mean duration from HIP events
                around every force launch of an eager K-step pass, against the
                FP32 vector peak; traffic (HBM bytes from rocprofv3 counters)
                and the issue counters are filled from the committed profile
                summaries when they were taken on the current sources.
  cpu_baseline  the FP64 oracle (-O3 -march=native) on the same population,
                on all of this process's host cores and on one.
  variants      other densities / FP64 / the caller-order state / clusters,
                fwd+bwd, the differentiated rollout and the batched workload.
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


def force_bytes(n, n_boxes, S, sorted_state=False):
    """Force step, per agent: payload 4S read and displacements 3S written,
    plus perm 4 read (caller order) or the state after the step 4S written
    (sorted state); box starts 4 per box."""
    if sorted_state:
        return 11 * S * n + 4 * n_boxes
    return (7 * S + 4) * n + 4 * n_boxes


def workload_stats(ms, ws, n):
    """Mean 27-box candidates C, contacts K, neighbours within the radius and
    occupancy, from the exported grid and neighbour lists."""
    import torch
    g = ms.grid_get(ws)
    info = g["info"][0]
    nx, ny, nz = info["dims"]
    start = g["start"].cpu().numpy().astype(np.int64)
    cnt = np.diff(start)
    ts = int(info["tile_shift"])
    if ts:   # tiled x-rows (ms_box_order): gather the rows back into (iz, iy) order
        t = 1 << ts
        iz, iy = np.meshgrid(np.arange(nz), np.arange(ny), indexing="ij")
        row = ((iz // t) * (-(-ny // t)) + iy // t) * t * t + (iz % t) * t + iy % t
        cnt = cnt.reshape(-1, nx)[row]
    cnt = cnt.reshape(nz, ny, nx)
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


def time_plain(ms, torch, arrs, dtype, steps, warmup, graph=True, events=False, backward=False,
               sorted_state=False, gather=None):
    """Returns (seconds for `steps` steps, mean force-step ms or None, ws, state).

    A step is grid build + force + displacement + integrate.  sorted_state:
    the rollout keeps its state in the build's slot order
    (ms_mech_step_integrate_sorted writes the state after the step into the
    other of two buffers, positions and diameters renumbered together);
    otherwise the state stays in the caller's order (ms_mech_step_integrate
    adds the displacements in place).  Both write the displacements too."""
    n = arrs[0].size
    # The differentiated step keeps the forward's forces for the backward of
    # the same build and parameters, as the autograd rollout does.
    ws = ms.Workspace(n, dtype=dtype, keep_forces=backward)
    in_t = torch.float32 if dtype == "f32" else torch.float64
    t = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda", in_t) for a in arrs]
    x0 = [a.clone() for a in t]
    bufs = [t, [torch.empty_like(a) for a in t]] if sorted_state else [t]
    cur = [0]
    out = tuple(torch.empty(n, dtype=ws.out_dtype, device="cuda") for _ in range(3))
    gout = tuple(torch.empty(n, dtype=ws.out_dtype, device="cuda") for _ in range(4))
    gkg = torch.empty(2, dtype=torch.float64, device="cuda")
    gin = tuple(torch.full((n,), 1e-3, dtype=ws.out_dtype, device="cuda") for _ in range(3))
    # row order of the boxes, then the launch shape of the gather (list
    # length, block size, run walk), picked on this workload outside the
    # timed region; `gather` fixes the launch shape instead (and leaves the
    # box order to the library's rule), so that the separate processes of a
    # profiling session all run the same kernel
    from paper_2105_00039_amd import autotune
    if gather is not None:
        ws.gather_list, ws.gather_block, ws.gather_walk = gather
        ms.grid_build(ws, *t)
        ws.tuning = dict(choice=tuple(gather), ms={}, source="fixed",
                         box_order=dict(choice="auto", ms={}))
    else:
        order = autotune.tune_box_order(ws, lambda: (ms.grid_build(ws, *t),
                                                     ms.mech_step(ws, PARAMS, out=out)))
        ws.tuning = autotune.tune(ws, lambda: ms.mech_step(ws, PARAMS, out=out))
        ws.tuning["box_order"] = order

    def one(ev=None, c=None):
        """One step from state buffer c (default: the current one)."""
        c = cur[0] if c is None else c
        src = bufs[c]
        ms.grid_build(ws, *src)
        if ev is not None:
            ev[0].record()
        if sorted_state:
            ms.mech_step_integrate_sorted(ws, PARAMS, *src, state_out=bufs[1 - c], disp_out=out)
        elif ev is not None:
            # roofline pass: events around the displacement step alone
            ms.mech_step(ws, PARAMS, out=out)
        else:
            # rollout step: displacements written and added to the positions
            ms.mech_step_integrate(ws, PARAMS, *src[:3], out=out)
        if ev is not None:
            ev[1].record()
        if backward:
            ms.mech_step_backward(ws, PARAMS, *gin, out=gout, g_params=gkg)
        if ev is not None and not sorted_state:
            ms.integrate(*src[:3], *out)
        if sorted_state:
            cur[0] = 1 - c

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
        # one graph per state buffer (a sorted rollout alternates between two)
        graphs = []
        saved = cur[0]
        for c in range(len(bufs)):
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr):
                one(c=c)
            graphs.append(gr)
        cur[0] = saved                   # capturing executes nothing

        def replay():
            graphs[cur[0]].replay()
            if sorted_state:
                cur[0] = 1 - cur[0]

        for _ in range(max(warmup, 1)):
            replay()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            replay()
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
    for a_, b_ in zip(t, x0):
        a_.copy_(b_)
    return total, force_ms, ws, t


def time_rollout_grad(ms, torch, dtype, steps=50, ckpt=10, reps=5, seed=0):
    """The differentiation workload: 262,144 agents at ~12 neighbours, a
    `steps`-step rollout with checkpoints every `ckpt` steps, loss = mean
    squared distance of the final positions to seeded targets, gradients with
    respect to the initial positions, diameters, kappa and gamma.  Timed with
    events around the forward rollout plus its backward (segment recompute
    from the checkpoints and the accumulating backward steps)."""
    from paper_2105_00039_amd import autograd as msa, workloads
    pop = workloads.workload("adjoint262k", seed=seed)
    tgt = workloads.targets(pop, seed=seed)
    in_t = torch.float32 if dtype == "f32" else torch.float64
    rest = dict(dt=PARAMS["dt"], max_disp=PARAMS["max_disp"], adherence=PARAMS["adherence"])
    ws = ms.Workspace(pop.n, dtype=dtype)
    base = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda", in_t) for a in pop.arrays()]
    tx, ty, tz = (torch.from_numpy(np.asarray(a)).to("cuda", in_t) for a in tgt)

    def once():
        t = [a.clone().requires_grad_(True) for a in base]
        k = torch.tensor(PARAMS["kappa"], dtype=torch.float64, requires_grad=True)
        g = torch.tensor(PARAMS["gamma"], dtype=torch.float64, requires_grad=True)
        px, py, pz = msa.rollout(*t, k, g, ws, rest, steps, ckpt)
        L = ((px - tx) ** 2 + (py - ty) ** 2 + (pz - tz) ** 2).mean()
        L.backward()
        return L

    once()
    torch.cuda.synchronize()
    # each rollout timed on its own and the median reported: the eager
    # rollout issues ~1,000 launches from the host, and a stall of the host
    # thread now and then doubles one rollout's time
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        once()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    ms.device_status(ws)
    sec = float(np.median(times))
    return dict(value=pop.n * steps / sec, unit="agent-steps/s", ms_per_rollout=sec * 1e3,
                ms_per_rollout_min_max=[min(times) * 1e3, max(times) * 1e3], reps=reps,
                n_agents=pop.n, steps=steps, ckpt_every=ckpt, dtype=dtype,
                what="forward rollout + backward (recompute from checkpoints, accumulating "
                     "backward steps) per agent-step of the rollout; eager, events around "
                     "each rollout, median of the repetitions")


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


def time_batched(ms, torch, steps, warmup, seed=0, sorted_state=True):
    """The batched workload: 256 simulations in one build and one force
    launch per step, FP32 force with FP64 positions; graph-replayed steps
    (sorted_state: the state kept in the build's slot order, two buffers)."""
    from paper_2105_00039_amd import workloads
    b = workloads.batched(seed=seed)
    n = b.n
    ws = ms.Workspace(n, max_sims=b.n_sims, dtype="f32_pos64")
    t = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in b.arrays(np.float64)]
    bufs = [t, [torch.empty_like(a) for a in t]] if sorted_state else [t]
    cur = [0]
    spec = ms.BatchSpec(b.offsets)
    P = ms.params_tensor([dict(PARAMS, kappa=float(k), gamma=float(g)) for k, g in zip(b.kappa, b.gamma)],
                         "cuda")
    out = tuple(torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3))
    from paper_2105_00039_amd import autotune
    ms.grid_build_batched(ws, *t, spec)
    tuning = autotune.tune(ws, lambda: ms.mech_step_batched(ws, P, out=out))

    def one(c=None):
        c = cur[0] if c is None else c
        ms.grid_build_batched(ws, *bufs[c], spec)
        if sorted_state:
            ms.mech_step_batched_integrate_sorted(ws, P, *bufs[c], state_out=bufs[1 - c], disp_out=out)
            cur[0] = 1 - c
        else:
            ms.mech_step_batched_integrate(ws, P, *bufs[c][:3], out=out)

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
    graphs = []
    saved = cur[0]
    for c in range(len(bufs)):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            one(c=c)
        graphs.append(gr)
    cur[0] = saved

    def replay():
        graphs[cur[0]].replay()
        if sorted_state:
            cur[0] = 1 - cur[0]

    replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        replay()
    e.record()
    torch.cuda.synchronize()
    ms.device_status(ws)
    sec = a.elapsed_time(e) / 1e3
    return dict(value=n * steps / sec, unit="agent-steps/s", n_sims=b.n_sims, n_agents=n, steps=steps,
                ms_per_step=sec / steps * 1e3, dtype="f32 force, f64 positions",
                gather=dict(list=tuning["choice"][0], block=tuning["choice"][1],
                            walk=tuning["choice"][2]),
                state_order="box-sorted slot order" if sorted_state else "caller order",
                workload="batched256: sizes 10^U(3,5), 4-30 neighbours, kappa U[1,4], gamma U[0.5,2]")


def host_cpu():
    """CPU model, sockets, cores and NUMA nodes of the host (lscpu), and the
    CPUs this process may run on."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return dict(model=info.get("Model name", "unknown"), sockets=info.get("Socket(s)"),
                cores_per_socket=info.get("Core(s) per socket"),
                threads_per_core=info.get("Thread(s) per core"), numa_nodes=info.get("NUMA node(s)"),
                allowed_cpus=len(os.sched_getaffinity(0)))


def numa_node0_cpus():
    """CPUs of NUMA node 0 (sysfs), or None."""
    path = "/sys/devices/system/node/node0/cpulist"
    if not os.path.exists(path):
        return None
    cpus = set()
    for part in open(path).read().strip().split(","):
        if "-" in part:
            a, b = part.split("-")
            cpus.update(range(int(a), int(b) + 1))
        elif part:
            cpus.add(int(part))
    return cpus


def cpu_baseline(arrs, budget_s=8.0, max_steps=6):
    """The FP64 oracle timed on the host's cores, as the paper times its CPU
    baseline (Section V): the -O3 -march=native build, one thread, then
    OpenMP over the CPU share of this process (at most OMP_NUM_THREADS, else
    16), kept on one NUMA node when the host has several.  Each agent's sums
    are sequential in both, so the results are the same."""
    import oracle
    host = host_cpu()
    allowed = os.sched_getaffinity(0)
    node0 = numa_node0_cpus()
    pinned = False
    if host.get("numa_nodes") not in (None, "1") and node0 and (allowed & node0):
        os.sched_setaffinity(0, allowed & node0)      # before the OpenMP threads start
        pinned = True
    use = os.sched_getaffinity(0)
    threads = min(len(use), int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
    oracle.use_native()
    a64 = [np.asarray(a, dtype=np.float64) for a in arrs]
    n = a64[0].size

    def run(t):
        oracle.set_threads(t)
        done = 0
        t0 = time.perf_counter()
        while done < max_steps:
            oracle.step(*a64, PARAMS)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        return done, time.perf_counter() - t0

    d1, s1 = run(1)
    dn, sn = run(threads)
    if pinned:
        os.sched_setaffinity(0, allowed)
    return dict(value=n * dn / sn, unit="agent-steps/s", cores=threads, kind="oracle",
                single_thread_value=n * d1 / s1, host=dict(host, numa_pinned=pinned),
                build="gcc -O3 -march=native -ffp-contract=off -fopenmp",
                sample=f"full steps (grid + force + displacement) of the same {n}-agent population, "
                       f"FP64: {dn} step(s) on {threads} threads in {sn:.1f} s, {d1} step(s) on one "
                       f"thread in {s1:.1f} s")


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
    ap.add_argument("--gather", default=None, metavar="LIST/BLOCK/WALK",
                    help="with --profile-only: fixed launch shape of the gather (e.g. 32/64/lanes) "
                         "instead of the autotuner's pick, so that every profiling pass runs the "
                         "same kernel")
    ap.add_argument("--order", default="sorted", choices=["sorted", "caller"],
                    help="state order of the rollout: the build's slot order (sorted, the "
                         "headline) or the caller's order")
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
            b = time_batched(ms, torch, args.steps, args.warmup, sorted_state=args.order == "sorted")
            log(f"batched {b['n_sims']} simulations, {b['n_agents']} agents: {b['ms_per_step']:.3f} ms/step, "
                f"{b['value']:.3e} agent-steps/s, gather {b['gather']}")
            return
        if args.workload == "clusters16M":
            del pop, arrs
            cl = workloads.workload("clusters16M", seed=args.seed)
            arrs = [a.astype(np.float32) for a in cl.arrays()]
            args.dtype = "f32"
            log(f"workload clusters16M f32: {arrs[0].size} agents")
        fixed = None
        if args.gather:
            lst, nt, walk = args.gather.split("/")
            fixed = (int(lst), int(nt), walk)
        sec, fms, ws, _ = time_plain(ms, torch, arrs, args.dtype, args.steps, args.warmup, events=True,
                                     backward=args.backward, sorted_state=args.order == "sorted",
                                     gather=fixed)
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

    # headline: graph-replayed rollout steps on the box-sorted state
    sorted_head = args.order == "sorted"
    sec, _, ws, t = time_plain(ms, torch, arrs, args.dtype, args.steps, args.warmup, graph=True,
                               sorted_state=sorted_head)
    head_tuning = ws.tuning
    value = N * args.steps / sec
    log(f"graph {args.steps} steps ({args.order} state): {sec * 1e3 / args.steps:.3f} ms/step, "
        f"{value:.3e} agent-steps/s")
    # roofline of the force kernel: eager pass with events around each launch
    sec_e, force_ms, ws, t = time_plain(ms, torch, arrs, args.dtype, args.steps, args.warmup, events=True,
                                        sorted_state=sorted_head)
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
    fb = force_bytes(N, st["n_boxes"], S, sorted_head)
    prof = f"{name}_{args.dtype}" + ("_sorted" if sorted_head else "")
    issue = issue_from_profiles(prof)
    traffic = traffic_from_profiles(prof)
    # Which roof binds, from the committed counters of the current sources:
    # the share of the SIMD cycles the kernel spends issuing VALU
    # instructions against the share of the HBM peak its counted traffic
    # uses over the measured launch.  Without counters the bound stays the
    # arithmetic one the flop count is priced against.
    hbm_use = traffic / (force_ms * 1e-3) / HBM_PEAK if traffic else None
    bound = "alu"
    if issue and hbm_use is not None and hbm_use > issue["valu_issue_frac"]:
        bound = "hbm"
    roofline = dict(bound=bound, achieved=achieved / 1e12, peak=peak / 1e12, unit="TFLOP/s",
                    frac=achieved / peak, traffic=traffic, traffic_hbm_frac=hbm_use,
                    kernel=("k_force (ms_mech_step_integrate_sorted: gather, Eq. 1, displacement "
                            "and the state after the step in slot order)") if sorted_head else
                    "ms_mech_step = k_force + k_soa", flops_per_agent=flops_agent,
                    force_us=force_ms * 1e3,
                    force_alg_bytes=fb, force_alg_GBps=fb / (force_ms * 1e-3) / 1e9,
                    force_hbm_frac=fb / (force_ms * 1e-3) / HBM_PEAK,
                    issue=issue,
                    bound_evidence=(f"VALU issue {issue['valu_issue_frac']:.2f} of the SIMD cycles, "
                                    f"texture data unit busy {issue['td_busy_frac']:.2f} (rocprofv3 "
                                    "counters) against counted HBM traffic at "
                                    + (f"{hbm_use:.2f}" if hbm_use is not None else "an unmeasured share")
                                    + " of the HBM peak")
                    if issue else None)
    balg = bytes_alg(N, st["n_boxes"], S)
    hbm = dict(step_alg_bytes=balg, step_alg_GBps=balg * args.steps / sec / 1e9,
               frac_of_peak=balg * args.steps / sec / HBM_PEAK)
    log(f"C={st['candidates']:.1f} K={K:.2f} nbrs={st['neighbors']:.2f} boxes={st['n_boxes']} "
        f"force {achieved / 1e12:.1f} TF/s; step {hbm['step_alg_GBps']:.0f} GB/s alg")

    extras = {}
    if not args.no_extras:
        def plain(a, dt, **kw):
            sx, _, wx, _ = time_plain(ms, torch, a, dt, args.steps, args.warmup, graph=True,
                                      sorted_state=sorted_head, **kw)
            c = wx.tuning["choice"]
            return a[0].size * args.steps / sx, sx / args.steps * 1e3, dict(
                list=c[0], block=c[1], walk=c[2], box_order=wx.tuning["box_order"]["choice"])

        other = "f64" if args.dtype == "f32" else "f32"
        oarrs = [a.astype(np.float32 if other == "f32" else np.float64) for a in pop.arrays()]
        v, _, lst_ = plain(oarrs, other)
        extras[f"plain_{other}_n{args.neighbors:g}"] = v
        extras[f"plain_{other}_n{args.neighbors:g}_gather"] = lst_
        del oarrs
        for nb in (4.0, 30.0):
            p2 = workloads.uniform(N, mean_neighbors=nb, seed=args.seed)
            a2 = [a.astype(np_in) for a in p2.arrays()]
            v, _, lst_ = plain(a2, args.dtype)
            extras[f"plain_{args.dtype}_n{nb:g}"] = v
            extras[f"plain_{args.dtype}_n{nb:g}_gather"] = lst_
        # the same step with the state kept in the caller's order
        sc, _, _, _ = time_plain(ms, torch, arrs, args.dtype, args.steps, args.warmup, graph=True,
                                 sorted_state=not sorted_head)
        extras["caller_order" if sorted_head else "sorted_state"] = N * args.steps / sc
        # clustered workload: 16,777,216 agents in 64 Gaussian clusters, FP32
        cl = workloads.workload("clusters16M", seed=args.seed)
        carrs = [a.astype(np.float32) for a in cl.arrays()]
        del cl
        v, msps, lst_ = plain(carrs, "f32")
        extras["clusters16M_f32"] = v
        extras["clusters16M_f32_gather"] = lst_
        extras["clusters16M_f32_ms_per_step"] = msps
        del carrs
        torch.cuda.empty_cache()
        host_state = time_host_state(ms, torch, arrs, args.steps, args.warmup) \
            if args.dtype == "f32" else None
        growing = time_growing(ms, torch, args.steps, seed=args.seed)
        s4, _, _, _ = time_plain(ms, torch, arrs, args.dtype, args.steps, args.warmup, graph=True,
                                 backward=True)
        fwd_bwd = dict(value=N * args.steps / s4, unit="agent-steps/s", ms_per_step=s4 / args.steps * 1e3,
                       what="grid build + forward + backward + integrate, same workload, caller order "
                            "(the gradients are in the caller's order)")
        rollout_grad = time_rollout_grad(ms, torch, args.dtype)
        batched = time_batched(ms, torch, max(args.steps // 2, 2), args.warmup, sorted_state=sorted_head)
        batched["other_order_value"] = time_batched(ms, torch, max(args.steps // 2, 2), args.warmup,
                                                    sorted_state=not sorted_head)["value"]
        log(f"variants {extras}; fwd+bwd {fwd_bwd['value']:.3e}; rollout grad {rollout_grad['value']:.3e}; "
            f"batched {batched['value']:.3e}; host state {host_state}; growing {growing}")
    else:
        fwd_bwd = batched = host_state = growing = rollout_grad = None

    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline ...")
        cpu = cpu_baseline(arrs)
        log(f"oracle {cpu['value']:.3e} agent-steps/s")

    rec = {
        "metric": METRIC, "value": value, "unit": "agent-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": name, "state_order": "box-sorted slot order of each build (kept "
                   "across the rollout)" if sorted_head else "caller order",
                   "n_agents": N, "mean_neighbors_target": args.neighbors,
                   "measured_neighbors": st["neighbors"], "contacts_per_agent": K,
                   "candidates_per_agent": st["candidates"], "n_boxes": st["n_boxes"],
                   "diameters": "U[8,12]", "params": PARAMS, "graph": True,
                   "gather": dict(list=head_tuning["choice"][0], block=head_tuning["choice"][1],
                                  walk=head_tuning["choice"][2]),
                   "gather_ms": head_tuning["ms"],
                   "box_order": head_tuning["box_order"]["choice"],
                   "box_order_ms": head_tuning["box_order"]["ms"]},
        "roofline": roofline, "hbm": hbm, "cpu_baseline": cpu,
        "variants": extras, "fwd_bwd": fwd_bwd, "rollout_grad_adjoint262k": rollout_grad,
        "batched": batched, "host_state": host_state, "growing_population": growing,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
