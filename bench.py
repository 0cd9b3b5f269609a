"""hPF-MD throughput benchmark on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c3]

A step is one pass of the whole hot path over the synthetic workload:
velocity-Verlet half kick + drift + wrap, the cell sort (every
``--sort-every`` steps), density scatter, field potential, field gradient,
force gather, bond forces, second half kick, and the FP64 energy / momentum
reductions. Inputs are resident in HBM before the timed region starts.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "hPF-MD particle-steps/s at 1M & 10M beads; %HBM peak; batched vs plain speedup"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(name: str, N: int, K: int, nm: int, D: int) -> float:
    """Bytes a kernel must move per launch on the method's minimal data (FP32 x, v; uint8
    types; 4-byte bond-partner slots; uint64 counts; FP32 V), each array read or written once.

    The fused depositing pass "advance" does the gather, bonds and both Verlet halves and
    deposits x_{n+1}: x, v, T read and x, v written (49 B per bead), the two bond-partner
    slots (8 B), and per mesh point and species V read (4 B) and the count flush (8 B).
    "finish_potential" reads and clears the counts (16 B) and writes V (4 B). Together
    with the deposit read of x, T (13 B) that the fusion saves, these are the two-pass step
    bytes 70 N + 32 K M^3. The gradient has no minimal-design bytes (the minimal pass reads
    V at the corners instead); its entry, like those of the six separate calls, is at the
    API level (their sum is 178 N + 56 K M^3)."""
    return {
        "verlet_half1": 60.0 * N,                   # x, v read + written; F read
        "density_scatter": 13.0 * N + 8.0 * K * nm,  # x, T read; counts written once
        "density_finish": 8.0 * K * nm,
        "finish_potential": 20.0 * K * nm,
        "field_potential": 20.0 * K * nm,            # counts read + cleared; V written
        "field_gradient": 16.0 * K * nm,             # V read; gradient (3 x FP32) written
        "force_gather": 25.0 * N + 12.0 * K * nm,    # x, T read; F written; gradient read
        "bond_forces": 36.0 * N + 4.0 * D * N,       # x, bond table, F read; F written
        "verlet_half2": 36.0 * N,                    # v read + written; F read
        "advance": 57.0 * N + 12.0 * K * nm,
        "reduce": 6 * 4096 * 8.0,
    }[name]


def layout_bytes(name: str, N: int, K: int, nm: int, D: int, P: int, nbricks: int) -> float:
    """Bytes the kernel moves by its data layout: 12-byte bead rows (x, v), the gradient mesh
    (12 B per point and species, read in place of V), and the partial deposit boxes of
    K P^3 uint64 per brick that the depositing pass writes and the finish reads."""
    box = 8.0 * K * P ** 3 * nbricks
    return {
        "advance": (49.0 + 4.0 * D) * N + 12.0 * K * nm + box,
        "finish_potential": 20.0 * K * nm + box,
        "field_gradient": 16.0 * K * nm,
    }.get(name)


class Timers:
    """HIP events around every call of the step, on torch's current stream
    (the stream the library launches on)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}

    def wrap(self, name, fn, *a, **kw):
        ev0 = self.torch.cuda.Event(enable_timing=True)
        ev1 = self.torch.cuda.Event(enable_timing=True)
        ev0.record()
        fn(*a, **kw)
        ev1.record()
        self.pairs.setdefault(name, []).append((ev0, ev1))

    def summary(self):
        out = {}
        for k, v in self.pairs.items():
            ts = [a.elapsed_time(b) for a, b in v]
            out[k] = {"avg_us": 1e3 * sum(ts) / len(ts), "launches": len(ts)}
        return out


def timed_step(st, hpf, engine, tm, sort):
    import torch  # noqa: F401
    tm.wrap("verlet_half1", hpf.verlet_step, st.R, st.Vel, st.F, st.dt, st.box, 1)
    if sort:
        tm.wrap("sort_by_cell", st.sort)
    tm.wrap("density_scatter", st.scatter)
    tm.wrap("field_potential", hpf.hpf_field_potential, st.counts, st.mesh, st.field, st.V,
            st.part[engine.ROW_W])
    tm.wrap("field_gradient", hpf.hpf_field_gradient, st.V, st.mesh, st.K, st.G)
    tm.wrap("force_gather", hpf.hpf_force_gather, st.R, st.T, st.mesh, st.K, st.G, st.F)
    tm.wrap("bond_forces", hpf.bond_forces, st.R, st.bonds, st.k_bond, st.r0, st.box, st.F,
            st.part[engine.ROW_EB])
    tm.wrap("verlet_half2", hpf.verlet_step, None, st.Vel, st.F, st.dt, st.box, 2,
            kin_part=st.part[engine.ROW_KE:engine.ROW_KE + 4])
    tm.wrap("reduce", hpf.hpf_reduce_partials, st.part, engine.N_ROWS, st.energy)
    st.steps_done += 1


def timed_step_fused(st, hpf, engine, tm, sort):
    if sort:
        tm.wrap("sort_by_cell", st.sort)
    if st.density_pending:
        tm.wrap("finish_potential", st.potential, True)
    else:
        tm.wrap("density_scatter", st.scatter)
        tm.wrap("field_potential", hpf.hpf_field_potential, st.counts, st.mesh, st.field, st.V,
                st.part[engine.ROW_W])
    tm.wrap("field_gradient", hpf.hpf_field_gradient, st.V, st.mesh, st.K, st.G)
    tm.wrap("advance", st.advance, True)
    tm.wrap("reduce", hpf.hpf_reduce_partials, st.part, engine.N_ROWS, st.energy)
    st.steps_done += 1


def replay_segments(st, one, steps, period, torch, engine, max_graphs=64):
    """Time `steps` steps replayed from HIP graphs; None if no segment split fits.

    One period of the step pattern returns every buffer swap to its start. It is cut into
    segments of gcd(steps, period) steps, each captured as one graph; the timed region
    replays the segments in order, steps / seg of them. The host-side stepping state is then
    put back to where the replays left the device."""
    seg = math.gcd(steps, period)
    nseg = period // seg
    if nseg > max_graphs:
        return None
    snaps, graphs = [], []
    for _ in range(nseg):
        snaps.append(st.snapshot())
        graphs.append(engine.Graph(lambda: [one() for _ in range(seg)]))
    # after capture the host state is one period ahead of the device (same buffers)
    base = st.snapshot()
    # every segment replays on one stream, so that they run in order
    stream = graphs[0].stream
    for g in graphs:                                 # untimed first replay of every segment
        g.launch(stream)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    n = steps // seg
    wall0 = time.perf_counter()
    t0.record(stream)
    for j in range(n):
        graphs[j % nseg].launch(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    done = snaps[n % nseg]
    done = dict(done, steps_done=done["steps_done"] + (base["steps_done"] - snaps[0]["steps_done"]) *
                (1 + n // nseg))
    st.restore(done)
    del graphs
    return ms, wall, seg, nseg


def run_workload(cfg, steps, warmup, sort_every, instrument=True, fused=True, graph=True, halo=2,
                 advance="scatter", field_every=1, thermostat=0.0, brick=0):
    """Warm up, time `steps` steps, then (instrument) time each call over one period of
    eager steps. With `graph`, the timed steps replay HIP graphs (replay_segments)."""
    import torch

    from paper_1310_2041_amd import engine, hpf
    from synth import workloads as wl

    spec = wl.SPECS[cfg]
    s = wl.build(spec)
    KEEP_SYSTEMS.setdefault(cfg, [s]) if cfg in KEEP_SYSTEMS_FOR else None
    st = engine.HpfState.from_system(s, halo=halo, advance=advance, field_every=field_every,
                                     sort_brick=brick)
    if thermostat > 0.0:
        st.set_thermostat(thermostat, seed=13102041 + spec.index)
    del s
    st.start(sort=True)
    if fused:
        st.prime()
    step = st.step_fused if fused else st.step

    def one(report=True):
        step(report=report, sort=sort_every > 0 and st.steps_done % sort_every == 0)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    # the step pattern repeats after two sort intervals and after the field interval
    period = math.lcm(2 * sort_every if sort_every > 0 else 2, field_every)
    rep = replay_segments(st, one, steps, period, torch, engine) if graph else None
    if rep is not None:
        ms, wall, seg, nseg = rep
        launch = {"mode": "hip_graph", "steps_per_graph": seg, "graphs": nseg}
    else:
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record()
        for _ in range(steps):
            one()
        t1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms = t0.elapsed_time(t1)
        launch = {"mode": "eager"}
    tm = Timers(torch)
    if instrument:
        for _ in range(period):
            do_sort = sort_every > 0 and st.steps_done % sort_every == 0
            (timed_step_fused if fused else timed_step)(st, hpf, engine, tm, do_sort)
        torch.cuda.synchronize()
    flags = hpf.hpf_get_device_status()
    e = st.energies()
    nb = 1
    for d in range(3):
        nb *= -(-st.mesh.M[d] // st.B)
    return {"spec": spec, "N": st.N, "K": st.K, "nm": st.nm, "D": st.bonds.shape[0],
            "B": st.B, "P": st.B + 1 + 2 * st.halo, "nbricks": nb,
            "ms_total": ms, "wall_s": wall, "kernels": tm.summary() if instrument else {},
            "flags": flags, "energies": e, "launch": launch,
            "advance_kernel": "scatter" if st.uses_scatter_advance() else "plain"}


def run_composition(steps=40, sort_every=20):
    """The composition list (MD-SCF section) on a dilute five-species system: 10,000 lipids
    (12 beads, species 0-3) in 1,080,000 waters (species 4), 1.2M beads. Whole steps (the
    six calls with angles, sorted every `sort_every`, replayed from a HIP graph) and the
    gradient pass alone, each with and without the list. The beads move identically either
    way; the list only skips the gradient of species absent from a mesh point."""
    import torch

    from paper_1310_2041_amd import engine, hpf
    from synth import workloads as wl

    s = wl.lipid_system(10000, 1080000)
    out = {"workload": "lipid_k5_dilute_1.2m", "beads": s.N, "species": s.K, "mesh": list(s.M)}
    for name, listed in (("all_species", False), ("listed", True)):
        st = engine.HpfState.from_system(s, composition_list=listed)
        st.start(sort=True)

        def seg():
            for _ in range(steps):
                st.step(report=True, sort=sort_every > 0 and st.steps_done % sort_every == 0)

        g = engine.Graph(seg)
        g.launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(g.stream)
        g.launch()
        e1.record(g.stream)
        torch.cuda.synchronize()
        step_ms = e0.elapsed_time(e1) / steps
        del g
        e0.record()
        for _ in range(20):
            hpf.hpf_field_gradient(st.V, st.mesh, st.K, st.G, present=st.present)
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"ms_per_step": step_ms, "gradient_us": e0.elapsed_time(e1) / 20 * 1e3}
        if listed:
            pr = st.present.cpu().numpy()
            out["absent_point_species_fraction"] = float(
                1.0 - sum(((pr >> k) & 1).mean() for k in range(s.K)) / s.K)
        del st
    out["note"] = ("six-call steps with angles (the fused passes take bonds only), graph-replayed; "
                   "gradient_us: the gradient pass alone")
    return out


def run_batched_sweep(replays=5, sort_every=10, tune=True):
    """64 uneven A10B10 replicas: batched entry points vs one single-system call chain
    per replica, both with the sort interval the tuner picks, captured in HIP graphs of two
    sort intervals (at least 20 steps, so every buffer swap returns) and replayed."""
    import torch

    from paper_1310_2041_amd import engine
    from synth import workloads as wl

    specs = wl.replica_specs()
    systems = [wl.build_replica(sp, r) for r, sp in enumerate(specs)]
    KEEP_SYSTEMS.setdefault("c4", systems) if "c4" in KEEP_SYSTEMS_FOR else None
    n_beads = sum(s.N for s in systems)

    batch = engine.BatchState(systems, sort_every=sort_every)
    batch.start()
    chosen, trials = (batch.tune(trial_steps=20) if tune else (None, []))
    if chosen:
        sort_every = chosen["sort_every"]
    steps_per_graph = math.lcm(2 * sort_every, 20)
    torch.cuda.synchronize()

    def time_graph(g):
        g.launch()                                   # warm-up replay
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(g.stream)
        for _ in range(replays):
            g.launch()
        e1.record(g.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / (replays * steps_per_graph)

    # the batch's step count is 0 here (after start or tuning): the graph begins with a sort
    gb = engine.Graph(lambda: batch.step(steps_per_graph, report_last=True))
    ms_batched = time_graph(gb)
    del gb

    states = [engine.HpfState.from_system(s) for s in systems]
    for st in states:
        st.start(sort=True)
        st.prime()
    torch.cuda.synchronize()

    def plain():
        for i in range(steps_per_graph):
            for st in states:
                st.step_fused(report=(i == steps_per_graph - 1),
                              sort=sort_every > 0 and st.steps_done % sort_every == 0)

    gp = engine.Graph(plain)
    ms_plain = time_graph(gp)
    del gp
    srt = sorted(trials)
    return {"workload": "c4_64_replica_a10b10_sweep", "replicas": len(systems), "beads": n_beads,
            "batched_value": n_beads / (ms_batched * 1e-3), "plain_value": n_beads / (ms_plain * 1e-3),
            "batched_ms_per_step": ms_batched, "plain_ms_per_step": ms_plain,
            "speedup": ms_plain / ms_batched, "tuned": chosen,
            "tune_trial_ms": [round(t, 4) for t in trials],
            "tune_margin": round(srt[1] / srt[0] - 1.0, 4) if len(srt) > 1 else None,
            "tune_vs_median": round(srt[len(srt) // 2] / srt[0] - 1.0, 4) if srt else None,
            "tune_vs_worst": round(srt[-1] / srt[0] - 1.0, 4) if srt else None,
            "note": "both paths replayed from HIP graphs of %d steps, sort every %d" %
                    (steps_per_graph, sort_every)}


# rocprofv3 kernel names behind each timed call of the step: a template name stands for
# every instantiation of that kernel ("name<"), a plain name for itself
ROCPROF_KERNELS = {
    "advance": ["hpf::k_advance<", "hpf::k_advance_scatter<"],
    "density_scatter": ["hpf::k_zero_u32_one", "hpf::k_scatter_bricks", "hpf::k_scatter_sum<false>",
                        "hpf::k_scatter_strays"],
    "density_finish": ["hpf::k_scatter_sum<true>"],
    "finish_potential": ["hpf::k_finish_potential<"],
    "field_potential": ["hpf::k_field_potential<"],
    "field_gradient": ["hpf::k_field_gradient"],
}


def rocprof_matches(pattern: str, name: str) -> bool:
    return name.startswith(pattern) if pattern.endswith("<") else name == pattern


def step_bandwidth(r, ms_step):
    """The whole step against the HBM peak on the two-pass step bytes 70 N + 32 K M^3: the
    least a design with one pass over the beads and one over the mesh must move (x, T read
    by the deposit 13 B, x, v, T read and x, v written by the force + integration pass 49 B,
    bond-partner slots 8 B per bead; per mesh point and species the counts written, read
    and cleared 24 B and V written and read 8 B). The sort and the gradient are not in it."""
    N, K, nm = r["N"], r["K"], r["nm"]
    b_min = 70.0 * N + 32.0 * K * nm
    gmin = b_min / (ms_step * 1e-3) / 1e9
    return {"bytes_per_step": b_min, "achieved": round(gmin, 1), "unit": "GB/s",
            "peak": HBM_PEAK_GBS, "frac": round(gmin / HBM_PEAK_GBS, 4),
            "note": "two-pass step bytes 70 N + 32 K M^3 over the whole measured step time"}


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary of
    `workload`, or None when there is none or the kernel sources changed since."""
    from paper_1310_2041_amd.profile_summary import read_record, source_hash
    d = read_record(os.path.join(ROOT, "profiles", f"{workload}_step.md"))
    if d is None or d.get("source_hash") != source_hash():
        return None
    tot, found = 0.0, False
    for name, e in d["kernels"].items():
        if not any(rocprof_matches(p, name) for p in ROCPROF_KERNELS.get(kernel, [])):
            continue
        if e.get("fetch_bytes") is not None and e.get("write_bytes") is not None:
            tot += e["fetch_bytes"] + e["write_bytes"]
            found = True
    return tot if found else None


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(cfg, n_steps):
    """The FP64 oracle on a bounded sample of the workload: one host thread (the parity
    build), and all the threads this process may use (the same source built with OpenMP)."""
    import oracle
    from synth import workloads as wl

    s = wl.build(wl.SPECS[cfg])
    threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))

    def timed(th):
        t0 = time.perf_counter()
        oracle.forces(s) if th is None else oracle.run(s, 0, threads=th)
        t_force = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.run(s, n_steps, threads=th)
        t_run = time.perf_counter() - t0
        return max(t_run - t_force, 1e-9)      # run() evaluates the initial forces first

    t1 = timed(None)
    tn = timed(threads)
    info = cpu_info()
    return {"value": s.N * n_steps / tn, "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle",
            "single_thread_value": s.N * n_steps / t1,
            "cpu": info,
            "sample": f"{n_steps} velocity-Verlet steps of the full {s.N}-bead {cfg} workload, FP64 C "
                      f"oracle: {tn:.1f} s on {threads} threads (OpenMP build of the same source), "
                      f"{t1:.1f} s on one thread; host {info['model']}, nproc {info['nproc']}"}


# host systems that the GPU runs built, kept for the oracle timings (filled when the oracle
# timings are requested, so that C4 and C5 are not built twice)
KEEP_SYSTEMS_FOR = set()
KEEP_SYSTEMS = {}


def oracle_timings(threads=None):
    """The FP64 oracle on every other workload, on all the threads this process may use:
    C1 and C2 for 100 steps, the 64 C4 replicas for 10 steps each, C5 for one step; C1 also
    on one thread. Each figure is the time of run(n) less that of run(0) (the initial force
    evaluation and set-up), both after an untimed run(0) except for C5."""
    import oracle
    from synth import workloads as wl

    threads = threads or int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))

    def timed(systems, n_steps, th):
        total = 0.0
        for s in systems:
            if s.N <= 10_000_000:
                oracle.run(s, 0, threads=th)          # untimed: first-touch of its buffers
            t0 = time.perf_counter()
            oracle.run(s, 0, threads=th)
            t_force = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.run(s, n_steps, threads=th)
            total += max(time.perf_counter() - t0 - t_force, 1e-9)
        return total

    out = {}
    for cfg, n_steps in (("c1", 100), ("c2", 100), ("c4", 10), ("c5", 1)):
        systems = KEEP_SYSTEMS.pop(cfg, None)
        if systems is None and cfg == "c4":
            systems = [wl.build_replica(sp, r) for r, sp in enumerate(wl.replica_specs())]
        elif systems is None:
            systems = [wl.build(wl.SPECS[cfg])]
        n = sum(s.N for s in systems)
        t = timed(systems, n_steps, threads)
        row = {"beads": n, "steps": n_steps, "seconds": round(t, 3), "threads": threads,
               "value": n * n_steps / t, "unit": "particle-steps/s"}
        if cfg == "c1":
            t1 = timed(systems, n_steps, None)
            row["single_thread_value"] = n * n_steps / t1
        out[cfg] = row
        del systems
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_table(r):
    kern = r["kernels"]
    out = {}
    for name, k in kern.items():
        if name == "sort_by_cell":
            out[name] = {"avg_us": round(k["avg_us"], 2), "launches": k["launches"]}
            continue
        b = algorithmic_bytes(name, r["N"], r["K"], r["nm"], r["D"])
        out[name] = {"avg_us": round(k["avg_us"], 2), "alg_GBs": round(b / (k["avg_us"] * 1e-6) / 1e9, 1)}
    return out


def roofline(r, name):
    avg_us = r["kernels"][name]["avg_us"]
    b = algorithmic_bytes(name, r["N"], r["K"], r["nm"], r["D"])
    lb = layout_bytes(name, r["N"], r["K"], r["nm"], r["D"], r["P"], r["nbricks"])
    achieved = b / (avg_us * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(r["spec"].name, name),
            "algorithmic_bytes": b, "avg_us": round(avg_us, 2),
            "layout_bytes": lb,
            "layout_frac": None if lb is None else round(lb / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "note": "achieved = minimal algorithmic bytes per launch / average launch time (HIP events "
                    "on the launch stream); layout_bytes = what this kernel's data layout moves "
                    "(12-byte bead rows and gradient corners, partial deposit boxes); "
                    "traffic = rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, calibrated"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--also", default="c2", help="second workload reported under 'also' ('' = none)")
    ap.add_argument("--sort-every", type=int, default=30)
    ap.add_argument("--mode", default="fused", choices=["fused", "api"],
                    help="fused: hpf_advance; api: the six separate calls")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-replica batched sweep")
    ap.add_argument("--no-composition", action="store_true",
                    help="skip the composition-list comparison on the dilute five-species system")
    ap.add_argument("--c5-steps", type=int, default=120,
                    help="steps of the 100M-bead three-species system reported under 'c5' (0 = skip)")
    ap.add_argument("--halo", type=int, default=2, help="drift halo (cells) of the brick deposit boxes")
    ap.add_argument("--brick", type=int, default=0,
                    help="sort brick edge in cells (3..16); 0 = the engine's choice for the mesh")
    ap.add_argument("--advance", default="scatter", choices=["scatter", "plain"],
                    help="fused pass on cell-sorted beads (scatter: with the density deposit)")
    ap.add_argument("--eager", action="store_true",
                    help="launch every call from Python instead of replaying HIP graphs")
    ap.add_argument("--field-interval", type=int, default=10,
                    help="also time the workload with the density field rebuilt every n steps "
                         "(the MD-SCF update interval; 0 = skip)")
    ap.add_argument("--thermostat", type=float, default=5.0,
                    help="Andersen collision rate of the field-interval run (0 = NVE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hPF-MD path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    fused = args.mode == "fused"
    if not args.no_cpu_baseline:
        KEEP_SYSTEMS_FOR.update({"c4", "c5"})
    log(f"{args.config}: {args.warmup} warm-up + {args.steps} timed steps")
    r = run_workload(args.config, args.steps, args.warmup, args.sort_every, fused=fused,
                     graph=not args.eager, halo=args.halo, advance=args.advance,
                     brick=args.brick)
    ms_step = r["ms_total"] / args.steps
    value = r["N"] * args.steps / (r["ms_total"] * 1e-3)
    per_kernel = kernel_table(r)
    dom = max((n for n in per_kernel if n != "sort_by_cell"), key=lambda n: per_kernel[n]["avg_us"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u64",
        "data": "synthetic",
        "config": {"workload": r["spec"].name, "beads": r["N"], "species": r["K"],
                   "mesh": [r["spec"].M] * 3, "box": r["spec"].L, "sort_every": args.sort_every,
                   "energy_report_every": 1, "step": args.mode, "advance": r["advance_kernel"],
                   "halo": args.halo, "brick": r["B"], "launch": r["launch"],
                   "parallelism": "single-gpu"},
        "roofline": roofline(r, dom),
        "step_roofline": step_bandwidth(r, ms_step),
        "kernels": per_kernel,
        "device_flags": r["flags"],
    }
    if "finish_potential" in r["kernels"]:
        out["roofline_finish_potential"] = roofline(r, "finish_potential")
    log(f"{args.config}: {ms_step:.4f} ms/step")
    if args.also and args.also != args.config:
        r2 = run_workload(args.also, args.steps, args.warmup, args.sort_every, instrument=False,
                          fused=fused, graph=not args.eager, halo=args.halo, advance=args.advance,
                     brick=args.brick)
        ms2 = r2["ms_total"] / args.steps
        out["also"] = {"workload": r2["spec"].name, "beads": r2["N"], "brick": r2["B"],
                       "value": r2["N"] * args.steps / (r2["ms_total"] * 1e-3),
                       "ms_per_step": ms2, "launch": r2["launch"],
                       "step_roofline": step_bandwidth(r2, ms2),
                       "note": "working set fits the 256 MB Infinity Cache"}
        log(f"{args.also}: {ms2:.4f} ms/step")
    if args.field_interval > 1 and fused:
        r3 = run_workload(args.config, args.steps, args.warmup, args.sort_every, instrument=False,
                          fused=True, graph=not args.eager, halo=args.halo, advance=args.advance,
                          field_every=args.field_interval, thermostat=args.thermostat, brick=args.brick)
        out["field_interval"] = {"workload": r3["spec"].name, "field_every": args.field_interval,
                                 "thermostat_rate": args.thermostat,
                                 "value": r3["N"] * args.steps / (r3["ms_total"] * 1e-3),
                                 "ms_per_step": r3["ms_total"] / args.steps, "launch": r3["launch"],
                                 "ke_per_bead_end": float(r3["energies"]["KE"]) / r3["N"],
                                 "ke_per_bead_end_every_step": float(r["energies"]["KE"]) / r["N"],
                                 "note": "density field rebuilt every field_every steps (MD-SCF), "
                                         "Andersen thermostat at kT = 1 with the given collision rate; "
                                         "value above rebuilds it every step (NVE)"}
        log(f"field interval {args.field_interval}: {r3['ms_total'] / args.steps:.4f} ms/step")
    if args.c5_steps > 0:
        log(f"c5: building the 100M-bead system, {args.warmup} warm-up + {args.c5_steps} steps")
        r5 = run_workload("c5", args.c5_steps, args.warmup, args.sort_every, instrument=True,
                          fused=fused, graph=not args.eager, halo=args.halo, advance=args.advance,
                     brick=args.brick)
        ms5 = r5["ms_total"] / args.c5_steps
        out["c5"] = {"workload": r5["spec"].name, "beads": r5["N"], "species": r5["K"], "brick": r5["B"],
                     "mesh": [r5["spec"].M] * 3, "steps": args.c5_steps,
                     "value": r5["N"] / (ms5 * 1e-3), "ms_per_step": ms5, "launch": r5["launch"],
                     "step_roofline": step_bandwidth(r5, ms5),
                     "roofline": roofline(r5, max((n for n in r5["kernels"] if n != "sort_by_cell"),
                                                  key=lambda n: r5["kernels"][n]["avg_us"])),
                     "kernels": kernel_table(r5), "device_flags": r5["flags"]}
        del r5
        log(f"c5: {ms5:.4f} ms/step")
    if not args.no_composition:
        log("composition list: dilute five-species system")
        out["composition_list"] = run_composition()
    if not args.no_batch:
        log("64-replica batched sweep")
        out["batched_sweep"] = run_batched_sweep()
    if not args.no_cpu_baseline:
        log(f"oracle on the host: {args.cpu_steps} steps of {args.config}")
        out["cpu_baseline"] = cpu_baseline(args.config, args.cpu_steps)
        log("oracle on the host: c1, c2, c4, c5")
        out["cpu_baseline"]["other_workloads"] = oracle_timings(out["cpu_baseline"]["cores"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
