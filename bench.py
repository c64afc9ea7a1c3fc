"""Benchmark of SMMO execution on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload spring|gol|nbody]

Default workload: the spring-mass structure of 1,000,000 nodes and 2,996,001
springs (1000 x 1000 jittered grid, stiffness log-uniform in [1e2, 1e4],
rest length = initial distance, float32, dt 1e-5, springs deleted past
strain 0.3).  One step = one pass of the hot path over the whole mesh:
parallel_do(Spring, spring.force) (Hooke force, breaking springs delete
themselves) and parallel_do(Node, spring.node_update).  The timed K steps
end at step 10,000 of the workload where the untimed probe steps and the W
warm-up steps fit before them (else they start right after those: the
default, K = 10,000); the steps in between bring the mesh to that point.
All inputs are resident in HBM before the timed region.

Prints one JSON line: object-method updates per second (live objects
processed by the do-alls, summed over launches, per second), the dominant
kernel's roofline (algorithmic bytes per launch / HIP-event-timed launch
duration, against 8 TB/s), and the CPU oracle timed on a bounded sample.
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "object-method updates/sec + HBM GB/s % peak; batched & adjoint vs plain"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3
COUNTERS_FILE = os.path.join(HERE, "profiles", "spring_counters.json")
SEG_MIN_STEPS = 100      # shortest event-bounded segment inside the timed steps


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=["spring", "gol", "nbody"], default="spring")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gol-form", choices=["three", "fused"], default="three",
                    help="--workload gol: the three do-alls per generation, or gol.generation")
    ap.add_argument("--kernel-steps", type=int, default=50,
                    help="steps timed per kernel with HIP events for the roofline")
    ap.add_argument("--cpu-steps", type=int, default=None)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with three plain 512 MiB device copies (reference for rocprofv3 byte counters)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR_OR_JSON",
                    help="FETCH_DIR WRITE_DIR [FETCH_JSON WRITE_JSON]: summarize two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this bench (and their JSON lines, to keep only the "
                         "timing-window dispatches) into profiles/spring_counters.json; needs no GPU")
    ap.add_argument("--counter-pass", metavar="BENCH_JSON",
                    help="profiling aid: replay the state of the given bench run's timing window "
                         "(for rocprofv3 --pmc)")
    ap.add_argument("--alloc-pass", action="store_true",
                    help="profiling aid: short runs of the allocator-bound kernels (for rocprofv3 --pmc)")
    ap.add_argument("--summarize-l2", nargs="+", metavar="DIR",
                    help="L2 hit rate and atomic counts per kernel from rocprofv3 --pmc runs; needs no GPU")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and adjoint measurements")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "BENCH_JSON"),
                    help="compare rocprofv3 --kernel-trace durations of a run of this bench with the "
                         "per-kernel times it printed (BENCH_JSON: its output line); needs no GPU")
    ap.add_argument("--launch", action="append", default=[], metavar="METHOD=WG,WAVES,GROUP",
                    help="in the measurements that tune the spring step on a heap of their own (spring_2000, "
                         "batched), use this launch shape instead of tuning (give spring.force and "
                         "spring.node_update; for counter passes that must run the shapes an earlier run picked)")
    ap.add_argument("--extra", choices=sorted(STANDALONE_EXTRAS),
                    help="run one of the other measurements alone and print its JSON (for profiling it)")
    ap.add_argument("--graph-steps", type=int, default=50,
                    help="steps per captured HIP graph in the timed region, at most half the timed steps "
                         "(0 = eager launches)")
    return ap.parse_args()


# launch shapes given on the command line (--launch), used instead of tuning
GIVEN_SHAPES = {}

# the measurements besides the headline, by the name they have in the output
# line (batched and adjoint give no ratio to the headline's rate alone)
STANDALONE_EXTRAS = {"batched": "measure_batched", "adjoint": "measure_adjoint",
                     "copy_bandwidth": "measure_copy_bandwidth", "coalescing": "measure_coalescing",
                     "allocation": "measure_allocation", "enumeration": "measure_enumeration",
                     "gol": "measure_gol_extra", "gol_16384": "measure_gol_large", "structure": "measure_structure",
                     "generation": "measure_generation", "partial_inlining": "measure_spring_pi",
                     "spring_2000": "measure_spring_large", "nbody": "measure_nbody_extra",
                     "linux_scalability": "measure_linux_scalability", "wator": "measure_wator"}


def events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


# the files the spring kernels are compiled from (and the build flags); for
# the method header only its spring-mass section counts
SPRING_KERNEL_SOURCES = ("paper_1908_05845_amd/csrc/spring.hip", "paper_1908_05845_amd/csrc/method_common.hpp",
                         "paper_1908_05845_amd/csrc/smmo_device.hpp", "paper_1908_05845_amd/csrc/smmo_layout.hpp",
                         "include/smmo_methods.h", "paper_1908_05845_amd/build.py")
SPRING_HEADER_SECTION = ("/* ---- spring-mass mesh", "} smmo_spring_args;")


def kernel_source_hash():
    """Hash of the spring kernels' sources: a counter summary taken from
    other sources is not reported as these kernels' traffic."""
    import hashlib

    import re

    h = hashlib.sha256()
    for fn in SPRING_KERNEL_SOURCES:
        with open(os.path.join(HERE, fn)) as f:
            text = f.read()
        if fn.endswith("smmo_methods.h"):
            a = text.index(SPRING_HEADER_SECTION[0])
            text = text[a:text.index(SPRING_HEADER_SECTION[1], a) + len(SPRING_HEADER_SECTION[1])]
        # comments and blank lines do not change the compiled kernels
        if fn.endswith(".py"):
            text = re.sub(r"#[^\n]*", "", text)
        else:
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())
        h.update(fn.encode())
        h.update(code.encode())
    return h.hexdigest()[:16]


def traffic_for(kernel, state):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if there is none for this kernel, the sources changed since, or the
    counters were taken at another mesh state (steps before the timing pass
    and live springs there) than `state`."""
    try:
        with open(COUNTERS_FILE) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("source_hash") != kernel_source_hash() or c.get("state") != state:
        return None
    k = c.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


# ------------------------------------------------------------------ spring --
def bench_spring(args, torch):
    import numpy as np

    from inputs import spring_mesh
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.sims import SpringSim

    W = H = 1000
    dt, limit = 1e-5, 0.3
    total = 10_000                      # the workload's steps
    steps = total if args.steps is None else args.steps
    warmup = 20 if args.warmup is None else args.warmup
    mesh = spring_mesh(W, H)
    sim = SpringSim(mesh, dt, limit)
    heap = sim.heap
    lib = smmo.load_library()
    stream = torch.cuda.current_stream().cuda_stream
    hp, cs, cn = heap.h, heap.cls["Spring"], heap.cls["Node"]
    mf, mn = sim.m_force, sim.m_node
    argp = smmo.C.byref(sim.args)
    asz = smmo.C.sizeof(sim.args)

    # dispatches of each kernel issued so far (graph replays included), so
    # that a rocprofv3 trace of this run can be cut at the same launches
    count = {"spring.force": 0, "spring.node_update": 0}

    def step(st=stream):
        lib.smmo_parallel_do(hp, cs, mf, argp, asz, st)
        lib.smmo_parallel_do(hp, cn, mn, argp, asz, st)

    def counted(n):
        count["spring.force"] += n
        count["spring.node_update"] += n

    heap.sync()
    frozen0 = smmo.smmo_spring_args(sim.args.node_class, sim.args.spring_class, 0.0, sim.args.strain_limit,
                                    sim.args.flags)
    tuned = None
    if not args.no_autotune:
        from paper_1908_05845_amd import autotune

        # Candidates are timed on whole frozen steps (the force pass, then the
        # node pass with dt = 0: the traffic of a real step, the state
        # unchanged), one kernel at a time with the other at its current
        # shape: each kernel evicts part of the other's inputs from the L2
        # and MALL, so shapes tuned on a kernel alone need not help a step.
        groups = (1, 2, 4)
        fz = smmo.C.byref(frozen0)
        n_frozen = [0]

        def frozen_steps(n=30, warm=3):
            for _ in range(warm):
                lib.smmo_parallel_do(hp, cs, mf, argp, asz, stream)
                lib.smmo_parallel_do(hp, cn, mn, fz, asz, stream)
            torch.cuda.synchronize()
            ev = events(torch, 2)
            ev[0].record()
            for _ in range(n):
                lib.smmo_parallel_do(hp, cs, mf, argp, asz, stream)
                lib.smmo_parallel_do(hp, cn, mn, fz, asz, stream)
            ev[1].record()
            torch.cuda.synchronize()
            n_frozen[0] += n + warm
            return ev[0].elapsed_time(ev[1]) / n * 1e-3

        t_default = frozen_steps(200) * 1e6
        tf = autotune.tune(heap, "spring.force", "Spring", sim.args, groups=groups, timer=frozen_steps)
        tn = autotune.tune(heap, "spring.node_update", "Node", frozen0, groups=groups, timer=frozen_steps)
        for t in (tf, tn):
            t.pop("tried")
        t_tuned = frozen_steps(200) * 1e6
        keep = t_tuned < t_default
        if not keep:
            smmo.smmo_set_launch(hp, mf, cs, 0, 0, 0)
            smmo.smmo_set_launch(hp, mn, cn, 0, 0, 0)
        count["spring.force"] += n_frozen[0]
        count["spring.node_update"] += n_frozen[0]
        tuned = {"spring.force": tf, "spring.node_update": tn, "step_us_tuned": t_tuned,
                 "step_us_default": t_default, "kept": "tuned" if keep else "default"}
    # eager reference: host-launched steps (reported, not the value)
    eager_n = min(1000, steps)
    torch.cuda.synchronize()
    ee = events(torch, 2)
    t0 = time.perf_counter()
    ee[0].record()
    for _ in range(eager_n):
        step()
    counted(eager_n)
    ee[1].record()
    torch.cuda.synchronize()
    eager_wall = time.perf_counter() - t0
    eager_ms = ee[0].elapsed_time(ee[1]) / max(eager_n, 1)
    done = eager_n                      # real steps taken so far
    # a HIP graph of G steps: the method kernels read the block lists and
    # their lengths on the device, so a captured step is the same work as a
    # launched one, without the host launch cost.  G is at most half the
    # timed steps, so that each timed half is whole replays (a 20-step window
    # replays two graphs of 10 steps).  The timed region uses the graph if it
    # is faster for windows of the timed halves' length: for halves of at
    # least four graphs, four replays against the long launched run above
    # (whose rate is the host's launch rate once the queue is full); for
    # shorter halves, one replay against G steps launched from an idle queue,
    # as a timed half starts (best of four of each).  The probes are counted
    # as warm-up.
    G = min(args.graph_steps, max(1, steps // 2)) if args.graph_steps > 0 else 0
    graph = None
    graph_ms = None
    window_eager_ms = None
    if G > 0:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            cap = torch.cuda.current_stream().cuda_stream
            for _ in range(G):
                step(cap)
        step()          # one launched step: the heap's last stream is ours again
        counted(1)
        done += 1

        def window_ms(run, reps=1):
            torch.cuda.synchronize()
            eg = events(torch, 2)
            eg[0].record()
            for _ in range(reps):
                run()
            eg[1].record()
            torch.cuda.synchronize()
            return eg[0].elapsed_time(eg[1]) / (G * reps)

        def launched():
            for _ in range(G):
                step()

        if steps // 2 >= 4 * G:
            graph_ms = window_ms(graph.replay, 4)
            counted(4 * G)
            done += 4 * G
            rival = eager_ms
        else:
            graph_ms = min(window_ms(graph.replay) for _ in range(4))
            window_eager_ms = min(window_ms(launched) for _ in range(4))
            counted(8 * G)
            done += 8 * G
            rival = window_eager_ms
        if graph_ms >= rival:
            graph = None

    def advance(n):
        """n real steps, as graph replays where whole graphs fit."""
        if graph is not None:
            for _ in range(n // G):
                graph.replay()
            for _ in range(n % G):
                step()
        else:
            for _ in range(n):
                step()
        counted(n)

    # The timed steps are the last `steps` of the workload's 10,000 (or, for
    # a longer request, start right after the probes and the warm-up), so a
    # short timed window sees the mesh as late in the run, springs breaking.
    # Untimed before them: the probes above, the steps that bring the mesh to
    # that point, and the requested warm-up steps right before the window.
    probes = done
    first_timed = max(warmup + probes, total - steps)
    advance(first_timed - warmup - probes)
    advance(warmup)
    done = first_timed
    heap.sync()
    st0 = heap.stats()
    live0 = (st0.live_objects[cs], st0.live_objects[cn])

    # kernel timing: `ks` back-to-back launches of each kernel between two HIP
    # events on the launch stream, at mid-run (between the two timed halves).
    # Repeated force passes are idempotent and the node passes run with dt = 0,
    # so the simulation state is unchanged.
    ks = args.kernel_steps
    frozen = smmo.smmo_spring_args(sim.args.node_class, sim.args.spring_class, 0.0, sim.args.strain_limit,
                                    sim.args.flags)
    fp = smmo.C.byref(frozen)

    window = {}

    def kernel_pass():
        ev = events(torch, 3)
        for k in count:
            window[k] = [count[k], count[k] + ks]
            count[k] += ks
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(ks):
            lib.smmo_parallel_do(hp, cs, mf, fp, asz, stream)
        ev[1].record()
        for _ in range(ks):
            lib.smmo_parallel_do(hp, cn, mn, fp, asz, stream)
        ev[2].record()
        torch.cuda.synchronize()
        st = heap.stats()
        return (ev[0].elapsed_time(ev[1]) / ks * 1e-3, ev[1].elapsed_time(ev[2]) / ks * 1e-3,
                st.live_objects[cs])

    half = steps // 2
    ms = 0.0
    wall = 0.0
    # five event-bounded segments per half (whole graph replays), only where
    # a segment spans at least SEG_MIN_STEPS steps: an event recorded between
    # two steps is a packet the queue processes between the kernels, and in
    # a 20-step window ten of them cost 5 percent of the timed time
    seg_ms = []
    seg_steps = []
    for part, n in enumerate((half, steps - half)):
        # the segment events exist before the timed region: creating one
        # inside it would hold back the host's launches
        seg_ev = events(torch, 5)
        torch.cuda.synchronize()
        e0, e1 = events(torch, 2)
        bounds = []
        t0 = time.perf_counter()
        e0.record()
        segmented = n >= 5 * SEG_MIN_STEPS
        if graph is not None:
            reps = n // G
            cut = {max(1, round(reps * (j + 1) / 5)) for j in range(5)} if reps and segmented else set()
            for r in range(reps):
                graph.replay()
                if r + 1 in cut:
                    ev = seg_ev[len(bounds)]
                    ev.record()
                    bounds.append((ev, (r + 1) * G))
            for _ in range(n % G):
                step()
        else:
            cut = {max(1, round(n * (j + 1) / 5)) for j in range(5)} if n and segmented else set()
            for i in range(n):
                step()
                if i + 1 in cut:
                    ev = seg_ev[len(bounds)]
                    ev.record()
                    bounds.append((ev, i + 1))
        e1.record()
        counted(n)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        ms += e0.elapsed_time(e1)
        prev_ev, prev_n = e0, 0
        for ev, k in bounds:
            if k > prev_n:
                seg_ms.append(prev_ev.elapsed_time(ev))
                seg_steps.append(k - prev_n)
            prev_ev, prev_n = ev, k
        if part == 0:
            t_force, t_node, s_mid = kernel_pass()
    heap.sync()
    st1 = heap.stats()
    live1 = (st1.live_objects[cs], st1.live_objects[cn])
    defrag = None if args.no_extras else measure_spring_defrag(torch, smmo, heap, lib, sim, stream, frozen)
    # live objects processed per step: springs alive at the start of each
    # force pass (breaks during the run counted at the mean) plus all nodes
    springs_mean = 0.5 * (live0[0] + live1[0])
    updates = steps * (springs_mean + live0[1])
    st2 = st1
    S = float(s_mid)
    N = live0[1]
    # algorithmic bytes per launch (each byte once, at the live degree):
    #   spring.force per live spring: a, b, k, L0 (16) + x, y of both nodes
    #     (16) + fx, fy written (8) = 40 B
    #   spring.node_update per node: a slot count (4) + one adjacency entry (4)
    #     and one gathered force (8) per live spring end + x, y, vx, vy, m read
    #     (20) + x, y, vx, vy written (16) = 40 + 12 deg B, deg = 2 S / N
    bytes_force = 40.0 * S
    bytes_node = 40.0 * N + 24.0 * S
    kernels = {
        "spring.force": {"avg_us": t_force * 1e6, "bytes": bytes_force,
                         "gbs": bytes_force / t_force / 1e9},
        "spring.node_update": {"avg_us": t_node * 1e6, "bytes": bytes_node,
                               "gbs": bytes_node / t_node / 1e9},
    }
    dom = "spring.force" if t_force >= t_node else "spring.node_update"
    kd = kernels[dom]
    kernel_state = {"after_steps": done + half, "live_springs": int(s_mid)}
    traffic = traffic_for(dom, kernel_state)
    step_bytes = bytes_force + bytes_node
    res = {
        "value": updates / (ms * 1e-3),
        "unit": "updates/s",
        "ms_per_step": ms / steps,
        "dtype": "f32",
        "config": {"workload": "spring-mass structure, 1000x1000 jittered grid: 1,000,000 Node and "
                               "2,996,001 Spring objects, dt 1e-5, strain limit 0.3",
                   "nodes": int(N), "first_timed_step": first_timed,
                   "untimed_before_warmup": {"probe_steps": probes,
                                             "state_steps": first_timed - warmup - probes},
                   "springs_at_start": int(live0[0]), "springs_at_end": int(live1[0]),
                   "springs_deleted_in_timed_steps": int(live0[0] - live1[0]),
                   "heap_blocks": heap.blocks, "block_bytes": heap.block_bytes},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kd["gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": kd["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": kd["bytes"], "avg_launch_us": kd["avg_us"],
                     "state": kernel_state},
        "step_hbm": {"algorithmic_bytes": step_bytes, "gbs": step_bytes / (ms * 1e-3 / steps) / 1e9,
                     "frac": step_bytes / (ms * 1e-3 / steps) / 1e9 / HBM_PEAK_GBS},
        "kernels": kernels,
        "autotune": tuned,
        "trace_window": {"note": "per-kernel dispatch index range of the timing pass (0-based, "
                                 "graph replays included); after_steps = real steps before it",
                         "after_steps": done + half, **window},
        "launch": {"mode": "hip graph of %d steps" % G if graph is not None else "launched steps",
                   "timed_host_wall_s": wall, "eager_ms_per_step": eager_ms,
                   "graph_ms_per_step": graph_ms, "window_eager_ms_per_step": window_eager_ms,
                   "eager_host_ms_per_step": eager_wall / max(eager_n, 1) * 1e3},
        "device_error": st2.device_error,
    }
    if defrag is not None:
        res["defrag"] = defrag
    if seg_ms:
        rates = sorted(k * (springs_mean + live0[1]) / (t * 1e-3) for k, t in zip(seg_steps, seg_ms) if t > 0)
        res["segments"] = {"note": "the timed steps in event-bounded segments (five per half); rates at the "
                                   "run's mean live springs", "count": len(rates),
                           "median_updates_per_s": float(np.median(rates)), "min_updates_per_s": rates[0],
                           "max_updates_per_s": rates[-1]}

    def cpu_leg():
        from oracle import spring_steps, threads

        k = args.cpu_steps or 1000     # about 10-20 s of float64 oracle work on 16 host threads
        t = time.perf_counter()
        r = spring_steps(mesh, dt, limit, k)
        el = time.perf_counter() - t
        objs = k * (mesh["N"] + 0.5 * (mesh["S"] + int(r["alive"].sum())))
        return {"value": objs / el, "unit": "updates/s", "cores": threads(), "kind": "oracle",
                "sample": "first %d steps of the same 1000x1000 mesh from its initial state, one "
                          "call of the float64 oracle (load, steps, unload), %.1f s" % (k, el)}

    return res, cpu_leg, steps, warmup


def tune_spring_step(torch, sim):
    """Autotunes the launch shapes of spring.force and spring.node_update on
    whole frozen steps of `sim` (force with the run's arguments, node update
    with dt = 0), as the plain run does; keeps the library's defaults unless
    the tuned shapes make the step faster.  Returns the record."""
    from paper_1908_05845_amd import autotune, smmo

    lib = smmo.load_library()
    heap = sim.heap
    hp, cs, cn = heap.h, heap.cls["Spring"], heap.cls["Node"]
    mf, mn = sim.m_force, sim.m_node
    if GIVEN_SHAPES:
        rec = {"kept": "given"}
        for name, m, c in (("spring.force", mf, cs), ("spring.node_update", mn, cn)):
            wg, waves, group = GIVEN_SHAPES[name]
            smmo.smmo_set_launch(hp, m, c, wg, waves, group)
            rec[name] = {"wg": wg, "waves": waves, "group": group}
        return rec
    stream = torch.cuda.current_stream().cuda_stream
    frozen = smmo.smmo_spring_args(sim.args.node_class, sim.args.spring_class, 0.0, sim.args.strain_limit,
                                   sim.args.flags)
    argp, fz, asz = smmo.C.byref(sim.args), smmo.C.byref(frozen), smmo.C.sizeof(sim.args)

    def frozen_steps(n=20, warm=3):
        for _ in range(warm):
            lib.smmo_parallel_do(hp, cs, mf, argp, asz, stream)
            lib.smmo_parallel_do(hp, cn, mn, fz, asz, stream)
        torch.cuda.synchronize()
        ev = events(torch, 2)
        ev[0].record()
        for _ in range(n):
            lib.smmo_parallel_do(hp, cs, mf, argp, asz, stream)
            lib.smmo_parallel_do(hp, cn, mn, fz, asz, stream)
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / n * 1e-3

    t_default = frozen_steps(60) * 1e6
    tf = autotune.tune(heap, "spring.force", "Spring", sim.args, groups=(1, 2, 4), timer=frozen_steps)
    tn = autotune.tune(heap, "spring.node_update", "Node", frozen, groups=(1, 2, 4), timer=frozen_steps)
    for t in (tf, tn):
        t.pop("tried")
    t_tuned = frozen_steps(60) * 1e6
    keep = t_tuned < t_default
    if not keep:
        smmo.smmo_set_launch(hp, mf, cs, 0, 0, 0)
        smmo.smmo_set_launch(hp, mn, cn, 0, 0, 0)
    return {"spring.force": tf, "spring.node_update": tn, "step_us_tuned": t_tuned, "step_us_default": t_default,
            "kept": "tuned" if keep else "default"}


def warm_replay(torch, graph, heap):
    """Replays `graph` once untimed and then puts the heap back as it was, so
    that the timed replay that follows runs the same work with the graph
    already on the device.  Every state the captured do-alls touch lives in
    the heap's buffer (objects, bitmaps, block lists, counters)."""
    snap = heap.buf.clone()
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    heap.buf.copy_(snap)
    torch.cuda.synchronize()
    del snap


def measure_batched(torch, plain_updates_per_s):
    """256 independent meshes (node counts log-uniform in [1e3, 6.4e4]) in one
    heap; launch shapes autotuned on frozen steps of this heap; the 1,000-step
    loop captured in one HIP graph, replayed once untimed, and timed on a
    second replay from the same state."""
    from inputs import batched_meshes, concat_meshes
    from paper_1908_05845_amd.sims import SpringSim

    mesh = concat_meshes(batched_meshes(256))
    dt, limit, T = 1e-5, 0.3, 1000
    sim = SpringSim(mesh, dt, limit)
    heap = sim.heap
    sim.step(5)
    heap.sync()
    tuned = tune_spring_step(torch, sim)
    heap.sync()
    st0 = heap.stats()
    s0 = st0.live_objects[heap.cls["Spring"]]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap = torch.cuda.current_stream()
        for _ in range(T):
            sim.step(1, stream=cap)
    sim.step(1)
    torch.cuda.synchronize()
    warm_replay(torch, g, heap)
    s0 = heap.stats().live_objects[heap.cls["Spring"]]
    e0, e1 = events(torch, 2)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    heap.sync()
    st1 = heap.stats()
    s1 = st1.live_objects[heap.cls["Spring"]]
    n = st1.live_objects[heap.cls["Node"]]
    ups = T * (n + 0.5 * (s0 + s1)) / (ms * 1e-3)
    # algorithmic bytes of a step as for the single mesh: 40 B per live
    # spring (force) and 40 + 12 deg B per node (update), deg = 2 S / N
    step_bytes = 40.0 * n + 64.0 * 0.5 * (s0 + s1)
    res = {"workload": "256 spring meshes in one heap, node counts log-uniform in [1e3, 6.4e4]",
           "nodes": int(n), "springs_at_start": int(s0), "springs_at_end": int(s1), "steps": T,
           "launch": "one HIP graph of %d steps (%d kernel launches)" % (T, 2 * T),
           "ms_per_step": ms / T, "updates_per_s": ups,
           "vs_plain": ups / plain_updates_per_s if plain_updates_per_s else None,
           "step_hbm_gbs": step_bytes / (ms * 1e-3 / T) / 1e9, "autotune": tuned,
           "device_error": st1.device_error}
    heap.close()
    return res


def measure_adjoint(torch, plain_updates_per_s):
    """The adjoint measurement on a created stream, on which the reverse sweep
    recomputes each segment beside the reverse steps of the one after it."""
    with torch.cuda.stream(torch.cuda.Stream()):
        return _measure_adjoint(torch, plain_updates_per_s)


def _measure_adjoint(torch, plain_updates_per_s):
    """316 x 317 mesh (100,172 nodes), breaking off, 200 steps forward with a
    checkpoint every 20 steps, then the reverse sweep (segment recompute
    included) for L = 1/2 |x_T - x_0|^2.  Timed twice: launched from the host
    (every do-all one library call; the reverse sweep also on one stream,
    without the recompute of the next segment beside it) and replayed from
    two captured HIP graphs (forward from the step-0 checkpoint; reverse
    sweep), whose gradients must equal the launched run's bit for bit."""
    import numpy as np

    from inputs import config_seed, spring_mesh
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.adjoint import DiffSpringSim

    mesh = spring_mesh(316, 317, seed=config_seed(5))
    dt, T, every = 1e-5, 200, 20
    sim = DiffSpringSim(mesh, dt, T, every)
    x0 = torch.from_numpy(np.stack([mesh["x"], mesh["y"]], 1)).to(sim.dev)
    # one untimed pass first (module loads, block lists)
    sim.forward()
    sim.backward(torch.zeros(sim.N, device=sim.dev), torch.zeros(sim.N, device=sim.dev))

    def timed(fn):
        torch.cuda.synchronize()
        ev = events(torch, 2)
        ev[0].record()
        fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1])

    # launch shapes of the forward and adjoint kernels, tuned on whole
    # forward + reverse sweeps (the reverse sweep re-seeds its state, so
    # repeated sweeps are the same work)
    from paper_1908_05845_amd import autotune

    sim.restart()
    sim.run_forward()
    g0 = (sim.positions() - x0).contiguous()
    tx, ty = g0[:, 0].contiguous(), g0[:, 1].contiguous()

    def sweep():
        def both():
            sim.restart()
            sim.run_forward()
            sim.run_backward(tx, ty)
        return timed(both) * 1e-3

    t_default = min(sweep() for _ in range(3)) * 1e6
    tuned = {}
    for method, cname, groups in (("spring.force", "Spring", (1, 2, 4)), ("adjoint.step_node", "Node", (1, 2, 4)),
                                  ("adjoint.spring", "Spring", (0,)), ("adjoint.node", "Node", (0,))):
        r = autotune.tune(sim.heap, method, cname, None, groups=groups, timer=sweep,
                          waves_per_cu=(4, 8, 16, 64))
        r.pop("tried")
        tuned[method] = r
    t_tuned = min(sweep() for _ in range(3)) * 1e6
    keep = t_tuned < t_default
    if not keep:
        for method, cname in (("spring.force", "Spring"), ("adjoint.step_node", "Node"),
                              ("adjoint.spring", "Spring"), ("adjoint.node", "Node")):
            smmo.smmo_set_launch(sim.heap.h, smmo.smmo_method_id(method), sim.heap.cls[cname], 0, 0, 0)
    tuned.update(sweep_us_tuned=t_tuned, sweep_us_default=t_default, kept="tuned" if keep else "default")

    # launched from the host
    sim.restart()
    fwd = timed(sim.run_forward)
    xT = sim.positions()
    g = (xT - x0).contiguous()
    sx, sy = g[:, 0].contiguous(), g[:, 1].contiguous()
    bwd1 = timed(lambda: sim.run_backward(sx, sy, overlap=False))
    bwd = timed(lambda: sim.run_backward(sx, sy))
    want = [t.cpu().numpy() for t in sim.gradients()]
    # captured once, replayed
    gf, gb = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(gf):
        st = torch.cuda.current_stream().cuda_stream
        sim.restart(st)
        sim.run_forward(st)
    with torch.cuda.graph(gb):
        sim.run_backward(sx, sy, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    gfw, gbw = [], []
    same = True
    for _ in range(3):
        gfw.append(timed(gf.replay))
        gbw.append(timed(gb.replay))
        got = [t.cpu().numpy() for t in sim.gradients()]
        same = same and all(np.array_equal(a, b) for a, b in zip(got, want))
    gfm, gbm = sorted(gfw)[1], sorted(gbw)[1]
    per_step = sim.N + sim.S
    gk, gv = want[0], want[1]
    res = {"workload": "316x317 spring mesh, 100,172 nodes, %d springs, breaking off, dt 1e-5" % sim.S,
           "steps": T, "checkpoint_every": every,
           "launched": {"forward_ms": fwd, "backward_ms": bwd, "backward_over_forward": bwd / fwd,
                        "backward_one_stream_ms": bwd1},
           "graph": {"forward_ms": gfm, "backward_ms": gbm, "backward_over_forward": gbm / gfm,
                     "replays": 3, "gradients_equal_launched": bool(same)},
           "forward_updates_per_s": T * per_step / (gfm * 1e-3),
           "backward_updates_per_s": T * per_step / (gbm * 1e-3),
           "backward_vs_plain_updates_per_s": (T * per_step / (gbm * 1e-3) / plain_updates_per_s
                                               if plain_updates_per_s else None),
           "loss": float(0.5 * (g.double() ** 2).sum().item()), "grad_k_norm": float(np.linalg.norm(gk)),
           "grad_v0_norm": float(np.linalg.norm(gv)), "autotune": tuned}
    sim.heap.close()
    return res


def measure_gol_extra(torch):
    """Game of Life, 256 x 256 torus, 25 % start: 100 generations captured in
    one HIP graph, replayed once untimed and timed on a second replay from the
    same state.  Births are device allocations, deaths device deletions.  Two
    forms of the same generation: the three do-alls (count, death, birth),
    and gol.generation (the count with the Alive snapshot, then death and
    birth in one launch), each on a heap of its own from the same start."""
    from inputs import gol_init
    from paper_1908_05845_amd.sims import GolSim

    W = H = 256

    def run(fused):
        sim = GolSim(W, H, gol_init(W, H), fused=fused)
        heap = sim.heap
        sim.step(2)
        heap.sync()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            cap = torch.cuda.current_stream()
            sim.step(100, stream=cap)
        sim.step(1)
        heap.sync()
        warm_replay(torch, g, heap)
        st0 = heap.stats()
        e0, e1 = events(torch, 2)
        torch.cuda.synchronize()
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st1 = heap.stats()
        ca = heap.cls["Alive"]
        heap.close()
        return ms, st0, st1, ca

    ms, st0, st1, ca = run(False)
    news = st1.device_news - st0.device_news
    dels = st1.device_deletes - st0.device_deletes
    alive = 0.5 * (st0.live_objects[ca] + st1.live_objects[ca])
    fms, f0, f1, _ = run(True)
    falive = 0.5 * (f0.live_objects[ca] + f1.live_objects[ca])
    res = {"workload": "Game of Life in SMMO form, 256x256 torus, 25% start, 100 generations",
           "launch": "one HIP graph of 100 generations", "us_per_generation": ms * 1e3 / 100,
           "updates_per_s": 100 * (2 * W * H + alive) / (ms * 1e-3),
           "births_per_s": news / (ms * 1e-3), "deaths_per_s": dels / (ms * 1e-3),
           "births": int(news), "deaths": int(dels), "alive_mean": alive,
           "fragmentation_end": st1.fragmentation, "device_error": st1.device_error,
           "fused": {"method": "gol.generation: the count with the Alive snapshot, then death and birth in "
                               "one launch", "us_per_generation": fms * 1e3 / 100,
                     "updates_per_s": 100 * (2 * W * H + falive) / (fms * 1e-3),
                     "births": int(f1.device_news - f0.device_news),
                     "deaths": int(f1.device_deletes - f0.device_deletes), "device_error": f1.device_error}}
    return res


def measure_gol_large(torch):
    """Game of Life, 16384 x 16384 torus (268M Cell objects), 25 % start:
    the supplemental size whose state (about 10 GB of blocks) is far beyond
    the 256 MB MALL, for an HBM figure.  Two generations to settle, then
    five timed with events around each of the three do-alls.

    Algorithmic bytes: Cell::count reads cell_id (4 B), the neighbour handle
    row (4 B, each handle reused by eight neighbours) and the state byte of
    each cell once, and writes count (4 B): 13 B per cell.  Cell::birth reads
    state and count (5 B per cell) and writes the state of a newborn.
    Alive::death reads cell_id, the cell handle and the cell's count (12 B per
    live Alive)."""
    from inputs import gol_init
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.sims import GolSim

    W = H = 16384
    print("extras: gol 16384^2 setup", file=sys.stderr, flush=True)
    sim = GolSim(W, H, gol_init(W, H))
    heap = sim.heap
    h, c, a = heap.h, heap.cls["Cell"], heap.cls["Alive"]
    sim.step(2)
    heap.sync()
    n = 5
    tot = [0.0, 0.0, 0.0]
    alive_sum = 0.0
    news = dels = 0
    fused = []
    # the two forms take turns, one generation each (the population changes
    # from generation to generation): three do-alls with events around
    # each, then gol.generation (an enumeration of Alive with its snapshot,
    # the count, death and birth in one launch) with one pair of events
    for _ in range(n):
        sb = heap.stats()
        alive_sum += sb.live_objects[a]
        ev = events(torch, 4)
        ev[0].record()
        smmo.smmo_parallel_do(h, c, sim.m_count, sim.args)
        ev[1].record()
        smmo.smmo_parallel_do(h, a, sim.m_death, sim.args)
        ev[2].record()
        smmo.smmo_parallel_do(h, c, sim.m_birth, sim.args)
        ev[3].record()
        torch.cuda.synchronize()
        for i in range(3):
            tot[i] += ev[i].elapsed_time(ev[i + 1]) * 1e3
        sm = heap.stats()
        news += sm.device_news - sb.device_news
        dels += sm.device_deletes - sb.device_deletes
        ev = events(torch, 2)
        ev[0].record()
        smmo.smmo_parallel_do(h, c, sim.m_gen, sim.args)
        ev[1].record()
        torch.cuda.synchronize()
        fused.append(ev[0].elapsed_time(ev[1]) * 1e3)
    st1 = heap.stats()
    cells = W * H
    alive = alive_sum / n
    us = [t / n for t in tot]
    gen_us = sum(us)
    res = {"workload": "Game of Life in SMMO form, 16384x16384 torus (268M cells), 25% start",
           "generations_timed": n, "us_per_generation": gen_us,
           "cell_updates_per_s": cells / (gen_us * 1e-6),
           "updates_per_s": (2 * cells + alive) / (gen_us * 1e-6),
           "alive_mean": alive,
           "count_us": us[0], "death_us": us[1], "birth_us": us[2],
           "count_gbs": 13.0 * cells / (us[0] * 1e-6) / 1e9,
           "birth_gbs": 5.0 * cells / (us[2] * 1e-6) / 1e9,
           "death_gbs": 12.0 * alive / (us[1] * 1e-6) / 1e9,
           "births_per_s": news / (gen_us * n * 1e-6),
           "deaths_per_s": dels / (gen_us * n * 1e-6),
           "device_error": st1.device_error,
           "fused": {"method": "gol.generation, on the generations between the timed three-do-all ones",
                     "us_per_generation": sum(fused) / n}}
    heap.close()
    return res


def measure_spring_large(torch):
    """Spring mesh 2000 x 2000 (4M nodes, 12.0M springs; about 900 MB of
    blocks, beyond the 256 MB MALL): the plain step's supplemental size.  The
    launch shapes are tuned for this heap (its own size bucket) on whole
    frozen steps, as for the 1000 x 1000 mesh.  20 steps to settle, then 50
    timed with events around each do-all; bytes per object as for the 1000 x
    1000 mesh (40 B per live spring; 40 + 12 deg B per node)."""
    from inputs import spring_mesh
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.sims import SpringSim

    print("extras: spring 2000^2 setup", file=sys.stderr, flush=True)
    mesh = spring_mesh(2000, 2000)
    sim = SpringSim(mesh, 1e-5, 0.3)
    heap = sim.heap
    cs, cn = heap.cls["Spring"], heap.cls["Node"]
    sim.step(20)
    heap.sync()
    tuned = tune_spring_step(torch, sim)
    heap.sync()
    n = 50
    ev = events(torch, 2 * n + 1)
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(n):
        sim.spring_force()
        ev[2 * i + 1].record()
        sim.node_update()
        ev[2 * i + 2].record()
    torch.cuda.synchronize()
    tf = sum(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(n)) * 1e3 / n
    tn = sum(ev[2 * i + 1].elapsed_time(ev[2 * i + 2]) for i in range(n)) * 1e3 / n
    st = heap.stats()
    live = st.live_objects[cs]
    N = st.live_objects[cn]
    step_us = ev[0].elapsed_time(ev[2 * n]) * 1e3 / n
    fb, nb = 40.0 * live, 40.0 * N + 24.0 * live
    res = {"workload": "spring-mass structure, 2000x2000 jittered grid: 4,000,000 Node and %d Spring objects"
                       % len(mesh["a"]),
           "steps_timed": n, "us_per_step": step_us, "updates_per_s": (N + live) / (step_us * 1e-6),
           "springs_live": int(live),
           "force_us": tf, "force_gbs": fb / (tf * 1e-6) / 1e9,
           "node_us": tn, "node_gbs": nb / (tn * 1e-6) / 1e9,
           "step_gbs": (fb + nb) / (step_us * 1e-6) / 1e9,
           "force_frac": fb / (tf * 1e-6) / 1e9 / HBM_PEAK_GBS, "node_frac": nb / (tn * 1e-6) / 1e9 / HBM_PEAK_GBS,
           "autotune": tuned, "device_error": st.device_error}
    heap.close()
    return res


def measure_structure(torch):
    """The fracture simulation ("structure"), 1000 x 1000 brick-wall mesh
    (1M nodes in three node classes, 1.5M springs), stretched uniformly
    (strain rate 0.5, pull nodes at the same speed) until its springs break
    (limits at 0.5-1.5 % strain): per iteration one pull, 40 compute steps
    (Spring::force, Node::update) and the BFS removal of disconnected nodes.
    One iteration to settle, then six timed (the mesh cracks and falls apart
    within them) with events around each phase.  The BFS runs as one call
    with its frontier in a queue (timed with events around its launches);
    the thesis's form, level passes launched 32 at a time between reads of
    their frontier flags, is timed on a second run of the same iterations."""
    from inputs import structure_mesh
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.sims import StructureSim

    print("extras: structure 1000^2 setup", file=sys.stderr, flush=True)
    W = H = 1000
    sub = 40
    mesh = structure_mesh(W, H, pull_speed=0.5, stretch_rate=0.5, break_strain=0.01)

    def run(bfs):
        sim = StructureSim(mesh, 1e-4, bfs_batch=32, bfs=bfs)
        heap = sim.heap
        c = heap.cls
        nodes = lambda st: sum(st.live_objects[c[n]] for n in ("AnchorNode", "AnchorPullNode", "Node"))
        sim.iterate(sub)
        heap.sync()
        st0 = heap.stats()
        n_it = 6
        t_pull = t_comp = t_bfs = 0.0
        levels = 0
        upd = 0.0
        for _ in range(n_it):
            st = heap.stats()
            upd += sub * (st.live_objects[c["Spring"]] + st.live_objects[c["Node"]])
            e = events(torch, 3)
            e[0].record()
            sim.pull(sim.dt * sub)
            e[1].record()
            for _ in range(sub):
                sim.compute_step()
            e[2].record()
            torch.cuda.synchronize()
            if bfs == "queue":
                eb = events(torch, 2)
                eb[0].record()
                smmo.smmo_structure_remove_disconnected(heap.h, sim.args, sim.bfs_work, sim.bfs_levels)
                eb[1].record()
                torch.cuda.synchronize()
                levels += int(sim.bfs_levels.cpu().item())
                t_bfs += eb[0].elapsed_time(eb[1]) * 1e3
            else:
                t0 = time.perf_counter()
                levels += sim.remove_disconnected()
                torch.cuda.synchronize()
                t_bfs += (time.perf_counter() - t0) * 1e6
            t_pull += e[0].elapsed_time(e[1]) * 1e3
            t_comp += e[1].elapsed_time(e[2]) * 1e3
        st1 = heap.stats()
        out = {"us_per_iteration": (t_pull + t_comp + t_bfs) / n_it,
               "compute_us_per_substep": t_comp / (n_it * sub), "compute_updates_per_s": upd / (t_comp * 1e-6),
               "bfs_us_per_iteration": t_bfs / n_it, "bfs_levels_per_iteration": levels / n_it,
               "bfs_us_per_level": t_bfs / max(levels, 1),
               "springs_start": int(st0.live_objects[c["Spring"]]),
               "springs_end": int(st1.live_objects[c["Spring"]]),
               "nodes_start": int(nodes(st0)), "nodes_end": int(nodes(st1)),
               "device_deletions": int(st1.device_deletes - st0.device_deletes),
               "device_error": st1.device_error}
        heap.close()
        return out, n_it

    res, n_it = run("queue")
    levels_form, _ = run("levels")
    res = {"workload": "structure (fracture), 1000x1000 brick-wall mesh: %d nodes (anchor, pull and free node "
                       "classes under an abstract NodeBase), %d springs" % (W * H, len(mesh["p1"])),
           "iterations_timed": n_it, "substeps_per_iteration": sub, "bfs": "frontier queue, one call", **res,
           "bfs_level_passes": {k: levels_form[k] for k in ("us_per_iteration", "bfs_us_per_iteration",
                                                            "bfs_levels_per_iteration", "bfs_us_per_level",
                                                            "nodes_end", "springs_end")}}
    return res


def measure_generation(torch):
    """generation (Game of Life with dying cells, rule Burst: survive
    0235678, birth 3468, dying 255), 256 x 256 torus, 25 % start: 300
    generations (past the dying period) captured in one HIP graph (replayed
    once untimed, timed on a second replay from the same state), three
    do-alls per generation; births are device allocations, expiries device
    deletions."""
    from inputs import gol_init
    from paper_1908_05845_amd.sims import GenerationSim

    W = H = 256
    sim = GenerationSim(W, H, gol_init(W, H))
    heap = sim.heap
    sim.step(2)
    heap.sync()
    n = 300
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sim.step(n, stream=torch.cuda.current_stream())
    warm_replay(torch, g, heap)
    st0 = heap.stats()
    e0, e1 = events(torch, 2)
    torch.cuda.synchronize()
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st1 = heap.stats()
    ca = heap.cls["Alive"]
    res = {"workload": "generation (rule Burst 0235678/3468/255), 256x256 torus, 25%% start, %d generations" % n,
           "launch": "one HIP graph", "us_per_generation": ms * 1e3 / n,
           "births_per_s": (st1.device_news - st0.device_news) / (ms * 1e-3),
           "expiries_per_s": (st1.device_deletes - st0.device_deletes) / (ms * 1e-3),
           "alive_objects_end": int(st1.live_objects[ca]), "fragmentation_end": st1.fragmentation,
           "device_error": st1.device_error}
    heap.close()
    return res


def measure_spring_pi(torch):
    """Partially inlined adjacency (Ch.4 "SOA with Partial Inlining") on a
    500 x 500 mesh with 250 hub nodes of about 64 extra springs each: for K
    inline slots in {2, 4, 6, 8}, the block size and the step's kernel times
    (spring_pi.force, spring_pi.node_update) over 50 frozen steps.  Slots
    past K are read from the array outside the heap."""
    import numpy as np

    from inputs import hub_mesh
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.sims import SpringPiSim

    print("extras: partial inlining setup", file=sys.stderr, flush=True)
    mesh = hub_mesh(500, 500, hubs=250, hub_springs=64)
    deg = (np.asarray(mesh["adj"]) >= 0).sum(axis=1)
    res = {"workload": "spring mesh 500x500 with 250 hubs: %d nodes, %d springs, degree up to %d (mean %.2f)"
                       % (deg.size, len(mesh["a"]), int(deg.max()), float(deg.mean())), "by_K": {}}
    for K in (2, 4, 6, 8):
        sim = SpringPiSim(mesh, 0.0, K, strain_limit=1e9)
        heap = sim.heap
        h, cs, cn = heap.h, heap.cls["Spring"], heap.cls["Node"]
        sim.step(5)
        n = 50
        ev = events(torch, 2 * n + 1)
        torch.cuda.synchronize()
        ev[0].record()
        for i in range(n):
            smmo.smmo_parallel_do(h, cs, sim.m_force, sim.args)
            ev[2 * i + 1].record()
            smmo.smmo_parallel_do(h, cn, sim.m_node, sim.args)
            ev[2 * i + 2].record()
        torch.cuda.synchronize()
        tf = sum(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(n)) * 1e3 / n
        tn = sum(ev[2 * i + 1].elapsed_time(ev[2 * i + 2]) for i in range(n)) * 1e3 / n
        res["by_K"][str(K)] = {"block_bytes": heap.block_bytes, "heap_mb": heap.nbytes / 1e6,
                               "out_of_line_slots": int(sim.args.overflow_len),
                               "force_us": tf, "node_update_us": tn, "step_us": tf + tn,
                               "device_error": heap.stats().device_error}
        heap.close()
        del sim
    return res


def measure_linux_scalability(torch):
    """Linux Scalability pattern (Ch.8 "Raw Allocation Performance") in SMMO
    form: a 1 GiB heap, 16,384 Worker objects each allocate n 64-byte Obj
    objects through the device allocator (one do-all), a second do-all frees
    them; time per n = (allocation + free time) / n.  Also: the largest n the
    heap holds (utilization = objects x 64 B / 1 GiB), and the allocator
    ablations of the thesis at n = 64."""
    from paper_1908_05845_amd import smmo

    classes = {"Worker": [("id", "i32", 1)], "Obj": [("payload", "u32", 16)]}
    workers = 16384

    def run(n, **kw):
        cfg = smmo.smmo_config_default()
        for k, v in kw.items():
            setattr(cfg, k, v)
        heap = smmo.Heap(classes, nbytes=1 << 30, cfg=cfg)
        heap.new("Worker", workers, id=torch.arange(workers, dtype=torch.int32, device="cuda"))
        handles = torch.full((n * workers,), -1, dtype=torch.int32, device="cuda")
        args = smmo.smmo_ls_args(heap.cls["Obj"], n, workers, 0, handles.data_ptr())
        heap.sync()
        ev = events(torch, 3)
        ev[0].record()
        heap.do("Worker", "alloc.ls_alloc", args)
        ev[1].record()
        heap.do("Worker", "alloc.ls_free", args)
        ev[2].record()
        torch.cuda.synchronize()
        st = heap.stats()
        out = {"n": n, "alloc_ms": ev[0].elapsed_time(ev[1]), "free_ms": ev[1].elapsed_time(ev[2]),
               "device_error": st.device_error, "allocated": int(st.device_news),
               "live_after_free": int(st.live_objects[heap.cls["Obj"]]), "retries": int(st.alloc_retries),
               "heap_blocks": heap.blocks}
        out["us_per_n"] = (out["alloc_ms"] + out["free_ms"]) * 1e3 / n
        heap.close()
        del handles
        return out

    res = {"workload": "1 GiB heap, 16,384 Worker objects, 64-byte Obj objects", "runs": []}
    for n in (1, 4, 16, 64, 256, 1000):
        res["runs"].append(run(n))
    # largest n that fits: the heap's blocks minus the Worker blocks, 64 objects each
    nblk = res["runs"][0]["heap_blocks"] - (workers + 63) // 64
    n_max = nblk * 64 // workers
    top = run(n_max)
    top["utilization"] = workers * n_max * 64 / float(1 << 30)
    res["max_n"] = top
    res["ablations_n64"] = {k: run(64, **kw) for k, kw in (
        ("no_rotation", {"rotation": 0}), ("no_coalescing", {"coalescing": 0}),
        ("retries_1", {"lookup_retries": 1}))}
    return res


def measure_wator(torch):
    """wa-tor (Ch.7 "wa-tor"), 1024 x 1024 torus, 30 % fish and 5 % sharks at
    the start, fish spawn 4, shark spawn 12, energy 8, boost 4: 500 timed
    iterations (eight do-alls each, fish and sharks created and deleted by
    the device allocator), then the fragmentation of the Fish and Shark
    blocks over a second run (sampled every 25 iterations), and the
    allocator ablations on a 512 x 512 torus."""
    from inputs import config_seed, wator_init
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.sims import WatorSim

    prm = (4, 12, 8, 4)
    seed = config_seed(7)

    def agent_frag(sim):
        st = sim.heap.stats()
        c = sim.heap.cls
        blocks = st.blocks[c["Fish"]] + st.blocks[c["Shark"]]
        live = st.live_objects[c["Fish"]] + st.live_objects[c["Shark"]]
        return st, (1.0 - live / (64.0 * blocks)) if blocks else 0.0

    def make(W, cfg=None):
        init = wator_init(W, W, fish_spawn=prm[0], shark_spawn=prm[1], energy0=prm[2])
        return WatorSim(W, W, seed, prm, init, cfg=cfg)

    W, iters = 1024, 500
    sim = make(W)
    sim.step(5)
    st0, _ = agent_frag(sim)
    torch.cuda.synchronize()
    ev = events(torch, 2)
    ev[0].record()
    sim.step(iters)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    st1, frag_end = agent_frag(sim)
    res = {"workload": "wa-tor 1024x1024 torus, fish/shark 0.30/0.05, params (fish_spawn, shark_spawn, "
                       "energy0, boost) = %s" % (prm,),
           "iterations": iters, "ms_per_iteration": ms / iters,
           "device_news_per_s": (st1.device_news - st0.device_news) / (ms * 1e-3),
           "device_deletes_per_s": (st1.device_deletes - st0.device_deletes) / (ms * 1e-3),
           "fish_end": int(st1.live_objects[sim.heap.cls["Fish"]]),
           "sharks_end": int(st1.live_objects[sim.heap.cls["Shark"]]),
           "agent_fragmentation_end": frag_end, "device_error": st1.device_error}
    sim.heap.close()
    sim = make(W)
    curve = []
    for k in range(0, iters + 1, 25):
        if k:
            sim.step(25)
        st, fr = agent_frag(sim)
        curve.append([k, int(st.live_objects[sim.heap.cls["Fish"]]), int(st.live_objects[sim.heap.cls["Shark"]]),
                      round(fr, 4)])
    res["fragmentation_curve"] = {"columns": ["iteration", "fish", "sharks", "agent_fragmentation"],
                                  "rows": curve}
    sim.heap.close()
    abl = {}
    for name, kw in (("default", {}), ("no_rotation", {"rotation": 0}), ("no_coalescing", {"coalescing": 0}),
                     ("retries_1", {"lookup_retries": 1})):
        cfg = smmo.smmo_config_default()
        for k, v in kw.items():
            setattr(cfg, k, v)
        sim = make(512, cfg)
        torch.cuda.synchronize()
        ev = events(torch, 2)
        ev[0].record()
        sim.step(300)
        ev[1].record()
        torch.cuda.synchronize()
        st, fr = agent_frag(sim)
        abl[name] = {"ms_per_iteration": ev[0].elapsed_time(ev[1]) / 300, "agent_fragmentation": fr,
                     "retries": int(st.alloc_retries), "slow_paths": int(st.slow_paths),
                     "device_error": st.device_error}
        sim.heap.close()
    res["ablations_512x512_300it"] = abl
    return res


def measure_spring_defrag(torch, smmo, heap, lib, sim, stream, frozen):
    """After the timed steps (springs broken, blocks part empty): whole-step
    time before and after CompactGpu merges the Spring blocks (n = 1, 2, 3
    in turn), on frozen steps (force pass, then node pass with dt = 0) so
    that the state is the same for every measurement."""
    cs, cn = heap.cls["Spring"], heap.cls["Node"]
    asz = smmo.C.sizeof(sim.args)

    def steps(n=200):
        for _ in range(10):
            lib.smmo_parallel_do(heap.h, cs, sim.m_force, smmo.C.byref(sim.args), asz, stream)
            lib.smmo_parallel_do(heap.h, cn, sim.m_node, smmo.C.byref(frozen), asz, stream)
        torch.cuda.synchronize()
        ev = events(torch, 2)
        ev[0].record()
        for _ in range(n):
            lib.smmo_parallel_do(heap.h, cs, sim.m_force, smmo.C.byref(sim.args), asz, stream)
            lib.smmo_parallel_do(heap.h, cn, sim.m_node, smmo.C.byref(frozen), asz, stream)
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / n * 1e3

    def state():
        st = heap.stats()
        return {"spring_blocks": int(st.blocks[cs]), "live_springs": int(st.live_objects[cs]),
                "spring_fragmentation": 1.0 - st.live_objects[cs] / (64.0 * st.blocks[cs])}

    out = {"before": dict(state(), step_us=steps()), "after": []}
    for n in (1, 2, 3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        passes, moved = heap.defragment("Spring", n=n, k1=0, max_passes=64)
        ms = (time.perf_counter() - t0) * 1e3
        out["after"].append(dict(state(), n=n, passes=passes, moved=moved, defrag_host_ms=ms, step_us=steps()))
    return out


def measure_enumeration(torch):
    """Enumeration cost against heap size (the thesis: the pre-pass that
    lists a class's blocks before a do-all costs about the same whatever the
    heap's size).  65,536 objects of a one-field class (1,024 full blocks) in
    heaps of 2^12 .. 2^24 blocks; a host-side parallel_new of one object
    (destroyed again) makes the class's list stale, so the next do-all
    (test.axpy) first enumerates.  Enumeration = that do-all's time minus the
    time of the same do-all right after it (list valid); medians of 20."""
    import numpy as np

    from paper_1908_05845_amd import smmo

    out = {}
    for lg in (12, 14, 16, 18, 20, 22, 24):
        M = 1 << lg
        heap = smmo.Heap({"Obj": [("x", "f32", 1)]}, blocks=M)
        heap.new("Obj", 65536, x=torch.ones(65536, device="cuda"))
        mid = smmo.smmo_method_id("test.axpy")
        args = smmo.smmo_axpy_args(1.0, 0.0)
        cls = heap.cls["Obj"]
        with_enum, without = [], []
        for _ in range(22):
            one = heap.new("Obj", 1, x=torch.ones(1, device="cuda"))
            smmo.smmo_destroy(heap.h, cls, one, 1)
            torch.cuda.synchronize()
            e = events(torch, 3)
            e[0].record()
            smmo.smmo_parallel_do(heap.h, cls, mid, args)
            e[1].record()
            smmo.smmo_parallel_do(heap.h, cls, mid, args)
            e[2].record()
            torch.cuda.synchronize()
            with_enum.append(e[0].elapsed_time(e[1]) * 1e3)
            without.append(e[1].elapsed_time(e[2]) * 1e3)
        a, b = float(np.median(with_enum[2:])), float(np.median(without[2:]))
        out["2^%d" % lg] = {"blocks": M, "do_all_us_with_enumeration": a, "do_all_us": b,
                            "enumeration_us": a - b}
        heap.close()
        print("extras: enumeration at 2^%d blocks: %.2f us" % (lg, a - b), file=sys.stderr, flush=True)
    return {"workload": "65,536 objects (1,024 full blocks) of a one-field class in heaps of 2^12 .. 2^24 blocks",
            "by_heap_blocks": out}


def measure_coalescing(torch):
    """The thesis's memory coalescing experiment (Ch.2) in wave64 form, on a
    1 GiB float array: read-modify-write of every element with the lanes of
    a wavefront spread over C arrays; median of 3 passes per C.  C = 1 is
    the attainable read-modify-write bandwidth."""
    from paper_1908_05845_amd import smmo

    n = 1 << 28
    data = torch.zeros(n, dtype=torch.float32, device="cuda")
    out = {"bytes_per_pass": 8 * n, "runs": []}
    for C in (1, 2, 4, 8, 16, 32, 64):
        smmo.smmo_coalescing_probe(data, C)
        ts = []
        for _ in range(3):
            ev = events(torch, 2)
            ev[0].record()
            smmo.smmo_coalescing_probe(data, C)
            ev[1].record()
            torch.cuda.synchronize()
            ts.append(ev[0].elapsed_time(ev[1]))
        t = sorted(ts)[1]
        out["runs"].append({"C": C, "ms": t, "gbs": 8 * n / (t * 1e-3) / 1e9})
    out["slowdown_C64_vs_C1"] = out["runs"][-1]["ms"] / out["runs"][0]["ms"]
    del data
    return out


def measure_allocation(torch):
    """Heap initialization and smmo_parallel_new on the spring mesh's classes
    (1,000,000 Node and 2,996,001 Spring objects), as allocations/s: the
    ordered bulk path, and the device allocator path (bulk_ordered = 0) for
    the springs."""
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.sims import SPRING_CLASSES

    N, S = 1_000_000, 2_996_001
    out = {}
    for ordered in (1, 0):
        cfg = smmo.smmo_config_default()
        cfg.bulk_ordered = ordered
        t0 = time.perf_counter()
        heap = smmo.Heap(SPRING_CLASSES, blocks=(N + 63) // 64 + (S + 63) // 64 + 64, cfg=cfg)
        heap.sync()
        init_ms = (time.perf_counter() - t0) * 1e3
        ids_n = torch.arange(N, dtype=torch.int32, device="cuda")
        ids_s = torch.arange(S, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        ev = events(torch, 3)
        ev[0].record()
        heap.new("Node", N, id=ids_n)
        ev[1].record()
        heap.new("Spring", S, id=ids_s)
        ev[2].record()
        torch.cuda.synchronize()
        st = heap.stats()
        key = "ordered_bulk" if ordered else "device_allocator"
        out[key] = {"heap_init_ms_host": init_ms, "node_new_ms": ev[0].elapsed_time(ev[1]),
                    "spring_new_ms": ev[1].elapsed_time(ev[2]),
                    "spring_allocations_per_s": S / (ev[1].elapsed_time(ev[2]) * 1e-3),
                    "live": [int(st.live_objects[heap.cls["Node"]]), int(st.live_objects[heap.cls["Spring"]])],
                    "device_error": st.device_error}
        heap.close()
    return out


def measure_copy_bandwidth(torch):
    """Attainable HBM bandwidth on this GPU: a device-to-device copy of 512
    MiB (read + write = 1 GiB of traffic), median of 5 timed copies."""
    n = (512 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(5):
        ev = events(torch, 2)
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    t = sorted(ts)[2]
    del src, dst
    return {"bytes_moved": 2 * 4 * n, "ms": t, "gbs": 2 * 4 * n / (t * 1e-3) / 1e9,
            "frac_of_peak": 2 * 4 * n / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}


def measure_nbody_extra(torch):
    """n-body, 65,536 bodies, 50 steps: device_do over all pairs (FP32 VALU bound)."""
    from inputs import nbody_init
    from paper_1908_05845_amd.sims import NbodySim

    n = 65536
    sim = NbodySim(nbody_init(n), 1.0 / n, 1e-3, 1e-4)
    sim.step(1)
    torch.cuda.synchronize()
    e = events(torch, 3)
    e[0].record()
    for _ in range(10):
        sim.force()
    e[1].record()
    sim.step(49)
    e[2].record()
    torch.cuda.synchronize()
    tf = e[0].elapsed_time(e[1]) / 10 * 1e-3
    ms = e[1].elapsed_time(e[2]) / 49
    pairs = float(n) * n
    res = {"workload": "n-body, 65,536 bodies, all pairs, softening 1e-3, dt 1e-4",
           "ms_per_step": ms, "force_us": tf * 1e6, "pairs_per_s": pairs / tf,
           "tflops_20_per_pair": 20 * pairs / tf / 1e12,
           "frac_fp32_peak": 20 * pairs / tf / 1e12 / FP32_VALU_PEAK_TFLOPS,
           "frac_fp32_nonpacked_peak": 20 * pairs / tf / 1e12 / (FP32_VALU_PEAK_TFLOPS / 2)}
    sim.heap.close()
    return res


# --------------------------------------------------------------------- gol --
def bench_gol(args, torch):
    from inputs import gol_init
    from paper_1908_05845_amd.sims import GolSim

    W = H = 256
    steps = 100 if args.steps is None else args.steps
    warmup = 5 if args.warmup is None else args.warmup
    init = gol_init(W, H)
    sim = GolSim(W, H, init, fused=args.gol_form == "fused")
    for _ in range(warmup):
        sim.step(1)
    sim.heap.sync()
    cls_a = sim.heap.cls["Alive"]
    alive_before = sim.heap.stats().live_objects[cls_a]
    torch.cuda.synchronize()
    e0, e1 = events(torch, 2)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sim.heap.sync()
    alive_after = sim.heap.stats().live_objects[cls_a]
    updates = steps * (2 * W * H + 0.5 * (alive_before + alive_after))
    res = {"value": updates / (ms * 1e-3), "unit": "updates/s", "ms_per_step": ms / steps, "dtype": "u8/i32",
           "config": {"workload": "Game of Life in SMMO form, 256x256 torus, 25% initial density",
                      "form": "gol.generation" if args.gol_form == "fused" else "three do-alls"},
           "roofline": None}

    def cpu_leg():
        from oracle import GolWorld

        w = GolWorld(W, H, init)
        t = time.perf_counter()
        w.step(steps)
        el = time.perf_counter() - t
        return {"value": updates / el, "unit": "updates/s", "cores": 1, "kind": "oracle",
                "sample": "%d generations from the initial state, %.2f s" % (steps, el)}

    return res, cpu_leg, steps, warmup


# ------------------------------------------------------------------- nbody --
def bench_nbody(args, torch):
    from inputs import nbody_init
    from paper_1908_05845_amd.sims import NbodySim

    n = 65536
    G, eps, dt = 1.0 / n, 1e-3, 1e-4
    steps = 50 if args.steps is None else args.steps
    warmup = 2 if args.warmup is None else args.warmup
    st = nbody_init(n)
    sim = NbodySim(st, G, eps, dt)
    sim.step(warmup)
    torch.cuda.synchronize()
    ev = events(torch, 3 * steps)
    for i in range(steps):
        ev[3 * i].record()
        sim.force()
        ev[3 * i + 1].record()
        sim.update()
        ev[3 * i + 2].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1])
    tf = sum(ev[3 * i].elapsed_time(ev[3 * i + 1]) for i in range(steps)) / steps * 1e-3
    pairs = float(n) * n
    flop = 20.0 * pairs
    res = {"value": steps * 2 * n / (ms * 1e-3), "unit": "updates/s", "ms_per_step": ms / steps, "dtype": "f32",
           "config": {"workload": "n-body, 65,536 bodies, all pairs, softening 1e-3, dt 1e-4"},
           "roofline": {"bound": "alu", "kernel": "nbody.force", "achieved": flop / tf / 1e12,
                        "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": flop / tf / 1e12 / FP32_VALU_PEAK_TFLOPS, "traffic": None,
                        "pairs_per_s": pairs / tf, "avg_launch_us": tf * 1e6}}

    def cpu_leg():
        from oracle import nbody_force_at

        import numpy as np
        k = 2048
        t = time.perf_counter()
        nbody_force_at(st["x"], st["y"], st["m"], G, eps, np.arange(k))
        el = time.perf_counter() - t
        return {"value": k / el * 2, "unit": "updates/s", "cores": 1, "kind": "oracle",
                "sample": "compute_force of %d of the 65,536 bodies (all pairs), %.1f s" % (k, el)}

    return res, cpu_leg, steps, warmup


COPY_BYTES = 512 << 20
KERNEL_KEYS = {"spring.force": "k_spring_force", "spring.node_update": "k_spring_node"}


def calibrate_copy(torch):
    """Three plain device-to-device copies of COPY_BYTES (reads and writes
    COPY_BYTES each): the reference that scales rocprofv3 byte counters."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def _read_counter_csv(d):
    import csv
    import glob

    rows = []
    for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(fn) as f:
            rows.extend(csv.DictReader(f))
    return rows


def summarize_counters(fetch_dir, write_dir, fetch_json=None, write_json=None):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the spring kernels,
    scaled by the ratio of true to counted bytes of the calibration copy.
    With the bench JSON lines of the two profiled runs, only the dispatches
    of each run's per-kernel timing window (its timed launch shapes) are
    averaged."""
    windows = {}
    states = []
    for counter, jf in (("FETCH_SIZE", fetch_json), ("WRITE_SIZE", write_json)):
        if jf:
            with open(jf) as f:
                ln = json.loads([ln for ln in f if ln.startswith("{")][-1])
            windows[counter] = ln["trace_window"]
            states.append({"after_steps": int(ln["steps_before"]), "live_springs": int(ln["live_springs"])})
    if len(states) == 2 and states[0] != states[1]:
        raise SystemExit("the two counter runs saw different mesh states: %s" % states)
    out = {"source_hash": kernel_source_hash(), "copy_bytes": COPY_BYTES, "kernels": {},
           "state": states[0] if states else None}
    lines = []
    factor = {}
    per = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _read_counter_csv(d) if r.get("Counter_Name") == counter]
        if not rows:
            raise SystemExit("no %s rows under %s" % (counter, d))
        # the calibration copies are the last three copy dispatches of the run
        # (earlier copies are host uploads and small staging transfers)
        copies = sorted((r for r in rows if "copy" in r["Kernel_Name"].lower()),
                        key=lambda r: int(r["Dispatch_Id"]))[-3:]
        cal = [float(r["Counter_Value"]) * 1024.0 for r in copies]
        factor[counter] = COPY_BYTES / (sum(cal) / len(cal))
        for name, key in KERNEL_KEYS.items():
            mine = sorted((r for r in rows if key in r["Kernel_Name"]), key=lambda r: int(r["Dispatch_Id"]))
            if counter in windows:
                lo, hi = windows[counter][name]
                mine = mine[lo:hi]
            vals = [float(r["Counter_Value"]) * 1024.0 for r in mine]
            per.setdefault(name, {})[counter] = (sum(vals) / len(vals), len(vals))
    for name, d in per.items():
        fetch = d["FETCH_SIZE"][0] * factor["FETCH_SIZE"]
        write = d["WRITE_SIZE"][0] * factor["WRITE_SIZE"]
        out["kernels"][name] = {"fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
                                "hbm_bytes_per_launch": fetch + write, "dispatches": d["FETCH_SIZE"][1]}
        lines.append("| %s | %d | %.1f MB | %.1f MB | %.1f MB |" % (
            name, d["FETCH_SIZE"][1], fetch / 1e6, write / 1e6, (fetch + write) / 1e6))
    out["copy_factor"] = factor
    path = os.path.join(HERE, "profiles", "spring_counters.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("copy calibration factor (true bytes / counted bytes): FETCH %.4f  WRITE %.4f"
          % (factor["FETCH_SIZE"], factor["WRITE_SIZE"]))
    print("| kernel | dispatches | FETCH (scaled) | WRITE (scaled) | HBM bytes / launch |")
    print("|---|---|---|---|---|")
    print("\n".join(lines))
    print("written", path)


def counter_pass(args, torch):
    """Profiling aid for rocprofv3 --pmc (one counter per run): rebuilds the
    bench's mesh, applies the launch shapes a bench run timed (its JSON line,
    args.counter_pass), runs as many real steps as that run did before its
    per-kernel timing pass, then the same timing pass (50 force launches, 50
    node launches with dt = 0) and, with --calibrate-copy, the calibration
    copies.  So the profiled window sees the same live objects as the bench's.
    Prints progress to stderr and a JSON line with the window's dispatch
    indices."""
    from inputs import spring_mesh
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.sims import SpringSim

    with open(args.counter_pass) as f:
        ref = json.loads([ln for ln in f if ln.startswith("{")][-1])
    n = int(ref["trace_window"]["after_steps"])
    sim = SpringSim(spring_mesh(1000, 1000), 1e-5, 0.3)
    heap = sim.heap
    lib = smmo.load_library()
    stream = torch.cuda.current_stream().cuda_stream
    hp, cs, cn = heap.h, heap.cls["Spring"], heap.cls["Node"]
    argp, asz = smmo.C.byref(sim.args), smmo.C.sizeof(sim.args)
    tuned = ref.get("autotune") or {}
    if tuned.get("kept") == "tuned":
        for m, cls, key in ((sim.m_force, cs, "spring.force"), (sim.m_node, cn, "spring.node_update")):
            t = tuned[key]
            smmo.smmo_set_launch(hp, m, cls, t["wg"], t["waves"], t.get("group", 0))
    for i in range(n):
        lib.smmo_parallel_do(hp, cs, sim.m_force, argp, asz, stream)
        lib.smmo_parallel_do(hp, cn, sim.m_node, argp, asz, stream)
        if (i + 1) % 1000 == 0:
            torch.cuda.synchronize()
            print("counter pass: %d of %d steps" % (i + 1, n), file=sys.stderr, flush=True)
    frozen = smmo.smmo_spring_args(sim.args.node_class, sim.args.spring_class, 0.0, sim.args.strain_limit,
                                    sim.args.flags)
    ks = args.kernel_steps
    for _ in range(ks):
        lib.smmo_parallel_do(hp, cs, sim.m_force, smmo.C.byref(frozen), asz, stream)
    for _ in range(ks):
        lib.smmo_parallel_do(hp, cn, sim.m_node, smmo.C.byref(frozen), asz, stream)
    torch.cuda.synchronize()
    st = heap.stats()
    print(json.dumps({"counter_pass_of": ref.get("config", {}).get("workload"), "steps_before": n,
                      "live_springs": int(st.live_objects[cs]),
                      "trace_window": {"spring.force": [n, n + ks], "spring.node_update": [n, n + ks]},
                      "kernels": ref.get("kernels")}), flush=True)
    if args.calibrate_copy:
        calibrate_copy(torch)


def alloc_pass(torch):
    """Profiling aid for rocprofv3 --pmc on the allocator-bound kernels: Game
    of Life 256 x 256 (50 generations), wa-tor 512 x 512 (50 iterations) and
    the Linux Scalability pattern (16,384 workers, n = 64).  Prints progress
    to stderr."""
    from inputs import config_seed, gol_init, wator_init
    from paper_1908_05845_amd import smmo
    from paper_1908_05845_amd.sims import GolSim, WatorSim

    sim = GolSim(256, 256, gol_init(256, 256))
    sim.step(50)
    sim.heap.sync()
    print("alloc pass: gol done", file=sys.stderr, flush=True)
    w = WatorSim(512, 512, config_seed(7), (4, 12, 8, 4), wator_init(512, 512))
    w.step(50)
    w.heap.sync()
    print("alloc pass: wa-tor done", file=sys.stderr, flush=True)
    heap = smmo.Heap({"Worker": [("id", "i32", 1)], "Obj": [("payload", "u32", 16)]}, nbytes=1 << 28)
    heap.new("Worker", 16384, id=torch.arange(16384, dtype=torch.int32, device="cuda"))
    handles = torch.full((64 * 16384,), -1, dtype=torch.int32, device="cuda")
    args = smmo.smmo_ls_args(heap.cls["Obj"], 64, 16384, 0, handles.data_ptr())
    heap.do("Worker", "alloc.ls_alloc", args)
    heap.do("Worker", "alloc.ls_free", args)
    heap.sync()
    print("alloc pass: linux scalability done", file=sys.stderr, flush=True)
    print(json.dumps({"alloc_pass": "gol 256x256 x 50, wa-tor 512x512 x 50, linux scalability n=64"}), flush=True)


def summarize_l2(dirs):
    """Per kernel: L2 hit rate (TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum))
    and atomics per dispatch (TCC_ATOMIC_sum at the L2, TCC_EA0_ATOMIC_sum
    towards memory), from rocprofv3 --pmc runs given as directories."""
    import re
    from collections import defaultdict

    acc = defaultdict(lambda: defaultdict(float))
    cnt = defaultdict(lambda: defaultdict(int))
    for d in dirs:
        for r in _read_counter_csv(d):
            name = re.sub(r"\(.*", "", r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", ""))
            acc[name][r["Counter_Name"]] += float(r["Counter_Value"])
            cnt[name][r["Counter_Name"]] += 1
    print("| kernel | dispatches | L2 hit rate | L2 atomics / dispatch | atomics to memory / dispatch |")
    print("|---|---|---|---|---|")
    for name in sorted(acc, key=lambda k: -acc[k].get("TCC_ATOMIC_sum", 0.0)):
        a, c = acc[name], cnt[name]
        if not (name.startswith("k_") or "copyBuffer" in name):
            continue
        hit, miss = a.get("TCC_HIT_sum"), a.get("TCC_MISS_sum")
        rate = "%.1f %%" % (100.0 * hit / (hit + miss)) if hit is not None and miss is not None and hit + miss else "-"
        at = "%.0f" % (a["TCC_ATOMIC_sum"] / c["TCC_ATOMIC_sum"]) if c.get("TCC_ATOMIC_sum") else "-"
        ea = "%.0f" % (a["TCC_EA0_ATOMIC_sum"] / c["TCC_EA0_ATOMIC_sum"]) if c.get("TCC_EA0_ATOMIC_sum") else "-"
        n = max(c.values())
        print("| %s | %d | %s | %s | %s |" % (name, n, rate, at, ea))


def summarize_trace(trace_dir, bench_json):
    """Average kernel durations from a rocprofv3 kernel trace: over the bench's
    timing-pass window (the same dispatches its HIP events timed) and over
    the whole run, next to the bench's own figures."""
    import csv
    import glob

    with open(bench_json) as f:
        line = json.loads([ln for ln in f if ln.startswith("{")][-1])
    rows = []
    for fn in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        with open(fn) as f:
            rows.extend(csv.DictReader(f))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    print("| kernel | dispatches | window | rocprofv3 avg in window (us) | bench HIP-event avg (us) "
          "| rocprofv3 avg whole run (us) |")
    print("|---|---|---|---|---|---|")
    for name, key in KERNEL_KEYS.items():
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3 for r in rows if key in r["Kernel_Name"]]
        lo, hi = line["trace_window"][name]
        win = d[lo:hi]
        print("| %s | %d | [%d, %d) | %.2f | %.2f | %.2f |" % (
            name, len(d), lo, hi, sum(win) / max(len(win), 1), line["kernels"][name]["avg_us"],
            sum(d) / max(len(d), 1)))


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_l2:
        summarize_l2(args.summarize_l2)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1908_05845_amd import smmo

    smmo.load_library()
    for spec in args.launch:
        name, vals = spec.split("=")
        GIVEN_SHAPES[name] = tuple(int(v) for v in vals.split(","))
    if GIVEN_SHAPES and set(GIVEN_SHAPES) != {"spring.force", "spring.node_update"}:
        print("--launch needs spring.force and spring.node_update", file=sys.stderr)
        sys.exit(2)
    if args.extra:
        fn = globals()[STANDALONE_EXTRAS[args.extra]]
        # the measurements compared with the plain mesh's rate get none alone
        res = fn(torch, None) if args.extra in ("batched", "adjoint") else fn(torch)
        print(json.dumps({args.extra: res}), flush=True)
        return
    if args.counter_pass:
        counter_pass(args, torch)
        return
    if args.alloc_pass:
        alloc_pass(torch)
        return
    fn = {"spring": bench_spring, "gol": bench_gol, "nbody": bench_nbody}[args.workload]
    res, cpu_leg, steps, warmup = fn(args, torch)
    extras = {}
    if args.workload == "spring" and not args.no_extras:
        def extra(name, fn, *a):
            # a failed extra is recorded in the line (and on stderr); the
            # headline figures above stand, and the other extras still run
            try:
                extras[name] = fn(*a)
            except Exception as e:
                print("extras: %s failed: %r" % (name, e), file=sys.stderr, flush=True)
                extras[name] = {"error": repr(e)[:500]}

        extra("copy_bandwidth", measure_copy_bandwidth, torch)
        extra("coalescing", measure_coalescing, torch)
        extra("allocation", measure_allocation, torch)
        extra("enumeration", measure_enumeration, torch)
        extra("batched", measure_batched, torch, res["value"])
        extra("adjoint", measure_adjoint, torch, res["value"])
        extra("gol", measure_gol_extra, torch)
        extra("gol_16384", measure_gol_large, torch)
        extra("structure", measure_structure, torch)
        extra("generation", measure_generation, torch)
        extra("partial_inlining", measure_spring_pi, torch)
        extra("spring_2000", measure_spring_large, torch)
        extra("nbody", measure_nbody_extra, torch)
        extra("linux_scalability", measure_linux_scalability, torch)
        extra("wator", measure_wator, torch)
    cpu = None if args.no_cpu_baseline else cpu_leg()
    if cpu is not None:
        cpu["cpu_model"] = _cpu_model()
        cpu["host_nproc"] = os.cpu_count()
        if args.workload == "spring" and not args.no_extras:
            for name, rec in cpu_baselines_of_extras().items():
                if isinstance(extras.get(name), dict):
                    extras[name]["cpu_baseline"] = rec
    line = {
        "metric": METRIC,
        "value": res["value"],
        "unit": res["unit"],
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": res["dtype"],
        "data": "synthetic",
        "config": res["config"],
        "roofline": res["roofline"],
        "cpu_baseline": cpu,
    }
    for k in ("step_hbm", "kernels", "autotune", "launch", "trace_window", "device_error", "defrag", "segments"):
        if k in res:
            line[k] = res[k]
    line.update(extras)
    print(json.dumps(line), flush=True)
    if args.calibrate_copy:
        calibrate_copy(torch)


def cpu_baselines_of_extras():
    """The float64 oracle timed on the other configurations, each on the
    bounded sample its own cost allows (the host's threads for the do-alls
    that use them): Game of Life 256 x 256 for all 100 generations, n-body
    65,536 for 2 steps, the 256-mesh batch for 10 steps, the adjoint
    configuration (316 x 317, 200 steps, checkpoints every 20) in full."""
    from inputs import batched_meshes, concat_meshes, gol_init, nbody_init, spring_mesh
    from oracle import GolWorld, nbody_steps, spring_adjoint, spring_steps, threads

    out = {}
    init = gol_init(256, 256)
    t = time.perf_counter()
    w = GolWorld(256, 256, init)
    w.step(100)
    el = time.perf_counter() - t
    out["gol"] = {"value": 100 * 2 * 256 * 256 / el, "unit": "cell updates/s", "cores": 1, "kind": "oracle",
                  "sample": "all 100 generations from the same start, %.1f s" % el}
    s = nbody_init(65536)
    n = 65536
    t = time.perf_counter()
    nbody_steps(s["x"], s["y"], s["vx"], s["vy"], s["m"], 1.0 / n, 1e-3, 1e-4, 2)
    el = time.perf_counter() - t
    out["nbody"] = {"value": 2.0 * n * n / el, "unit": "pairs/s", "cores": threads(), "kind": "oracle",
                    "sample": "first 2 of the 50 steps, %.1f s" % el}
    mesh = concat_meshes(batched_meshes(256))
    t = time.perf_counter()
    r = spring_steps(mesh, 1e-5, 0.3, 10)
    el = time.perf_counter() - t
    out["batched"] = {"value": 10 * (mesh["N"] + 0.5 * (mesh["S"] + int(r["alive"].sum()))) / el,
                      "unit": "updates/s", "cores": threads(), "kind": "oracle",
                      "sample": "first 10 of the 1,000 steps (load, steps, unload), %.1f s" % el}
    mesh = spring_mesh(316, 317)
    t = time.perf_counter()
    spring_adjoint(mesh, 1e-5, 200, every=20)
    el = time.perf_counter() - t
    out["adjoint"] = {"value": el * 1e3, "unit": "ms per forward + checkpointed reverse sweep",
                      "cores": threads(), "kind": "oracle", "sample": "the whole configuration, %.1f s" % el}
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
