"""Benchmark: elements/s of J + exact grad J for 3D Neo-Hookean on ~6M tetrahedra (one GPU).

One step = one energy-and-gradient evaluation through the autograd hook
(``p1_energy(vhat).backward()``: element tiles with energy, forces and in-tile patch sums,
halo rows, compensated finalize; the backward scales the forward's gradient buffer in place,
which writes nothing for dJ/dJ = 1) on the 460x46x46-cube Kuhn box (5,840,160 tets), mixed
precision, inputs resident in HBM. Prints ONE JSON line with:

* value / ms_per_step: K steps bracketed by device synchronisations (wall clock), after W
  untimed steps (the default W = 500, about 60 ms of work, brings the GPU out of the idle
  clock state the host-side oracle timing leaves it in), and the median from HIP events around
  each step of a second pass; the step is timed in two forms, issued eagerly from Python
  (eager_autograd) and as replays of the step captured once in a HIP graph (GraphedStep,
  graph_replay), and the faster is reported (step_form): the eager rate depends on how fast
  the host issues a step, a replay costs a few microseconds of GPU time for the graph launch.
  The replays' J and gradient equal the eager step's bitwise
  (graph_replay_bitwise_equal_eager);
* roofline: the dominant kernel against the HBM roofline (HIP events around each kernel over
  a third pass), with the counter-measured traffic and VALU-issue fraction when a profile of
  the current kernel sources is committed;
* oracle_rel_err: the FP64 oracle's error of every timed result (mixed and FP64 J + exact
  gradient on the whole mesh; patch central differences on sampled DOFs);
* extras: FP64 J + grad J, the patch differences (second and fourth order) on the same mesh,
  the mixed J + grad J on the 930x93x93-cube box (48,261,420 tets, a working set far above
  the 256 MB last-level cache), and on a jittered 6M-tet box with no geometry classes
  (element geometry formed from the vertex coordinates, and stored per element);
* cpu_baseline: the oracle (plain C element loops) timed on the host before the GPU is
  touched, on all host cores (one process per contiguous element range) and on one core,
  median of 5;
* serve: the serving benchmark (256 minimization requests, Poisson arrivals, continuous
  batching vs one-at-a-time FP64 solves: req/s, p50/p99 latency, with and without mesh setup).

Usage: python bench.py [--gpus 1] [--steps 200] [--warmup 500] [--no-cpu-baseline] [--no-serve]
                [--no-graph]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
MAX_CPU_WORKERS = 16   # host share of one GPU


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--config", default="nh3d_box_6M")
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip FP64, FD and 48M timings")
    ap.add_argument("--no-large", action="store_true", help="skip the 48M-tet timing")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving benchmark")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the eager step only (no HIP graph capture)")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-iters", type=int, default=200)
    ap.add_argument("--fd-sample", type=int, default=3000,
                    help="DOFs at which the oracle checks the patch differences")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run plain device-to-device copies of this many MiB (a reference "
                         "for hardware byte counters)")
    return ap.parse_args()


def algorithmic_bytes(info, prec):
    """Compulsory HBM bytes of one J + exact grad J call, per kernel (each array touched once).

    k_tile_force: local connectivity 2(dim+1) B per element and its geometry (by the mesh's
    geometry mode: a one-byte class per element; or B^-1 and |T|, dim^2 + 1 words per element;
    or, formed on the fly, a coordinate offset of dim words per tile node); local patch
    entries 2 B per free-node incidence; the tile
    node records (node, record, slot: 12 B; row pointer: 2 B) per tile node; per node the
    DOF map 4 B and the subtrahend/prescribed values 8d B; per free DOF vhat and b read and
    g written (rows complete in one tile); per free row its row info 4 B; the halo partial
    sums d words per slot written (FP32 in mixed precision). k_halo: per halo row 8 B of row
    index and pointer, its row info 4 B, b read and g written (8d B each); per slot its index
    4 B and partial d words read. k_scale_inplace: the incoming gradient is 1 here, so the kernel reads its 8-byte
    scale and writes nothing (with another scale: 16 B per free DOF)."""
    ne, nn, nf, nfd, nnz = (info["ne"], info["nn"], info["n_free_nodes"], info["n_free_dofs"],
                            info["nnz"])
    dim, d = info["dim"], info["ncomp"]
    w = 4 if prec == "mixed" else 8
    tn, nh, ns = info["n_tile_nodes"], info["n_halo_rows"], info["n_halo_slots"]
    mode = info["geometry_mode"]
    geo = ne if mode == 1 else ne * w * (dim * dim + 1) if mode == 0 else tn * w * dim
    complete_dofs = d * (nf - nh)
    tile = (ne * 2 * (dim + 1) + geo + 2 * nnz + 14 * tn + nn * (4 + 8 * d) + 16 * nfd
            + 4 * nf + 8 * complete_dofs + w * d * ns)
    halo = nh * (12 + 16 * d) + ns * (4 + w * d)
    return {"k_tile_force": tile, "k_halo": halo, "k_scale_inplace": 0}


def kernel_source_hash():
    """Hash of the code (comments and blank lines dropped) of the sources the profiled kernels
    are built from: a profile stays valid across edits of comments only."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("p1e_device.h", "p1e_kernels.hip", "p1e_internal.h", "p1e_tiles.cpp"):
        with open(os.path.join(ROOT, "paper_2109_01158_amd", "csrc", f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def profile_record(config, prec):
    """The committed counter summary of this workload (HBM traffic and VALU issue per kernel),
    or None if there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_jgrad_{prec}_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t


# ------------------------------------------------------------------ host CPU and the oracle
def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "available": avail}


def _oracle_range_worker(prob, lo, hi, rounds, barrier, q):
    """One process of the all-core timing: the oracle on elements [lo, hi) of the mesh (its
    geometry set up before the first round), energy + exact gradient once per round; each
    round starts at a barrier shared by all workers."""
    from dataclasses import replace
    import oracle
    O = oracle.Oracle(replace(prob, conn=prob.conn[lo:hi]))
    O.energy(prob.v)
    O.grad_exact(prob.v)
    for r in range(rounds):
        barrier.wait()
        t0 = time.perf_counter()
        O.energy(prob.v)
        O.grad_exact(prob.v)
        q.put((r, time.perf_counter() - t0))


def cpu_leg(prob, fd_sample, rounds=5, seed=7):
    """Oracle references for the timed GPU results, and the oracle's own speed on the host.
    Runs before the GPU is initialised (the all-core timing forks worker processes)."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    oracle.build(force=False)
    O = oracle.Oracle(prob)
    ref = O.energy(prob.v)
    gref = O.grad_exact(prob.v)
    one = []
    for _ in range(rounds):
        t0 = time.perf_counter()
        O.energy(prob.v)
        O.grad_exact(prob.v)
        one.append(time.perf_counter() - t0)
    rng = np.random.default_rng(seed)
    nfd = prob.n_free_dofs
    sample = np.sort(rng.choice(nfd, size=min(fd_sample, nfd), replace=False))
    fd = O.grad_patch_fd(prob.v, prob.eps, sample=sample, with_cond=True)
    fd4 = O.grad_patch_fd(prob.v, prob.eps, sample=sample, with_cond=True, order=4)
    del O
    # all cores: one process per contiguous element range
    cpu = host_cpu()
    P = max(1, min(MAX_CPU_WORKERS, cpu["available"] or 1))
    ctx = mp.get_context("fork")
    barrier = ctx.Barrier(P)
    q = ctx.Queue()
    cuts = np.linspace(0, prob.ne, P + 1).astype(np.int64)
    procs = [ctx.Process(target=_oracle_range_worker,
                         args=(prob, int(cuts[i]), int(cuts[i + 1]), rounds, barrier, q))
             for i in range(P)]
    for p in procs:
        p.start()
    per_round = [[] for _ in range(rounds)]
    for _ in range(P * rounds):
        r, dt = q.get(timeout=600)
        per_round[r].append(dt)
    for p in procs:
        p.join()
    wall = [max(x) for x in per_round]
    t_all, t_one = float(np.median(wall)), float(np.median(one))
    base = {
        "value": prob.ne / t_all, "unit": "elements/s", "cores": P, "kind": "oracle",
        "sample": f"energy + exact gradient over the full {prob.ne}-element mesh, FP64 C element "
                  f"loops, {P} processes on contiguous element ranges, median of {rounds} rounds "
                  f"({t_all:.3f} s per round)",
        "single_thread": {"value": prob.ne / t_one, "cores": 1,
                          "sample": f"the same on one core, median of {rounds} ({t_one:.3f} s)"},
        "host_cpu": cpu,
    }
    refs = {"J": ref["J"], "g": gref, "sample": sample, "fd": fd, "fd4": fd4}
    return base, refs


def _rel(a, b):
    import numpy as np
    a, b = np.atleast_1d(a), np.atleast_1d(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def fd_errors(g, ref, v_free, eps, order):
    """Relative 2-norm error over the sample, and the largest per-DOF ratio to the parity
    bound of the tests: 32u cond/(2 eps) + 4u(|v| + h)/eps gabs + 1e-12|g_ref| with the
    oracle's rounding scales cond and gabs of the scheme, h its largest step."""
    import numpy as np
    u = 2.0 ** -53
    gref, cond, gabs = ref
    step = eps if order == 2 else 2 * eps
    tol = (32 * u * cond / (2 * eps) + 4 * u * (np.abs(v_free) + step) / eps * gabs
           + 1e-12 * np.abs(gref))
    return {"rel_err_2norm": _rel(g, gref),
            "max_err_over_bound": float(np.max(np.abs(g - gref) / tol))}


# ------------------------------------------------------------------ GPU timing helpers
def time_steps(fn, steps):
    """Wall clock of `steps` calls bracketed by synchronisations, ms per call."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def median_step_ms(fn, steps):
    """Median of per-call HIP event times on the current stream (no synchronisation between
    calls)."""
    import numpy as np
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def large_timing(P, steps, warmup):
    """Mixed J + grad J through the autograd hook on the 48M-tet box (930x93x93 cubes)."""
    import torch
    import p1e_synth as S
    t0 = time.perf_counter()
    prob = S.config_problem("nh3d_box_48M")
    mesh = P.Mesh.from_problem(prob, modes=P.P1E_MIXED)
    setup = time.perf_counter() - t0
    info = mesh.info
    vhat = torch.tensor(prob.vhat(), device="cuda").requires_grad_(True)
    seed = torch.ones((), dtype=torch.float64, device="cuda")

    def step():
        vhat.grad = None
        J = P.p1_energy(vhat, mesh, "mixed")
        torch.autograd.backward(J, seed)

    for _ in range(warmup):
        step()
    ms = time_steps(step, steps)
    med = median_step_ms(step, steps)
    P.prof_reset()
    P.prof_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    P.prof_enable(False)
    kern = {k: 1e3 * t / c for k, (c, t) in P.prof_collect().items()}
    ab = algorithmic_bytes(info, "mixed")
    out = {"workload": "nh3d_box_48M: 930x93x93 cubes x 6 Kuhn tets, mixed J + exact grad J "
                       "through the autograd hook",
           "ne": info["ne"], "elements_per_s": info["ne"] / (ms * 1e-3), "ms": ms,
           "ms_median": med, "kernels_avg_us": kern,
           "k_tile_alg_GBs": ab["k_tile_force"] / (kern["k_tile_force"] * 1e-6) / 1e9,
           "bound_buffer_bytes": mesh.nbytes, "setup_s": setup}
    del vhat, mesh
    torch.cuda.empty_cache()
    return out


def geometry_timing(P, steps, warmup):
    """Mixed J + grad J on the 6M-tet box with interior nodes jittered by up to 0.2 h (every
    element its own shape: no geometry classes), with B^-1 and |T| formed in the element pass
    from the vertex coordinates (the default) and stored per element (P1E_FULL_GEOMETRY)."""
    import torch
    import p1e_synth as S
    prob = S.neohooke_box_3d(460, 46, 46, seed=0, jitter=0.2)
    out = {"workload": "nh3d_box_6M with interior nodes jittered by up to 0.2 h (no geometry "
                       "classes): mixed J + exact grad J through the autograd hook"}
    for flags, name in ((0, "on_the_fly"), (P.P1E_FULL_GEOMETRY, "stored_per_element")):
        mesh = P.Mesh.from_problem(prob, modes=P.P1E_MIXED, flags=flags)
        info = mesh.info
        vhat = torch.tensor(prob.vhat(), device="cuda").requires_grad_(True)
        seed = torch.ones((), dtype=torch.float64, device="cuda")

        def step():
            vhat.grad = None
            J = P.p1_energy(vhat, mesh, "mixed")
            torch.autograd.backward(J, seed)

        for _ in range(warmup):
            step()
        ms = time_steps(step, steps)
        P.prof_reset()
        P.prof_enable(True)
        time_steps(step, steps)
        P.prof_enable(False)
        kern = {k: 1e3 * t / c for k, (c, t) in P.prof_collect().items()}
        ab = algorithmic_bytes(info, "mixed")
        ach = ab["k_tile_force"] / (kern["k_tile_force"] * 1e-6) / 1e9
        out[name] = {"geometry_mode": info["geometry_mode"], "n_tiles": info["n_tiles"],
                     "elements_per_s": info["ne"] / (ms * 1e-3), "ms": ms,
                     "kernels_avg_us": kern, "bound_buffer_bytes": mesh.nbytes,
                     "k_tile_alg_bytes_per_element": ab["k_tile_force"] / info["ne"],
                     "k_tile_roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}}
        del vhat, mesh
        torch.cuda.empty_cache()
    return out


def main():
    a = _args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(json.dumps({"error": "single-GPU build: bench.py measures one MI355X only; "
                          "sharding across GPUs is not implemented",
                          "n_gpus": a.gpus}))
        sys.exit(2)

    import p1e_synth as S
    prob = S.config_problem(a.config)
    # the oracle leg first: it forks worker processes, which must not inherit a GPU context
    base, refs = (None, None) if a.no_cpu_baseline else cpu_leg(prob, a.fd_sample)

    import numpy as np
    import torch
    import paper_2109_01158_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    modes = P.P1E_MIXED if a.prec == "mixed" else P.P1E_FP64
    if not a.no_extras:
        modes |= P.P1E_FP64 | P.P1E_FD
    t0 = time.perf_counter()
    mesh = P.Mesh.from_problem(prob, modes=modes, device=dev)
    setup_s = time.perf_counter() - t0
    info = mesh.info
    vhat0 = torch.tensor(prob.vhat(), device=dev)
    vhat = vhat0.clone().requires_grad_(True)
    seed = torch.ones((), dtype=torch.float64, device=dev)  # dJ/dJ, allocated once
    res = {}

    def step():
        vhat.grad = None
        J = P.p1_energy(vhat, mesh, a.prec)
        torch.autograd.backward(J, seed)
        res["J"] = J

    for _ in range(a.warmup):
        step()
    # eager autograd steps: K steps bracketed by device synchronisations, then the median of
    # per-step HIP events (these include the host's time to issue each step whenever the host
    # is slower than the GPU)
    ms_eager = time_steps(step, a.steps)
    ms_median_eager = median_step_ms(step, a.steps)
    J_eager = float(res["J"].item())
    g_eager = vhat.grad.detach().clone()
    # every library kernel bracketed by HIP events on its launch stream: per-kernel durations
    # for the roofline (the events themselves cost a few us per kernel)
    P.prof_reset()
    P.prof_enable(True)
    ms_events = time_steps(step, a.steps)
    P.prof_enable(False)
    kern = P.prof_collect()
    # the same autograd step captured once in a HIP graph and replayed (the step's kernels for
    # one graph launch), K replays bracketed by device synchronisations, then the median of
    # per-replay HIP events; J and the gradient of the replays must equal the eager step's
    # bitwise. The faster of the two forms is reported (a slow host favours the graph, whose
    # launch costs a few microseconds of GPU time).
    gstep, ms_graph, ms_median_graph, graph_bitwise, graph_error = None, None, None, None, None
    J_timed, g_timed = J_eager, g_eager.cpu().numpy()
    if not a.no_graph:
        try:
            gstep = P.GraphedStep(vhat, mesh, a.prec)
        except RuntimeError as e:  # a capture the runtime refuses: report the eager step only
            graph_error = str(e)[:200]
            torch.cuda.synchronize()
        if gstep is not None:
            for _ in range(20):
                gstep.replay()
            ms_graph = time_steps(gstep.replay, a.steps)
            ms_median_graph = median_step_ms(gstep.replay, a.steps)
            graph_bitwise = (float(gstep.J.item()) == J_eager
                             and bool(torch.equal(gstep.grad, g_eager)))
            if graph_bitwise:
                J_timed, g_timed = float(gstep.J.item()), gstep.grad.detach().cpu().numpy()
    del g_eager
    # the graph form is reported only if its results equal the eager step's
    step_form = "graph" if graph_bitwise and ms_graph < ms_eager else "eager"
    ms, ms_median = (ms_graph, ms_median_graph) if step_form == "graph" else (ms_eager,
                                                                           ms_median_eager)
    value = info["ne"] / (ms * 1e-3)

    abytes = algorithmic_bytes(info, a.prec)
    kstats = {k: {"launches": c, "avg_us": 1e3 * t / c} for k, (c, t) in kern.items()}
    dom = max(kstats, key=lambda k: kstats[k]["avg_us"])
    dom_bytes = abytes.get(dom)
    achieved = dom_bytes / (kstats[dom]["avg_us"] * 1e-6) / 1e9 if dom_bytes else None
    for k, s in kstats.items():
        if k in abytes:
            s["alg_GBs"] = abytes[k] / (s["avg_us"] * 1e-6) / 1e9
    step_bytes = sum(abytes.values())
    prof = profile_record(a.config, a.prec)
    hbm_frac = achieved / HBM_PEAK_GBS if achieved else None
    issue_frac = (prof or {}).get("valu_issue", {}).get(dom, {}).get("frac")
    limiter = None
    if issue_frac is not None and hbm_frac is not None:
        limiter = "valu_issue" if issue_frac > hbm_frac else "hbm"

    errs = {}
    if refs is not None:
        errs[f"{a.prec}_jgrad"] = {"J": _rel(J_timed, refs["J"]), "grad": _rel(g_timed, refs["g"])}

    extras = {}
    if not a.no_extras:
        # FP64 J + grad J and the FP64 patch central differences on the same mesh
        g = torch.empty_like(vhat0)
        out3 = torch.empty(3, dtype=torch.float64, device=dev)
        flag = torch.empty(1, dtype=torch.int32, device=dev)
        last = {}

        def fd2():
            last["fd"] = mesh.grad_patch_fd(vhat0, prob.eps)

        def fd4():
            last["fd4"] = mesh.grad_patch_fd4(vhat0, prob.eps)

        for name, fn in (("fp64_jgrad", lambda: mesh.grad_exact(vhat0, "fp64", g=g, out3=out3,
                                                                  flag=flag)),
                         ("patch_fd_fp64", fd2), ("patch_fd4_fp64", fd4)):
            for _ in range(2):
                fn()
            n = max(3, a.steps // 2)
            dt = time_steps(fn, n)
            extras[name] = {"elements_per_s": info["ne"] / (dt * 1e-3), "ms": dt,
                            "ms_median": median_step_ms(fn, n)}
        if refs is not None:
            errs["fp64_jgrad"] = {"J": _rel(out3[0].item(), refs["J"]),
                                  "grad": _rel(g.cpu().numpy(), refs["g"])}
            v_free = prob.vhat()[refs["sample"]]
            for key, name, order in (("fd", "patch_fd_fp64", 2), ("fd4", "patch_fd4_fp64", 4)):
                gs = last[key][0].cpu().numpy()[refs["sample"]]
                r = refs[key]
                errs[name] = dict(fd_errors(gs, r, v_free, prob.eps, order),
                                  sampled_dofs=int(refs["sample"].size))
    if a.copy_calibration > 0:
        src = torch.empty(a.copy_calibration << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    out = {
        "metric": "elements/s for J+∇J (3D Neo-Hookean, 6M tets); serve req/s + p50/p99",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "ms_per_step_median": ms_median,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64" if a.prec == "mixed" else "fp64",
        "data": "synthetic (seeded mesh and displacement field)",
        "config": {
            "workload": f"{a.config}: 3D Neo-Hookean box [0,1]x[0,0.1]^2, 460x46x46 cubes x 6 Kuhn "
                        f"tets, E=2e8 nu=0.3, x=0 face clamped, u=amp*U[-1,1] (amp={prob.amp:.3g}); "
                        f"J + exact grad J through the autograd hook, {a.prec}; timed as "
                        f"issued eagerly and as replays of the step captured in a HIP graph, "
                        f"the faster reported (step_form)",
            "ne": info["ne"], "nn": info["nn"], "n_free_dofs": info["n_free_dofs"],
            "patch_incidences": info["nnz"], "parallelism": "single GPU",
        },
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": hbm_frac,
                     "traffic": (prof or {}).get("traffic_bytes_per_launch", {}).get(dom),
                     "alg_bytes_per_launch": dom_bytes,
                     "alg_bytes_per_element": dom_bytes / info["ne"] if dom_bytes else None,
                     "valu_issue_frac_profiled": issue_frac,
                     "limiter": limiter},
        "ms_per_step_with_kernel_events": ms_events,
        "step_form": step_form,
        "eager_autograd": {"value": info["ne"] / (ms_eager * 1e-3), "ms_per_step": ms_eager,
                           "ms_per_step_median": ms_median_eager},
        "graph_replay": None if a.no_graph else (
            {"error": graph_error} if gstep is None else {
                "value": info["ne"] / (ms_graph * 1e-3), "ms_per_step": ms_graph,
                "ms_per_step_median": ms_median_graph}),
        "graph_replay_bitwise_equal_eager": graph_bitwise,
        "step_alg_bytes_per_element": step_bytes / info["ne"],
        "step_alg_GBs": step_bytes / (ms * 1e-3) / 1e9,
        "kernels": kstats,
        "J": J_timed,
        "oracle_rel_err": errs,
        "setup_s": setup_s,
        "extras": extras,
    }
    if base is not None:
        out["cpu_baseline"] = base
    del gstep, mesh, vhat, vhat0
    torch.cuda.empty_cache()
    if not a.no_extras and not a.no_large:
        extras["nh3d_box_48M_mixed_jgrad"] = large_timing(P, a.steps, a.warmup)
    if not a.no_extras:
        extras["jittered_6M_geometry"] = geometry_timing(P, a.steps, a.warmup)
    if not a.no_serve:
        from paper_2109_01158_amd import serving
        out["serve"] = serving.benchmark(
            n_requests=a.serve_requests, iters=a.serve_iters,
            log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
