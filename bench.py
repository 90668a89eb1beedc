"""Benchmark: elements/s of J + exact grad J for 3D Neo-Hookean on ~6M tetrahedra (one GPU).

One step = one energy-and-gradient evaluation through the autograd hook
(``p1_energy(vhat).backward()``: element tiles with energy, forces and in-tile patch sums,
halo rows, compensated finalize; the backward scales the forward's gradient buffer in place,
which writes nothing for dJ/dJ = 1) on the 460x46x46-cube Kuhn box (5,840,160 tets), mixed
precision, inputs resident in HBM. Prints ONE JSON line. Extra fields report the FP64 path, the patch central-difference
gradient on the same mesh, the serving benchmark (256 minimization requests, Poisson arrivals,
continuous batching vs one-at-a-time FP64 solves: req/s, p50/p99 latency), the dominant kernel against the HBM roofline (HIP events around
each kernel over a second pass of the same K steps) and the FP64 oracle timed on the host CPU.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline] [--no-serve]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="nh3d_box_6M")
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip FP64 and FD extra timings")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving benchmark")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-iters", type=int, default=200)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run plain device-to-device copies of this many MiB (a reference "
                         "for hardware byte counters)")
    return ap.parse_args()


def algorithmic_bytes(info, prec, classed):
    """Compulsory HBM bytes of one J + exact grad J call, per kernel (each array touched once).

    k_tile_force: local connectivity 2(dim+1) B and the geometry class 1 B (or B^-1 and |T|,
    dim^2 + 1 words) per element; local patch entries 2 B per free-node incidence; the tile
    node records (node, record, slot: 12 B; row pointer: 2 B) per tile node; per node the
    DOF map 4 B and the subtrahend/prescribed values 8d B; per free DOF vhat and b read and
    g written (rows complete in one tile); per free row its row info 4 B; the halo partial
    sums 8d B per slot written. k_halo: per halo row 8 B of row index and pointer, its row
    info 4 B, b read and g written (8d B each); per slot its index 4 B and partial 8d B
    read. k_scale_inplace: the incoming gradient is 1 here, so the kernel reads its 8-byte
    scale and writes nothing (with another scale: 16 B per free DOF)."""
    ne, nn, nf, nfd, nnz = (info["ne"], info["nn"], info["n_free_nodes"], info["n_free_dofs"],
                            info["nnz"])
    dim, d = info["dim"], info["ncomp"]
    w = 4 if prec == "mixed" else 8
    tn, nh, ns = info["n_tile_nodes"], info["n_halo_rows"], info["n_halo_slots"]
    geo = ne if classed else ne * w * (dim * dim + 1)
    complete_dofs = d * (nf - nh)
    tile = (ne * 2 * (dim + 1) + geo + 2 * nnz + 14 * tn + nn * (4 + 8 * d) + 16 * nfd
            + 4 * nf + 8 * complete_dofs + 8 * d * ns)
    halo = nh * (12 + 16 * d) + ns * (4 + 8 * d)
    return {"k_tile_force": tile, "k_halo": halo, "k_scale_inplace": 0}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("p1e_device.h", "p1e_kernels.hip", "p1e_internal.h", "p1e_tiles.cpp"):
        with open(os.path.join(ROOT, "paper_2109_01158_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
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


def cpu_baseline(prob, target_s=12.0):
    """The FP64 oracle (single-threaded C loops) on the same mesh: energy + exact gradient,
    repeated until about target_s seconds of CPU time."""
    import oracle
    oracle.build(force=False)
    O = oracle.Oracle(prob)
    reps, t = 0, 0.0
    while t < target_s and reps < 20:
        t0 = time.perf_counter()
        O.energy(prob.v)
        O.grad_exact(prob.v)
        t += time.perf_counter() - t0
        reps += 1
    return {"value": prob.ne * reps / t, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} x (energy + exact gradient) over the full {prob.ne}-element mesh, "
                      f"{t:.1f} s, single thread"}


def main():
    a = _args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(json.dumps({"error": "single-GPU build: bench.py measures one MI355X only; "
                          "sharding across GPUs is not implemented",
                          "n_gpus": a.gpus}))
        sys.exit(2)

    import torch
    import p1e_synth as S
    import paper_2109_01158_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = S.config_problem(a.config)
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

    def step():
        vhat.grad = None
        J = P.p1_energy(vhat, mesh, a.prec)
        torch.autograd.backward(J, seed)
        return J

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K steps bracketed by device synchronisations
    t0 = time.perf_counter()
    for _ in range(a.steps):
        J = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / a.steps
    value = info["ne"] / (ms * 1e-3)
    Jv = float(J.item())
    # the same K steps again with every library kernel bracketed by HIP events on its launch
    # stream: per-kernel durations for the roofline (the events themselves cost a few us per
    # kernel, visible as ms_per_step_with_kernel_events)
    P.prof_reset()
    P.prof_enable(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    ms_events = (time.perf_counter() - t2) * 1e3 / a.steps
    P.prof_enable(False)
    kern = P.prof_collect()

    abytes = algorithmic_bytes(info, a.prec, info["geometry_classes"] > 0)
    kstats = {k: {"launches": c, "avg_us": 1e3 * t / c} for k, (c, t) in kern.items()}
    dom = max(kstats, key=lambda k: kstats[k]["avg_us"])
    dom_bytes = abytes.get(dom)
    achieved = dom_bytes / (kstats[dom]["avg_us"] * 1e-6) / 1e9 if dom_bytes else None
    for k, s in kstats.items():
        if k in abytes:
            s["alg_GBs"] = abytes[k] / (s["avg_us"] * 1e-6) / 1e9
    step_bytes = sum(abytes.values())
    prof = profile_record(a.config, a.prec)

    extras = {}
    if not a.no_extras:
        # FP64 J + grad J and the FP64 patch central differences on the same mesh
        g = torch.empty_like(vhat0)
        out3 = torch.empty(3, dtype=torch.float64, device=dev)
        flag = torch.empty(1, dtype=torch.int32, device=dev)
        for name, fn in (("fp64_jgrad", lambda: mesh.grad_exact(vhat0, "fp64", g=g, out3=out3,
                                                                  flag=flag)),
                         ("patch_fd_fp64", lambda: mesh.grad_patch_fd(vhat0, prob.eps)),
                         ("patch_fd4_fp64", lambda: mesh.grad_patch_fd4(vhat0, prob.eps))):
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            n = max(3, a.steps // 2)
            t0 = time.perf_counter()
            for _ in range(n):
                fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / n
            extras[name] = {"elements_per_s": info["ne"] / dt, "ms": dt * 1e3}

    if a.copy_calibration > 0:
        src = torch.empty(a.copy_calibration << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()

    out = {
        "metric": "elements/s for J+\u2207J (3D Neo-Hookean, 6M tets); serve req/s + p50/p99",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64" if a.prec == "mixed" else "fp64",
        "data": "synthetic (seeded mesh and displacement field)",
        "config": {
            "workload": f"{a.config}: 3D Neo-Hookean box [0,1]x[0,0.1]^2, 460x46x46 cubes x 6 Kuhn "
                        f"tets, E=2e8 nu=0.3, x=0 face clamped, u=amp*U[-1,1] (amp={prob.amp:.3g}); "
                        f"J + exact grad J through the autograd hook, {a.prec}",
            "ne": info["ne"], "nn": info["nn"], "n_free_dofs": info["n_free_dofs"],
            "patch_incidences": info["nnz"], "parallelism": "single GPU",
        },
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": (prof or {}).get("traffic_bytes_per_launch", {}).get(dom),
                     "alg_bytes_per_launch": dom_bytes,
                     "alg_bytes_per_element": dom_bytes / info["ne"] if dom_bytes else None,
                     "valu_issue_frac_profiled":
                         (prof or {}).get("valu_issue", {}).get(dom, {}).get("frac")},
        "ms_per_step_with_kernel_events": ms_events,
        "step_alg_bytes_per_element": step_bytes / info["ne"],
        "step_alg_GBs": step_bytes / (ms * 1e-3) / 1e9,
        "kernels": kstats,
        "J": Jv,
        "setup_s": setup_s,
        "extras": extras,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    if not a.no_serve:
        from paper_2109_01158_amd import serving
        del mesh, vhat, vhat0
        torch.cuda.empty_cache()
        out["serve"] = serving.benchmark(
            n_requests=a.serve_requests, iters=a.serve_iters,
            log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
