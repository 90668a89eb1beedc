"""Serving benchmark driver: continuous batching vs one-at-a-time solves.

Workload: n requests with Poisson arrivals; each is a first-order minimization (L-BFGS,
memory 5, a fixed number of iterations) of one mesh whose size is log-uniform in
[1e4, 2e6] elements and whose class is uniform over {p-Laplacian p = 1.5, 3, 5 on the unit
square; 2D Neo-Hookean beam; 3D Neo-Hookean box}. Mesh shapes per size S: square with
n = round(sqrt(S/2)) cells per side; beam with ny = round(sqrt(S/20)), nx = 10 ny; box with
n = round((S/60)^(1/3)), nx = 10 n.

* batched: all requests go through one p1e_server (slots, memory admission, one graph replay
  per step for all active requests), arrivals in real time;
* baseline: the same minimizations one at a time in arrival order (p1e_minimize, no graph, no
  batching), each with its own mesh setup; latencies follow the single-server queue
  start = max(arrival, previous finish). A second comparison gives the baseline the server's
  pool of setup threads, so that only the device-side service (bind + minimize) is serial.
Latency = finish - arrival. Throughput = requests / (last finish - first arrival).
"""

import time

import numpy as np

KINDS = ("plap1.5", "plap3", "plap5", "nh2d", "nh3d")


def request_specs(n, seed=2, lo=1e4, hi=2e6):
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    kinds = rng.integers(0, len(KINDS), n)
    return [(KINDS[k], float(s)) for k, s in zip(kinds, sizes)]


def build_problem(kind, size, seed):
    import p1e_synth as S
    if kind.startswith("plap"):
        n = max(2, int(round(np.sqrt(size / 2))))
        prob = S.plaplace_square(n=n, p=float(kind[4:]), f=-10.0, seed=seed)
        prob.v[:] = 0.0  # start from v = 0
        return prob
    if kind == "nh2d":
        ny = max(1, int(round(np.sqrt(size / 20))))
        return S.neohooke_beam_2d(10 * ny, ny, 2.0, 0.2, seed=seed, amp=0.0)
    n = max(1, int(round((size / 60) ** (1 / 3))))
    return S.neohooke_box_3d(10 * n, n, n, 1.0, 0.1, 0.1, seed=seed, amp=0.0)


def poisson_arrivals(n, rate, seed=1):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n)) - 0.0


def percentiles(x):
    x = np.asarray(x, dtype=np.float64)
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)),
            "mean": float(x.mean()), "max": float(x.max())}


def run_baseline(probs, iters, prec="fp64", history=5):
    """One request at a time: mesh setup (p1e_mesh_create), upload (p1e_mesh_bind) and
    p1e_minimize, no graph, no batching. Returns the per-request times of the three phases
    (s) and the final energies."""
    import torch
    from . import api
    t_setup, t_bind, t_min, J = [], [], [], []
    for prob in probs:
        torch.cuda.synchronize()
        mesh = api.Mesh.from_problem(prob, modes=api.P1E_FP64 if prec == "fp64" else api.P1E_MIXED)
        v = torch.tensor(prob.vhat(), device=mesh.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = api.mesh_minimize(mesh, v, history=history, max_iters=iters, prec=prec)
        torch.cuda.synchronize()
        t_min.append(time.perf_counter() - t0)
        t_setup.append(mesh.create_s)
        t_bind.append(mesh.bind_s)
        J.append(rep["J"])
        mesh.close()
    return np.array(t_setup), np.array(t_bind), np.array(t_min), np.array(J)


def queue_latency(arrivals, service, setup=None, setup_threads=16):
    """Single-server queue in arrival order: start = max(ready, previous finish), where a
    request is ready at its arrival, or (setup given) once its mesh setup has run on the first
    free one of setup_threads host threads from its arrival on. Returns (latency, finish)."""
    import heapq
    free = [0.0] * setup_threads
    done, t = [], -np.inf
    for i, (a, s) in enumerate(zip(arrivals, service)):
        ready = a
        if setup is not None:
            t0 = max(a, heapq.heappop(free))
            ready = t0 + setup[i]
            heapq.heappush(free, ready)
        t = max(t, ready) + s
        done.append(t)
    done = np.array(done)
    return done - arrivals, done


def run_server(probs, arrivals, iters, pool_bytes, max_slots=256, prec="fp64", history=5,
               use_graph=True, setup_threads=16):
    """Replay the arrival trace: every request is submitted with its arrival time (it is
    neither built nor admitted earlier), then the server runs its own loop until idle."""
    from . import api
    srv = api.Server(pool_bytes, max_slots=max_slots, history=history, max_iters=iters,
                     prec=prec, use_graph=use_graph, setup_threads=setup_threads)
    n = len(probs)
    t_base = srv.clock() + 0.2  # time to hand over the trace
    ids, info, steps, peak = {}, {}, 0, 0
    for i in range(n):
        ids[srv.submit_at(probs[i], t_base + arrivals[i], vhat0=probs[i].vhat())] = i
    while len(info) < n:
        active, waiting = srv.run(max_steps=64)
        steps += 64
        peak = max(peak, active)
        for r in srv.poll():
            info[ids[r["id"]]] = r
            srv.release(r["id"])
    srv.close()
    done = np.array([info[i]["t_done"] - t_base for i in range(n)])
    J = np.array([info[i]["J"] for i in range(n)])
    status = np.array([info[i]["status"] for i in range(n)])
    return {"done": done, "J": J, "status": status, "steps": steps, "peak_active": peak,
            "iterations": np.array([info[i]["iterations"] for i in range(n)])}


def benchmark(n_requests=256, iters=200, pool_gb=24.0, seed_sizes=2, seed_arrivals=1,
              log=print, setup_threads=16):
    """Both sides on the same requests; returns a dict for the benchmark's JSON line.

    Two comparisons. (1) As deployed: the one-at-a-time baseline builds each mesh itself
    before its solve (setup on the critical path), arrivals at twice its service rate. (2)
    Setup excluded: the baseline gets the server's setup pool (setup_threads host threads
    building meshes from their arrival on, solves one at a time as meshes are ready), arrivals
    at twice the rate of its bind + minimize service; the server replays the same trace. The
    all-at-once burst measures the server's capacity against both service rates."""
    specs = request_specs(n_requests, seed=seed_sizes)
    t0 = time.perf_counter()
    probs = [build_problem(k, s, seed=i) for i, (k, s) in enumerate(specs)]
    ne = np.array([p.ne for p in probs])
    log(f"serving: built {n_requests} requests ({ne.sum()} elements) in "
        f"{time.perf_counter() - t0:.1f} s")
    t_setup, t_bind, t_min, J_base = run_baseline(probs, iters)
    service = t_setup + t_bind + t_min
    thr_base = n_requests / service.sum()
    pool = int(pool_gb * (1 << 30))
    # (1) as deployed
    rate = 2.0 * thr_base
    arrivals = poisson_arrivals(n_requests, rate, seed=seed_arrivals)
    lat_base, done_base = queue_latency(arrivals, service)
    log(f"serving: baseline {service.sum():.1f} s of service (setup {t_setup.sum():.1f}, bind "
        f"{t_bind.sum():.1f}, minimize {t_min.sum():.1f}), {thr_base:.2f} req/s")
    res = run_server(probs, arrivals, iters, pool, setup_threads=setup_threads)
    lat = res["done"] - arrivals
    makespan = res["done"].max() - arrivals[0]
    makespan_base = done_base.max() - arrivals[0]
    # (2) setup excluded: both sides with the same setup pool
    service_dev = t_bind + t_min
    thr_dev = n_requests / service_dev.sum()
    rate2 = 2.0 * thr_dev
    arrivals2 = poisson_arrivals(n_requests, rate2, seed=seed_arrivals)
    lat_pool, done_pool = queue_latency(arrivals2, service_dev, setup=t_setup,
                                        setup_threads=setup_threads)
    res2 = run_server(probs, arrivals2, iters, pool, setup_threads=setup_threads)
    lat2 = res2["done"] - arrivals2
    makespan2 = res2["done"].max() - arrivals2[0]
    makespan_pool = done_pool.max() - arrivals2[0]
    burst = run_server(probs, np.zeros(n_requests), iters, pool, setup_threads=setup_threads)
    burst_rate = n_requests / burst["done"].max()
    rel = np.abs(res["J"] - J_base) / np.maximum(np.abs(J_base), 1e-300)
    log(f"serving: batched makespan {makespan:.1f} s, peak {res['peak_active']} active; setup "
        f"excluded: batched {n_requests / makespan2:.1f} req/s vs {n_requests / makespan_pool:.1f}")
    return {
        "requests": n_requests, "iterations_per_request": iters,
        "arrival_rate_req_s": rate, "elements_total": int(ne.sum()),
        "batched": {"req_s": n_requests / makespan, "latency_s": percentiles(lat),
                    "makespan_s": makespan, "engine_steps": res["steps"],
                    "peak_active": res["peak_active"]},
        "one_at_a_time_fp64": {"req_s": n_requests / makespan_base,
                               "service_req_s": thr_base,
                               "latency_s": percentiles(lat_base), "makespan_s": makespan_base},
        "speedup_req_s": (n_requests / makespan) / (n_requests / makespan_base),
        "baseline_setup_s": float(t_setup.sum()),
        "baseline_bind_s": float(t_bind.sum()),
        "baseline_minimize_s": float(t_min.sum()),
        "setup_excluded": {
            "arrival_rate_req_s": rate2, "setup_threads": setup_threads,
            "batched": {"req_s": n_requests / makespan2, "latency_s": percentiles(lat2),
                        "makespan_s": makespan2, "peak_active": res2["peak_active"]},
            "one_at_a_time_fp64_setup_pool": {"req_s": n_requests / makespan_pool,
                                              "service_req_s": thr_dev,
                                              "latency_s": percentiles(lat_pool),
                                              "makespan_s": makespan_pool},
            "final_J_bitwise_equal": bool(np.array_equal(res2["J"], J_base)),
        },
        "speedup_req_s_setup_excluded": (n_requests / makespan2) / (n_requests / makespan_pool),
        "burst_all_at_t0": {"req_s": burst_rate,
                            "latency_s": percentiles(burst["done"]),
                            "peak_active": burst["peak_active"],
                            "vs_one_at_a_time_service": burst_rate / thr_base,
                            "vs_one_at_a_time_bind_minimize_service": burst_rate / thr_dev,
                            "final_J_bitwise_equal": bool(np.array_equal(burst["J"], J_base))},
        "final_J_max_rel_diff_vs_one_at_a_time": float(rel.max()),
        "final_J_bitwise_equal": bool(np.array_equal(res["J"], J_base)),
        "status_counts": {int(s): int((res["status"] == s).sum()) for s in np.unique(res["status"])},
    }
