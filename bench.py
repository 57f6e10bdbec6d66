#!/usr/bin/env python3
"""Benchmark of the bipartite H*psi on one MI355X.

A timed step is one H*psi application (left operator, right operator,
diagonal and cross-cut terms: the whole per-application hot path) on the
16-site Hubbard chain at half filling, U=8, up/down cut: Psi is
12870 x 12870 FP64 (1.33 GB), resident in HBM before timing starts.

Prints one JSON line: applies/s, the roofline of the dominant kernel
(algorithmic bytes / average kernel time from HIP events on the launch
stream), the oracle timed on a bounded sample on the host cores, a short
Lanczos-step timing, the apply time of the other configurations (Heisenberg
16, Hubbard 12, J1-J2 6x5), the workload's ground-state solve (full
reorthogonalisation over at most 150 stored vectors, tol 1e-10) against the
oracle's stored energy, and
the serving comparison (sequential vs continuous batching).
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def _code_only(text):
    """The source without its comments and blank space, so that an edit of
    a comment leaves the hash (and the counters it guards) valid."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    """Hash of the sources that decide what a profiled kernel does: the
    kernels, their constants and argument structs, and the work lists
    (their code, not their comments)."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels.h", "ecut_internal.h", "sectors.cpp"):
        with open(os.path.join(ROOT, "paper_2605_07621_amd", "csrc", name), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


# Launch tuning of each workload's timed applies: the autotuner's pick on
# MI355X (its candidates within run noise of each other), pinned so that the
# rocprofv3 counters committed under profiles/ describe the benchmarked run.
PINNED_TUNING = {"hubbard16": "8,8,8,7,0", "j1j2_6x5": "4,8,0,2,0"}


def traffic_from_profile(kernel, workload, per_launch_alg):
    """HBM traffic per launch from the committed rocprofv3 counter summary
    and the launch tuning the counters were taken with (grid,n_xcd,
    row_order,variant), or (None, None) if there is none or the kernel
    source changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_source_hash():
        return None, None
    words = d.get("commands", {}).get("fetch", "").split()
    tuning = words[words.index("--tuning") + 1] if "--tuning" in words[:-1] else None
    return d.get("bytes_per_launch"), tuning


def tuning_str(t):
    return ",".join(str(t[k]) for k in ("grid", "n_xcd", "row_order", "variant", "tile"))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, seconds):
    """The oracle on the host cores, timed on a bounded contiguous sample of
    the workload's rows (the whole-sector CSR of the 16-site chain is 34 GB
    and takes minutes to build): the CSR of the sample rows is built once,
    then its product with the seeded input is timed on one thread and on all
    threads; the row-by-row generator (no stored matrix) is timed on the
    same sample.  Rates are scaled to whole applications (sample rows / dim
    of an application per second of the sample)."""
    import numpy as np
    import oracle as O
    from paper_2605_07621_amd import inputs as I
    words = O.enumerate_basis(p.model.kind, p.model.n_sites, p.n_up, p.n_dn)
    n = len(words)
    psi = I.psi(p.meta["seed"], n)
    sec = O.Sector.__new__(O.Sector)
    sec.model, sec.om, sec.words, sec.n = p.model, O.OracleModel(p.model), words, n
    all_threads = O.num_threads()
    start = int(np.random.default_rng(11).integers(0, n // 2))
    # sample size: about `seconds` of row-by-row work on all threads
    probe = np.arange(start, start + 20000, dtype=np.int64)
    t0 = time.perf_counter()
    sec.apply_rows(psi, probe)
    dt = time.perf_counter() - t0
    m = int(min(n - start, max(20000, 20000 * seconds / 4 / max(dt, 1e-6))))
    rows = np.arange(start, start + m, dtype=np.int64)
    t0 = time.perf_counter()
    sec.apply_rows(psi, rows)
    t_rows = time.perf_counter() - t0
    t0 = time.perf_counter()
    rp, col, val = sec.csr_rows(start, start + m)
    t_build = time.perf_counter() - t0
    legs = {}
    for threads in (1, all_threads):
        O.set_threads(threads)
        O.spmv_csr(rp, col, val, psi)   # first touch
        reps, t_acc = 0, 0.0
        while t_acc < (2.0 if threads == 1 else 1.0) or reps < 3:
            t0 = time.perf_counter()
            O.spmv_csr(rp, col, val, psi)
            t_acc += time.perf_counter() - t0
            reps += 1
        legs[threads] = t_acc / reps
    O.set_threads(all_threads)
    frac = m / n
    return dict(value=frac / legs[all_threads], unit="H*psi/s", cores=all_threads, kind="oracle",
                sample=f"rows {start}..{start + m - 1} ({m} of {n}, contiguous): CSR of the sample rows "
                       f"(oracle row generator), product timed; rate scaled to whole applications",
                csr_spmv={"threads_all": all_threads, "threads_all_s_per_apply": legs[all_threads] / frac,
                          "threads_1_s_per_apply": legs[1] / frac, "sample_nnz": int(len(col)),
                          "sample_build_s": round(t_build, 2)},
                row_generator={"threads": all_threads, "s_per_apply": t_rows / frac},
                nproc=os.cpu_count(), cpu_model=_cpu_model(),
                oracle_lanczos=_golden_lanczos_time(p))


def _golden_lanczos_time(p):
    """Seconds per step of the oracle's own Lanczos run that wrote the
    workload's stored energy (tests/golden; that run's host and threads)."""
    path = os.path.join(ROOT, "tests", "golden", f"{p.meta.get('name', '')}_energy.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    return {"s_per_step": round(d["lanczos_s"] / d["steps"], 3), "steps": d["steps"], "threads": d["oracle_threads"],
            "method": d["method"], "host": "the host that wrote tests/golden (not the benchmark host)"}


# the two-lane server's threshold: the mix's 14-site Hubbard chains (11.8M
# amplitudes) get their own worker and stream, everything else batches on the other
LARGE_DIM = 1 << 22


def _run_server(reqs, arrivals, budget, max_active, sequential, tol=1e-10, max_steps=600, large_dim=0):
    from paper_2605_07621_amd import ecut
    # each problem shape is autotuned once per process (first request), in every mode
    srv = ecut.Server(int(budget), max_active=max_active, max_steps=max_steps, tol=tol, sequential=sequential,
                      autotune=True, large_dim=large_dim)
    t0 = srv.now()
    ids = [srv.submit(p, seed=p.meta["seed"], not_before=t0 + float(a)) for p, a in zip(reqs, arrivals)]
    srv.drain()
    res = {r["req_id"]: r for r in srv.poll(len(reqs) + 8)}
    srv.close()
    out = [res[i] for i in ids]
    bad = [r for r in out if r["status"] != 0]
    if bad:
        raise RuntimeError(f"{len(bad)} serving requests failed, first status {bad[0]['status']}")
    return out


def _lat_stats(out, start):
    import numpy as np
    lat = np.array([r["t_done"] - r["t_submit"] for r in out])
    span = max(r["t_done"] for r in out) - start
    return dict(solves_per_s=round(len(out) / span, 3), makespan_s=round(span, 3),
                p50_s=round(float(np.percentile(lat, 50)), 5), p99_s=round(float(np.percentile(lat, 99)), 5))


def _warm_tunings(reqs, budget):
    """Tune every problem shape of the mix once, before the timed runs, so
    that neither the sequential nor the batched run pays for it (the server
    keeps the tunings for the life of the process)."""
    from paper_2605_07621_amd import ecut
    seen, first = set(), []
    for p in reqs:
        key = (p.model.kind, p.model.n_sites, p.n_up, p.n_dn)
        if key not in seen:
            seen.add(key)
            first.append(p)
    # one server per mode: the sequential baseline keeps each shape's tuning
    # for a problem alone, a batching server the tuning whose launches merge
    for max_active in (1, 32):
        srv = ecut.Server(int(budget), max_active=max_active, max_steps=2, tol=1e-10, autotune=True)
        for p in first:
            srv.submit(p, seed=p.meta["seed"])
        srv.drain()
        srv.poll(len(first) + 8)   # two-step solves: statuses are not looked at
        srv.close()
    return len(first)


def _serving_oracle(n_requests):
    """The oracle's ground energy of every request of the serving mix
    (tests/golden/serving_2026_energies.json, written by
    tests/golden/make_golden.py), or None for another mix."""
    path = os.path.join(ROOT, "tests", "golden", "serving_2026_energies.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d["requests"] != n_requests:
        return None
    return [e["energy"] for e in d["energies"]]


def _max_err(out, ref):
    return max(abs(r["energy"] - e) for r, e in zip(out, ref))


def serving_bench(n_requests, budget_gb):
    """Mixed ground-state requests (seeded XXZ and Hubbard chains, Sz=0 / half
    filling, tol 1e-10): sequential one-at-a-time solves vs continuous batching
    (every admitted request active, and at most 32 active), closed loop (all at
    t=0) and Poisson arrivals at 0.5x and 2x the sequential rate."""
    import numpy as np
    from paper_2605_07621_amd import inputs as I
    reqs = I.serving_requests(n_requests, seed=2026)
    budget = budget_gb * 2**30
    zeros = np.zeros(len(reqs))
    n_shapes = _warm_tunings(reqs, budget)
    progress(f"serving: {n_shapes} problem shapes tuned")
    seq = _run_server(reqs, zeros, budget, 1, True)
    progress("serving: sequential closed loop done")
    s_seq = _lat_stats(seq, min(r["t_submit"] for r in seq))
    bat = _run_server(reqs, zeros, budget, 0, False)
    s_bat = _lat_stats(bat, min(r["t_submit"] for r in bat))
    cap = _run_server(reqs, zeros, budget, 32, False)
    s_cap = _lat_stats(cap, min(r["t_submit"] for r in cap))
    lan = _run_server(reqs, zeros, budget, 0, False, large_dim=LARGE_DIM)
    s_lan = _lat_stats(lan, min(r["t_submit"] for r in lan))
    progress("serving: batched closed loops done")
    de = max(max(abs(a["energy"] - b["energy"]), abs(a["energy"] - c["energy"]), abs(a["energy"] - d["energy"]))
             for a, b, c, d in zip(seq, bat, cap, lan))
    ref = _serving_oracle(n_requests)
    out = {"requests": len(reqs), "tol": 1e-10, "two_lane_large_dim": LARGE_DIM,
           "closed_loop": {"sequential": s_seq, "batched": s_bat, "batched_max32": s_cap,
                           "batched_two_lanes": s_lan},
           "max_energy_diff_batched_vs_sequential": de,
           "max_abs_energy_error_vs_oracle": None if ref is None else {
               "sequential": _max_err(seq, ref), "batched": _max_err(bat, ref), "batched_max32": _max_err(cap, ref),
               "batched_two_lanes": _max_err(lan, ref)},
           "speedup_solves_per_s": round(s_bat["solves_per_s"] / s_seq["solves_per_s"], 3),
           "speedup_solves_per_s_max32": round(s_cap["solves_per_s"] / s_seq["solves_per_s"], 3),
           "speedup_solves_per_s_two_lanes": round(s_lan["solves_per_s"] / s_seq["solves_per_s"], 3)}
    mu = s_seq["solves_per_s"]
    for rho in (0.5, 2.0):
        arr = I.poisson_arrivals(len(reqs), rho * mu)
        r_seq = _run_server(reqs, arr, budget, 1, True)
        r_bat = _run_server(reqs, arr, budget, 0, False)
        r_cap = _run_server(reqs, arr, budget, 32, False)
        r_lan = _run_server(reqs, arr, budget, 0, False, large_dim=LARGE_DIM)
        progress(f"serving: poisson rho={rho} done")
        out[f"poisson_rho{rho}"] = {"rate_per_s": round(rho * mu, 3),
                                    "max_abs_energy_error_vs_oracle": None if ref is None else max(
                                        _max_err(r_seq, ref), _max_err(r_bat, ref), _max_err(r_cap, ref),
                                        _max_err(r_lan, ref)),
                                    "sequential": _lat_stats(r_seq, min(r["t_submit"] for r in r_seq)),
                                    "batched": _lat_stats(r_bat, min(r["t_submit"] for r in r_bat)),
                                    "batched_max32": _lat_stats(r_cap, min(r["t_submit"] for r in r_cap)),
                                    "batched_two_lanes": _lat_stats(r_lan, min(r["t_submit"] for r in r_lan))}
    return out


def kernel_name(S):
    """Name of the kernel that carries the apply under the handle's tuning."""
    info, t = S.info, S.get_tuning()
    if info.kernel == 1:
        v = t["variant"]
        if v == 0:
            return "k_hub3" if info.kernel_flags & 2 else "k_hub2"
        return {1: "k_hub", 2: "k_hub2", 3: "k_upslab+k_hub3", 4: "k_hubrow", 5: "k_hubseg", 6: "k_hubU+k_hubD",
                7: "k_hubU+k_hub3"}[v]
    if info.kernel_flags & 64 and t["variant"] == 2:
        return "k_spinL+k_spinR"
    return "k_spin" if (info.kernel_flags & 4 and t["variant"] == 0) else "k_rows"


def time_applies(S, x, y, stream, reps, warmup=2):
    import torch
    for _ in range(warmup):
        S.apply(x, y, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        S.apply(x, y, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def other_workloads(names, stream):
    """H*psi time of the other measured configurations (autotuned), each
    with its algorithmic bytes per application (read psi, write y, metadata)."""
    import torch
    from paper_2605_07621_amd import ecut, inputs as I
    out = {}
    for name in names:
        p = I.WORKLOADS[name]()
        S = ecut.Sectors.from_problem(p)
        x = S.import_(torch.from_numpy(I.psi(p.meta["seed"], S.dim)).to("cuda:0"))
        y = torch.empty_like(x)
        S.autotune(x, y, stream=stream)
        progress(f"{name}: tuned")
        reps = 10 if S.dim > 10**7 else 200
        ms = time_applies(S, x, y, stream, reps)
        alg = 2 * S.dim * 8 + int(S.info.device_bytes)
        out[name] = {"dim": S.dim, "blocks": int(S.info.n_blocks), "kernel": kernel_name(S), "ms": round(ms, 4),
                     "applies_per_s": round(1e3 / ms, 2), "algorithmic_GBps": round(alg / (ms * 1e-3) / 1e9, 1)}
        steps = p.meta.get("lanczos_steps")
        if name in ("j1j2_6x5", "hubbard14_spatial"):
            # Lanczos energy to 1e-10 (three-term recurrence) against the
            # oracle's stored energy
            v0 = S.import_(torch.from_numpy(I.psi(p.meta["seed"] + 1, S.dim)).to("cuda:0"))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, st, _ = S.lanczos(v0, 600, tol=1e-10, allow_notconv=True)
            out[name]["lanczos"] = {"steps": st["steps"], "converged": bool(st["converged"]),
                                    "seconds": round(time.perf_counter() - t0, 3), "energy": e, "tol": 1e-10}
            gold = os.path.join(ROOT, "tests", "golden", f"{name}_energy.json")
            if os.path.exists(gold):
                with open(gold) as f:
                    ref = json.load(f)["energy"]
                out[name]["lanczos"]["oracle_energy"] = ref
                out[name]["lanczos"]["abs_diff_vs_oracle"] = abs(e - ref)
            del v0
        if steps:
            # the configuration's fixed-step Lanczos energy (start vector: seed + 1)
            v0 = S.import_(torch.from_numpy(I.psi(p.meta["seed"] + 1, S.dim)).to("cuda:0"))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e, st, _ = S.lanczos(v0, steps, fixed_steps=True)
            dt = time.perf_counter() - t0
            lz = {"steps": st["steps"], "seconds": round(dt, 4), "energy": e}
            gold = os.path.join(ROOT, "tests", "golden", f"{name}_energy.json")
            if os.path.exists(gold):
                with open(gold) as f:
                    ref = json.load(f)["energy"]
                lz["oracle_energy"] = ref
                lz["abs_diff_vs_oracle"] = abs(e - ref)
            out[name]["lanczos"] = lz
            del v0
        del S, x, y
    torch.cuda.empty_cache()
    return out


def analyses(stream):
    """The analyses built on the layout, timed on device-resident states
    (their parity with the oracle is in the GPU tests):
     - entanglement spectrum of the spatial-cut Hubbard benchmark's ground
       state (64 blocks, Gram matrices with rocBLAS dsyrk, eigenvalues with
       rocSOLVER dsyevd);
     - Krylov dynamical correlations on the 14-site Hubbard chain (up/down
       cut): c+ of one mode from the ground state's sector to the next, and
       the Lanczos coefficients of G+(omega) from that vector."""
    import numpy as np
    import torch
    from paper_2605_07621_amd import ecut, inputs as I
    out = {}
    p = I.hubbard14_spatial()
    S = ecut.Sectors.from_problem(p)
    x = torch.from_numpy(I.psi(p.meta["seed"], S.dim)).to("cuda:0")
    S.autotune(S.import_(x), torch.empty_like(x), stream=stream)
    v0 = S.import_(torch.from_numpy(I.psi(p.meta["seed"] + 1, S.dim)).to("cuda:0"))
    e0, st, gs = S.lanczos(v0, 150, tol=1e-12, reorth=True, max_restarts=8, want_gs=True)
    blocks = S.blocks()
    m = np.minimum(blocks[:, 2], blocks[:, 3]).astype(np.float64)
    k = np.maximum(blocks[:, 2], blocks[:, 3]).astype(np.float64)
    ent = S.entanglement(gs, n_parts=8, cutoff=1e-12)
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        ent = S.entanglement(gs, n_parts=8, cutoff=1e-12)
        times.append(time.perf_counter() - t0)
    out["entanglement"] = {
        "workload": "hubbard14_spatial ground state", "energy": e0, "lanczos_steps": st["steps"],
        "blocks": int(S.info.n_blocks), "schmidt_values": int(sum(len(l) for l in ent["lam"])),
        "ms": round(min(times) * 1e3, 3), "gram_gflop": round(float(np.sum(m * (m + 1) * k)) / 1e9, 3),
        "entropy": ent["entropy"], "n_eff": ent["n_eff"], "w_p_8": [round(float(w), 6) for w in ent["w_p"]]}
    progress("entanglement spectrum timed")
    del S, x, v0, gs
    # c+ and the Lanczos coefficients of G+ on the 14-site Hubbard chain
    m0 = I.hubbard_chain(14, 1.0, 4.0)
    S0 = ecut.Sectors(m0, I.Cut("updn"), 7, 7)
    S1 = ecut.Sectors(m0, I.Cut("updn"), 8, 7)
    x = torch.from_numpy(I.psi(1006, S0.dim)).to("cuda:0")
    for T in (S0, S1):
        xt = torch.from_numpy(I.psi(1006, T.dim)).to("cuda:0")
        T.autotune(T.import_(xt), torch.empty_like(xt), stream=stream)
    e0, st, gs = S0.lanczos(S0.import_(x), 150, tol=1e-12, reorth=True, max_restarts=8, want_gs=True)
    y = ecut.apply_cdag(S0, S1, 0, 0, True, gs)
    reps = 20
    torch.cuda.synchronize()
    e_0 = torch.cuda.Event(enable_timing=True)
    e_1 = torch.cuda.Event(enable_timing=True)
    e_0.record(stream)
    for _ in range(reps):
        ecut.apply_cdag(S0, S1, 0, 0, True, gs, out=y, stream=stream)
    e_1.record(stream)
    torch.cuda.synchronize()
    ms = e_0.elapsed_time(e_1) / reps
    n_steps = 200
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, b, w = ecut.lanczos_tridiag(S1, y, n_steps)
    dt = time.perf_counter() - t0
    omega = np.linspace(-10.0, 10.0, 201)
    g = ecut.continued_fraction(a, b, w, e0, True, omega, 0.1)
    out["green_function"] = {
        "workload": "hubbard_chain_14 (t=1, U=4), c+ of site 0, spin up, from (7,7) to (8,7)",
        "ground_energy": e0, "cdag_ms": round(ms, 4), "cdag_GBps": round((S0.dim + S1.dim) * 8 / (ms * 1e-3) / 1e9, 1),
        "cdag_roofline_frac": round((S0.dim + S1.dim) * 8 / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "weight": w, "lanczos_steps": len(a), "ms_per_lanczos_step": round(dt * 1e3 / max(len(a), 1), 4),
        "spectral_sum": float(-np.trapezoid(g.imag, omega) / np.pi)}
    progress("dynamical correlations timed")
    del S0, S1, x, y, gs
    torch.cuda.empty_cache()
    return out


def ground_state_solve(S, p, n_keep, tol):
    """Lanczos to the ground energy with full reorthogonalisation over at
    most n_keep stored vectors (explicit restarts), compared with the
    oracle's energy stored under tests/golden."""
    import torch
    from paper_2605_07621_amd import inputs as I
    v0 = S.import_(torch.from_numpy(I.psi(p.meta["seed"] + 1, S.dim)).to("cuda:0"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, st, _ = S.lanczos(v0, n_keep, tol=tol, reorth=True, max_restarts=20)
    dt = time.perf_counter() - t0
    out = {"energy": e, "steps": st["steps"], "restarts": st["restarts"], "converged": bool(st["converged"]),
           "seconds": round(dt, 3), "n_keep": n_keep, "tol": tol,
           "reorth": "classical Gram-Schmidt, second pass when the first removes over half the squared norm"}
    gold = os.path.join(ROOT, "tests", "golden", f"{p.meta.get('name', '')}_energy.json")
    if os.path.exists(gold):
        with open(gold) as f:
            ref = json.load(f)["energy"]
        out["oracle_energy"] = ref
        out["abs_diff_vs_oracle"] = abs(e - ref)
    del v0
    torch.cuda.empty_cache()
    return out


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _csv_rows(d, suffix=".csv"):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True):
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def summarize_profiles(workload, kernel, copy_bytes, trace_dir, fetch_dir, write_dir, commands):
    """Write the committed profile summaries of one kernel and workload:
    profiles/<kernel>_<workload>_trace.txt, the per-kernel statistics of a
    rocprofv3 --kernel-trace --stats run, and
    profiles/<kernel>_<workload>_traffic.json, the HBM bytes per launch from
    a FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch), each scaled by
    what the same counter reads for a plain copy of copy_bytes bytes in the
    same run (the profiled command makes those copies with --copy-probe)."""
    import statistics
    stats = [r for r in _csv_rows(trace_dir, "kernel_stats.csv") if "AverageNs" in r and "Calls" in r]
    lines = [f"# rocprofv3 kernel statistics: {workload}", "", "command (from the repository root):",
             "  " + commands.get("setup", ""), "  " + commands["trace"], "",
             f"{'kernel':72s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s}"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"{r['Name'][:72]:72s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.3f}")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"{kernel}_{workload}_trace.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    out = {"kernel": kernel, "workload": workload, "kernel_hash": kernel_source_hash(), "copy_bytes": copy_bytes,
           "commands": commands}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        # an apply may be several launches (e.g. k_spin<true> + k_spin<false>):
        # sum every launch of the kernel family, divide by the number of applies
        per_name, cs = {}, []
        for r in _csv_rows(d):
            if r.get("Counter_Name") != name:
                continue
            kn = r["Kernel_Name"]
            v = float(r["Counter_Value"]) * 1024.0
            if any(f"ecut::{k}" in kn for k in kernel.split("+")):
                per_name.setdefault(kn, []).append(v)
            elif "copyBuffer" in kn:
                cs.append(v)
        n_apply = max((len(v) for v in per_name.values()), default=0)
        big = [c for c in cs if c > 0.25 * copy_bytes / 2]
        scale = copy_bytes / statistics.mean(big) if big else None
        out[name] = {"kernel_raw_bytes_per_launch": sum(sum(v) for v in per_name.values()) / n_apply if n_apply else None,
                     "launches": {k: len(v) for k, v in per_name.items()},
                     "copy_raw_bytes": statistics.mean(big) if big else None, "scale": scale}
    f_, w_ = out["FETCH_SIZE"], out["WRITE_SIZE"]
    if f_["kernel_raw_bytes_per_launch"] and f_["scale"] and w_["kernel_raw_bytes_per_launch"] and w_["scale"]:
        out["bytes_per_launch"] = (f_["kernel_raw_bytes_per_launch"] * f_["scale"]
                                   + w_["kernel_raw_bytes_per_launch"] * w_["scale"])
    with open(os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json"), "w") as f:
        json.dump(out, f, indent=1)
    return out


SERVING_TRACES = {
    "max32": ("batched_max32_closed_loop", "serving_c5_batched32_trace.txt",
              "batched closed loop on one worker (at most 32 active)"),
    "two_lanes": ("two_lanes_closed_loop", "serving_c5_two_lanes_trace.txt",
                  "closed loop on the two-lane server (14-site Hubbard requests one at a time on their own stream)"),
}


def serving_trace(n_requests, budget_gb, mode="max32"):
    """One closed-loop serving run alone (the batched server with at most 32
    active, or the two-lane server), after the tuning warm-up, for a kernel
    trace: prints its statistics and its timed window on the monotonic clock
    (the clock of rocprofv3's stamps)."""
    import numpy as np
    from paper_2605_07621_amd import inputs as I
    reqs = I.serving_requests(n_requests, seed=2026)
    budget = budget_gb * 2**30
    _warm_tunings(reqs, budget)
    t0 = time.monotonic_ns()
    if mode == "two_lanes":
        out = _run_server(reqs, np.zeros(len(reqs)), budget, 0, False, large_dim=LARGE_DIM)
    else:
        out = _run_server(reqs, np.zeros(len(reqs)), budget, 32, False)
    t1 = time.monotonic_ns()
    return dict(run=SERVING_TRACES[mode][0], requests=n_requests, window_ns=[t0, t1],
                **_lat_stats(out, min(r["t_submit"] for r in out)))


def summarize_serving(trace_dir, run, window, command):
    """profiles/serving_c5_<mode>_trace.txt: the kernels of the timed serving
    window from a rocprofv3 kernel trace, and how busy the GPU was."""
    import csv
    mode = next(k for k, v in SERVING_TRACES.items() if v[0] == run)
    t0, t1 = window
    rows = []
    for fn in os.listdir(trace_dir):
        if fn.endswith("kernel_trace.csv"):
            with open(os.path.join(trace_dir, fn)) as f:
                rows += [r for r in csv.DictReader(f) if t0 <= int(r["Start_Timestamp"]) <= t1]
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows)
    busy, cs, ce = 0, None, None
    for s, e in iv:
        if ce is None or s > ce:
            busy += 0 if ce is None else ce - cs
            cs, ce = s, e
        else:
            ce = max(ce, e)
    if ce is not None:
        busy += ce - cs
    span = t1 - t0
    per = {}
    for r in rows:
        k = r["Kernel_Name"].split("(")[0].replace("void ", "")
        n, tot = per.get(k, (0, 0))
        per[k] = (n + 1, tot + int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    ktime = sum(tot for _, tot in per.values())
    lines = [f"# rocprofv3 kernel trace: 256 mixed serving requests, {SERVING_TRACES[mode][2]}", "",
             "command (from the repository root):", "  cd /tmp && export TMPDIR=/tmp && cd -", "  " + command, "",
             f"timed window {span / 1e9:.3f} s, {len(rows)} kernels, GPU busy {busy / 1e9:.3f} s "
             f"({100.0 * busy / span:.1f}% of the window); kernel time summed over all queues {ktime / 1e9:.3f} s",
             f"({ktime / max(busy, 1):.2f}x the busy time: kernels of different queues overlap, so the shares, of",
             "the busy time, can sum above 100%; uploads of sector tables run beside the steps)", "",
             f"{'kernel':60s} {'calls':>8s} {'total_ms':>10s} {'share':>7s}"]
    for k, (n, tot) in sorted(per.items(), key=lambda kv: -kv[1][1])[:16]:
        lines.append(f"{k[:60]:60s} {n:8d} {tot / 1e6:10.1f} {100.0 * tot / max(busy, 1):6.1f}%")
    path = os.path.join(ROOT, "profiles", SERVING_TRACES[mode][1])
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


def summarize_solve(trace_dir, bench_json, command):
    """profiles/lanczos_reorth_hubbard16_trace.txt: the kernels of the
    ground-state solve (full reorthogonalisation) from a rocprofv3 kernel trace
    of a bench run, and the streaming rate of the projection kernels.  Their
    first pass at step j reads j + 1 basis vectors, so the median growth of
    the launch time from one step to the next is the time of one vector."""
    import csv
    import numpy as np
    res = json.loads(open(bench_json).read().strip().splitlines()[-1])
    gs, dim = res["ground_state"], res["config"]["dim"]
    rows = []
    for fn in os.listdir(trace_dir):
        if fn.endswith("kernel_trace.csv"):
            with open(os.path.join(trace_dir, fn)) as f:
                rows += list(csv.DictReader(f))
    for r in rows:
        r["k"] = r["Kernel_Name"].split("(")[0].replace("void ", "")
        r["t0"], r["t1"] = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
    proj = [r for r in rows if r["k"].startswith(("ecut::k_multidot<", "ecut::k_multiaxpy<"))]
    t0, t1 = min(r["t0"] for r in proj), max(r["t1"] for r in proj)
    win = [r for r in rows if t0 <= r["t0"] <= t1]
    per = {}
    for r in win:
        n, tot = per.get(r["k"], (0, 0))
        per[r["k"]] = (n + 1, tot + r["t1"] - r["t0"])
    busy = sum(v[1] for v in per.values())
    vec_bytes = 8.0 * dim
    lines = ["# rocprofv3 kernel trace: ground-state solve, 16-site Hubbard chain (dim 165,636,900), "
             f"full reorthogonalisation over at most {gs['n_keep']} vectors", "",
             "command (from the repository root):", "  cd /tmp && export TMPDIR=/tmp && cd -", "  " + command, "",
             f"solve: {gs['steps']} steps, {gs['restarts']} restart(s), {gs['seconds']} s (bench clock), "
             f"|E - E_oracle| = {gs.get('abs_diff_vs_oracle')}",
             f"kernels between the first and last projection launch: {len(win)}, {busy / 1e9:.3f} s of kernel time", "",
             f"{'kernel':40s} {'calls':>7s} {'total_ms':>10s} {'share':>7s}  per added basis vector"]
    for k, (n, tot) in sorted(per.items(), key=lambda kv: -kv[1][1])[:10]:
        extra = ""
        if k in ("ecut::k_multidot<true>", "ecut::k_multiaxpy<true>"):
            d = np.array([r["t1"] - r["t0"] for r in sorted((r for r in win if r["k"] == k), key=lambda r: r["t0"])],
                         dtype=float)
            d = d[d > 20e3]   # first passes (a skipped second pass returns at once)
            inc = np.diff(d)
            inc = inc[inc > 0]   # a restart shortens the basis
            if len(inc):
                m = float(np.median(inc))
                extra = f"  {m / 1e3:.1f} us = {vec_bytes / m / 1e3:.2f} TB/s"
        lines.append(f"{k[:40]:40s} {n:7d} {tot / 1e6:10.1f} {100.0 * tot / max(busy, 1):6.1f}%{extra}")
    path = os.path.join(ROOT, "profiles", "lanczos_reorth_hubbard16_trace.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="hubbard16")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lanczos-steps", type=int, default=10)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--serving", type=int, default=256, help="requests in the serving run (0: skip)")
    ap.add_argument("--no-solve", action="store_true", help="skip the ground-state solve of the workload")
    ap.add_argument("--solve-keep", type=int, default=150)
    ap.add_argument("--no-others", action="store_true", help="skip the other configurations")
    ap.add_argument("--no-analyses", action="store_true",
                    help="skip the timed entanglement spectrum and dynamical correlations")
    ap.add_argument("--tuning", default=None,
                    help="grid,n_xcd,row_order,variant,tile (default: the pinned tuning of the workload, if any)")
    ap.add_argument("--autotune", action="store_true", help="autotune instead of the pinned tuning")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, make 3 plain device copies of psi (scale reference for counter runs)")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write the profiles/ summaries from rocprofv3 output and exit (no GPU use)")
    ap.add_argument("--kernel", default="k_hub3", help="kernel named in --summarize")
    ap.add_argument("--commands", default=None, help="JSON of the profiling commands, for --summarize")
    ap.add_argument("--serving-budget-gb", type=float, default=24.0)
    ap.add_argument("--serving-trace", nargs="?", const="max32", default=None, choices=sorted(SERVING_TRACES),
                    help="run only one serving closed loop (for a kernel trace) and print its window")
    ap.add_argument("--summarize-solve", nargs=2, metavar=("TRACE_DIR", "BENCH_JSON"),
                    help="write profiles/lanczos_reorth_hubbard16_trace.txt from a kernel trace of a bench run")
    ap.add_argument("--summarize-serving", nargs=2, metavar=("TRACE_DIR", "WINDOW_JSON"),
                    help="write profiles/serving_c5_<mode>_trace.txt from a --serving-trace kernel trace")
    args = ap.parse_args()
    if args.summarize_solve:
        print(summarize_solve(args.summarize_solve[0], args.summarize_solve[1], args.commands or ""))
        return
    if args.summarize_serving:
        w = json.loads(open(args.summarize_serving[1]).read().strip().splitlines()[-1])
        print(summarize_serving(args.summarize_serving[0], w["run"], w["window_ns"], args.commands or ""))
        return
    if args.serving_trace:
        print(json.dumps(serving_trace(args.serving, args.serving_budget_gb, args.serving_trace)), flush=True)
        return
    if args.summarize:
        from paper_2605_07621_amd import inputs as I
        p = I.WORKLOADS[args.workload]()
        import math
        dim = math.comb(p.model.n_sites, p.n_up) * (math.comb(p.model.n_sites, p.n_dn) if p.n_dn or
                                                         p.model.kind == "hubbard" else 1)
        cmds = json.loads(args.commands) if args.commands else {}
        out = summarize_profiles(args.workload, args.kernel, 8 * dim, *args.summarize, cmds)
        print(json.dumps(out))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_07621_amd import ecut, inputs as I

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = I.WORKLOADS[args.workload]()
    S = ecut.Sectors.from_problem(p)
    n = S.dim
    x = S.import_(torch.from_numpy(I.psi(p.meta.get("seed", 1), n)).to(dev))
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    if args.tuning is None and not args.autotune:
        args.tuning = PINNED_TUNING.get(args.workload)
    if args.tuning:
        S.set_tuning(*[int(v) for v in args.tuning.split(",")])
        tuning = S.get_tuning()
    else:
        tuning = S.autotune(x, y, stream=stream) if not args.no_autotune else S.get_tuning()
    for _ in range(args.warmup):
        S.apply(x, y, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        S.apply(x, y, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    if args.copy_probe:
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    alg_bytes = 2 * n * 8 + int(S.info.device_bytes)
    kernel = kernel_name(S)
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic, traffic_tuning = traffic_from_profile(kernel, args.workload, alg_bytes)
    if traffic is not None and traffic_tuning != tuning_str(tuning):
        # counters taken at another launch tuning describe another kernel run
        traffic = None

    # a few fused Lanczos steps (H*psi + alpha + update + beta) on the same input
    lz = None
    if args.lanczos_steps > 0:
        S.lanczos(x, 2, fixed_steps=True)
        torch.cuda.synchronize()
        tl = time.perf_counter()
        e, st, _ = S.lanczos(x, args.lanczos_steps, fixed_steps=True)
        lz = dict(steps=st["steps"], ms_per_step=round((time.perf_counter() - tl) * 1e3 / st["steps"], 4))

    line = {
        "metric": "H\u00b7\u03c8 applies/s + HBM GB/s (16-site Hubbard); batched solves/s, p50/p99 lat",
        "value": round(args.steps / wall, 3),
        "unit": "H*psi/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": p.model.name + "_" + p.cut.kind, "sites": p.model.n_sites,
                   "n_up": p.n_up, "n_dn": p.n_dn, "dim": n, "blocks": int(S.info.n_blocks),
                   "kernel": kernel, "tuning": tuning},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "traffic_tuning": traffic_tuning, "algorithmic_bytes": alg_bytes,
                     "kernel_ms": round(kern_ms, 5), "kernel": kernel},
        "lanczos": lz,
    }
    del y
    torch.cuda.empty_cache()
    progress(f"headline done: {kern_ms:.4f} ms per apply")
    if not args.no_others:
        line["other_workloads"] = other_workloads([w for w in ("heisenberg16", "hubbard12", "j1j2_6x5",
                                                             "hubbard14_spatial") if w != args.workload], stream)
    progress("other workloads done")
    if not args.no_solve:
        p.meta["name"] = args.workload
        line["ground_state"] = ground_state_solve(S, p, args.solve_keep, 1e-10)
    progress("ground-state solve done")
    if not args.no_analyses and not args.no_others:
        line["analyses"] = analyses(stream)
    if args.serving > 0:
        line["serving"] = serving_bench(args.serving, args.serving_budget_gb)
    progress("serving done")
    if not args.no_cpu_baseline:
        p.meta["name"] = args.workload
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
