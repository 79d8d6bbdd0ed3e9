#!/usr/bin/env python3
"""Benchmark of the coupled LBM-PSM-DEM time step on one MI355X.

Workload (default): the precision form's lattice, 512^3 periodic, tau = 0.55,
Kolmogorov forcing of amplitude 1e-6; 50,000 prolate ellipsoids (6, 3, 3) at
seeded non-overlapping positions with uniform random orientations, density
ratio 1.2; linear spring-dashpot k_n = 1e3, restitution 0.8, Coulomb mu = 0.3,
18 DEM substeps; FP32 populations (shifted storage), FP64 particles; 50 warm-up
and 500 timed coupled steps.  Synthetic seeded data.  --workload couette runs
the bounded Couette suspension (128^3, 500 spheres of radius 5).

Prints one JSON line: coupled-step MLUPS (lattice updates per second of whole
coupled steps, every phase included), the roofline of the dominant kernel
(measured with HIP events on the domain stream), the roofline of the whole
coupled step (its algorithmic bytes over the step time), and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "coupled-step MLUPS + % HBM peak; ensemble jobs/s and p99 latency at equal error"
STORAGE_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}


def parse():
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=500)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--precision", default="fp32", choices=list(STORAGE_BYTES))
    p.add_argument("--workload", default="kolmogorov", choices=["couette", "kolmogorov", "bed", "fluidized"],
                   help="kolmogorov: prolate ellipsoids in a forced periodic box (512^3, 50,000 ellipsoids); "
                        "couette: spheres in bounded shear (128^3, 500 spheres); bed: polydisperse spheres "
                        "settling in a walled 256x256x128 box (n_sub 32); fluidized: the paper's fluidized bed")
    p.add_argument("--n", type=int, default=0, help="lattice edge of the workload (0: 512 kolmogorov, 128 couette)")
    p.add_argument("--phi", type=float, default=0.15, help="solid volume fraction of the fluidized bed")
    p.add_argument("--fluidized-sweep", action="store_true",
                   help="the paper's performance study: fluidized bed 500x200x800 at phi = 0, 0.15, 0.30, "
                        "0.45 in FP32, FP64 and BF16 storage, one JSON line per point")
    p.add_argument("--collision", default=None, choices=["bgk", "trt"],
                   help="fluid operator inside the PSM collision (TRT: the paper's tau- rule); default: the "
                        "workload's own (TRT for the fluidized bed, as in the paper's studies, else BGK)")
    p.add_argument("--spheres", type=int, default=500)
    p.add_argument("--cpu-sample-steps", type=int, default=-1,
                   help="coupled steps of the CPU oracle sample (0: skip the CPU baseline; -1: the workload's "
                        "default, 600 on the 64^3 ellipsoid box of the same recipe, 120 on the Couette workload)")
    p.add_argument("--no-timing", action="store_true", help="skip the per-kernel event timing pass")
    p.add_argument("--serve-jobs", type=int, default=32,
                   help="jobs of the ensemble-serving sample (0: skip the serving measurement)")
    p.add_argument("--serve-steps", type=int, default=100, help="coupled steps per served job")
    p.add_argument("--serve-rate", type=float, default=50.0, help="mean arrival rate of served jobs (1/s)")
    p.add_argument("--serve-slots", type=int, default=32, help="active slots of the server")
    p.add_argument("--serve-budget-gb", type=float, default=2.0, help="HBM budget of the held jobs (GiB)")
    p.add_argument("--stream-probe", type=int, default=0, metavar="MIB",
                   help="attainable streaming bandwidth: copy / read / write kernels over MIB-sized buffers")
    p.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                   help="only run 20 plain device copies of MIB MiB (calibrates the HBM byte counters)")
    p.add_argument("--lbm-sweep", type=int, default=0, metavar="N",
                   help="only time the LBM pass of a periodic fluid-only N^3 lattice in every precision")
    p.add_argument("--precision-study", type=int, default=0, metavar="N",
                   help="only run the Kolmogorov-ellipsoid N^3 workload in FP64, FP32, BF16 and FP16 from the same "
                        "start: coupled-step speed and the errors of each against the FP64 run at step 200")
    p.add_argument("--summarize", nargs="+", metavar="DIR",
                   help="print a per-kernel summary of rocprofv3 CSV output (no GPU): DIR of a --kernel-trace "
                        "--stats run, or four DIRs of --pmc runs: FETCH_SIZE, WRITE_SIZE, and the same two "
                        "counters over --copy-probe")
    p.add_argument("--kernel", default="k_lbm", help="kernel-name filter of the counter summary")
    return p.parse_args()


def lbm_source_digest():
    """Digest of the LBM kernel source: counter-derived traffic is reported only
    while the kernel is the one the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "paper_2512_04997_amd", "csrc", "lbm.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per LBM pass from a committed counter summary
    (profiles/lbm_*_traffic.txt), if one was taken on this workload and
    precision and on the current kernel source; else None."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "lbm_*_traffic.txt"))):
        try:
            rec = json.loads(open(path).read().split("JSON:", 1)[1].strip().splitlines()[0])
        except (OSError, IndexError, ValueError):
            continue
        if (rec.get("lbm_source") == lbm_source_digest() and rec.get("precision") == precision
                and rec.get("workload") == workload):
            return rec.get("bytes_per_pass")
    return None


def _csv(path):
    import csv
    return list(csv.DictReader(open(path)))


def summarize(dirs, kernel_filter):
    """Per-kernel tables from rocprofv3 CSV output (host-only parsing)."""
    import glob
    if len(dirs) == 1:
        f = glob.glob(os.path.join(dirs[0], "*kernel_stats.csv"))[0]
        rows = sorted(_csv(f), key=lambda r: -float(r["TotalDurationNs"]))
        tot = sum(float(r["TotalDurationNs"]) for r in rows)
        print("| kernel | calls | avg us | total ms | % |")
        print("|---|---|---|---|---|")
        for r in rows[:25]:
            print(f"| `{r['Name'][:100]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                  f"{float(r['TotalDurationNs']) / 1e6:.3f} | {100 * float(r['TotalDurationNs']) / tot:.1f} |")
        return
    if len(dirs) != 4:
        raise SystemExit("--summarize takes one kernel-trace directory or four counter directories")

    def per_kernel(d, counter):
        f = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
        out = {}
        for r in _csv(f):
            if r["Counter_Name"] != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    fetch, write = per_kernel(dirs[0], "FETCH_SIZE"), per_kernel(dirs[1], "WRITE_SIZE")
    cf, cw = per_kernel(dirs[2], "FETCH_SIZE"), per_kernel(dirs[3], "WRITE_SIZE")
    # the copy probe: 20 copies of a known size; the counters' KiB against the bytes moved
    probe_kib = max(max(v) for k, v in cw.items() if "copyBuffer" in k or "copy" in k.lower())
    ck = [k for k in cf if "copyBuffer" in k][0]
    f_fetch = probe_kib / (sum(cf[ck]) / len(cf[ck]))
    f_write = probe_kib / (sum(cw[ck]) / len(cw[ck]))
    print(f"copy probe: {probe_kib:.0f} KiB read and written per copy; FETCH_SIZE reads "
          f"{sum(cf[ck]) / len(cf[ck]):.0f} KiB (factor {f_fetch:.3f}), WRITE_SIZE reads "
          f"{sum(cw[ck]) / len(cw[ck]):.0f} KiB (factor {f_write:.3f})")
    print("| kernel | dispatches | FETCH_SIZE KiB (avg) | WRITE_SIZE KiB (avg) | scaled MB per dispatch |")
    print("|---|---|---|---|---|")
    for k in sorted(set(fetch) | set(write)):
        if kernel_filter not in k:
            continue
        fv, wv = fetch.get(k, [0.0]), write.get(k, [0.0])
        mb = (f_fetch * sum(fv) / len(fv) + f_write * sum(wv) / len(wv)) * 1024 / 1e6
        print(f"| `{k[:90]}` | {len(fv)} | {sum(fv) / len(fv):.0f} | {sum(wv) / len(wv):.0f} | {mb:.1f} |")
    return f_fetch, f_write, fetch, write


def lbm_sweep(n, collision="bgk"):
    """LBM pass of a periodic fluid-only n^3 lattice (body force on), all precisions."""
    import torch
    from paper_2512_04997_amd import psmdem, workloads
    torch.cuda.set_device(0)
    for prec, sb in STORAGE_BYTES.items():
        cfg = workloads.base_config((n, n, n), 0.7, precision=prec, body_force=[1e-6, 0.0, 0.0],
                                    collision=collision)
        D = psmdem.Domain(cfg, None)
        D.step(10)
        D.sync()
        D.set_timing(True)
        D.step(50)
        D.set_timing(False)
        ms, _ = D.timing("lbm")
        N = n ** 3
        print(json.dumps({"lbm_sweep": prec, "collision": collision, "n": n, "lbm_ms": round(ms, 4), "mlups": round(N / ms / 1e3, 1),
                          "alg_GBs": round(N * 2 * 19 * sb / (ms * 1e-3) / 1e9, 1),
                          "frac": round(N * 2 * 19 * sb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}), flush=True)
        D.close()


def fluidized_sweep(warmup, steps, collision):
    """Coupled-step throughput of the paper's fluidized bed (500 x 200 x 800,
    D = 20, 10 substeps, distance solid fraction) against the solid fraction,
    in FP64, FP32 and BF16 storage: one JSON line per point.  Each point runs
    warmup + steps + 20 timed-pass steps from the same start in every
    precision, and FP32 and BF16 state their errors against the FP64 run at
    the end (fluid velocity against max(|u|, 1e-3) and in relative L2;
    particle velocities against the largest of the FP64 run; hydrodynamic
    forces in relative L2)."""
    import numpy as np
    import torch
    from paper_2512_04997_amd import psmdem, workloads
    torch.cuda.set_device(0)
    for phi in (0.0, 0.15, 0.30, 0.45):
        cfg, parts, meta = workloads.fluidized_bed(phi=phi)
        ref = None
        for prec in ("fp64", "fp32", "bf16"):
            cfg = dict(cfg, precision=prec)
            if collision:
                cfg["collision"] = collision
            N = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
            D = psmdem.Domain(cfg, parts, stream=torch.cuda.current_stream())
            D.step(warmup)
            D.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            D.step(steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            D.sync()
            D.set_timing(True)
            D.step(min(steps, 20))
            D.set_timing(False)
            parts_ms = {k: round(D.timing(k)[0], 4) for k in ("lbm", "voxel", "dem", "hydro")}
            dem_n = D.timing("dem")[1] // max(D.timing("lbm")[1], 1)
            parts_ms["dem"] = round(parts_ms["dem"] * dem_n, 4)
            ctr = D.counters()
            out = {"fluidized_bed": meta["workload"], "phi": phi, "precision": prec,
                   "particles": 0 if parts is None else len(parts["pos"]), "steps": steps,
                   "ms_per_step": round(el / steps * 1e3, 4), "mlups": round(N * steps / el / 1e6, 1),
                   "per_step_ms": parts_ms, "contacts": ctr["n_contacts"], "pairs": ctr["n_pairs"]}
            _, u = D.fields()
            P = D.particles() if parts is not None else None
            if ref is None:
                ref = (u, P)
                out["max_u"] = float(np.abs(u).max())
            else:
                u0, P0 = ref
                out["errors_vs_fp64"] = {"u_rel_l2": _rel_l2(u, u0), "u_rel_linf": _rel_inf(u, u0, 1e-3)}
                if P is not None:
                    out["errors_vs_fp64"].update({"v_rel_linf": _rel_inf(P["vel"], P0["vel"]),
                                                  "f_hyd_rel_l2": _rel_l2(P["f_hyd"], P0["f_hyd"])})
            print(json.dumps(out), flush=True)
            D.close()
            del D, u, P
            torch.cuda.empty_cache()


def _rel_l2(a, b):
    import numpy as np
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / nb if nb > 0 else float(np.linalg.norm(a - b))


def _rel_inf(a, b, floor=0.0):
    import numpy as np
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), floor)


def precision_study(n, warmup=20, timed=100, check=200):
    """Same particle set and start in every population precision; speed of the
    coupled step and of the LBM pass, and the errors against the FP64 run at
    step `check` (fluid velocity against max(|u|, 1e-3) and in relative L2;
    particle velocities and rotation rates against the largest of the FP64
    run; hydrodynamic forces and torques in relative L2).  One domain at a
    time; the FP64 reference state is kept on the host."""
    import numpy as np
    import torch
    from paper_2512_04997_amd import psmdem, workloads
    torch.cuda.set_device(0)
    cfg, parts, meta = workloads.kolmogorov_ellipsoids(n=n)
    N = n ** 3
    ref = None
    for prec in ("fp64", "fp32", "bf16", "fp16"):
        D = psmdem.Domain(dict(cfg, precision=prec), parts)
        D.step(warmup)
        D.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        D.step(timed)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / timed
        D.set_timing(True)
        D.step(10)
        D.set_timing(False)
        lbm_ms, _ = D.timing("lbm")
        D.step(check - warmup - timed - 10)
        D.sync()
        _, u = D.fields()
        P = D.particles()
        out = {"precision_study": prec, "workload": meta["workload"], "n_sub": D.info()["n_sub"],
               "ms_per_step": round(dt * 1e3, 4), "mlups": round(N / dt / 1e6, 1), "lbm_ms": round(lbm_ms, 4),
               "lbm_GBs": round(N * 2 * 19 * STORAGE_BYTES[prec] / (lbm_ms * 1e-3) / 1e9, 1), "step": check}
        if ref is None:
            ref = (u.astype(np.float64), {k: P[k].copy() for k in ("vel", "omega", "f_hyd", "m_hyd")})
            out["max_u"] = float(abs(u).max())
            out["max_v"] = float(abs(P["vel"]).max())
        else:
            u0, P0 = ref
            out.update({"u_rel_l2": _rel_l2(u, u0), "u_rel_linf": _rel_inf(u, u0, 1e-3),
                        "v_rel_linf": _rel_inf(P["vel"], P0["vel"]),
                        "omega_rel_linf": _rel_inf(P["omega"], P0["omega"]),
                        "f_hyd_rel_l2": _rel_l2(P["f_hyd"], P0["f_hyd"]),
                        "m_hyd_rel_l2": _rel_l2(P["m_hyd"], P0["m_hyd"])})
        print(json.dumps(out), flush=True)
        D.close()
        del u, P, D
        torch.cuda.empty_cache()


def stream_probe(mib):
    """The device's attainable streaming rates (plain copy, read, write kernels
    of the measurement library), the ceiling beside the roofline's 8 TB/s."""
    import torch
    from paper_2512_04997_amd import probe
    torch.cuda.set_device(0)
    nbytes = mib << 20
    a = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    for grid in (1024, 4096, 16384):
        for kind, moved in (("copy", 2 * nbytes), ("read", nbytes), ("write", nbytes)):
            ms = probe.stream(kind, a.data_ptr(), b.data_ptr(), nbytes, grid)
            print(json.dumps({"stream_probe": kind, "grid": grid, "bytes_moved": moved, "ms": round(ms, 4),
                              "TB_s": round(moved / (ms * 1e-3) / 1e12, 3),
                              "frac_of_peak": round(moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}), flush=True)


def copy_probe(mib):
    """Plain device-to-device copies of a known size: the reference that scales
    the FETCH_SIZE / WRITE_SIZE counters of the profiler into HBM bytes."""
    import torch
    n = mib * 2 ** 20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 20}))


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def serve_batched(stream, slots, precision, budget_gb=16.0):
    """The job stream through the continuous-batching server: arrivals on the
    wall clock, a done job released at once.  Latency = done - arrival."""
    from paper_2512_04997_amd import psmdem
    S = psmdem.Server(max_jobs=slots, hbm_budget=int(budget_gb * 2 ** 30), precision=precision)
    t0 = psmdem.clock()
    ids = {}
    lat = []
    k = 0
    n_done = 0
    shown = t0
    while n_done < len(stream):
        if psmdem.clock() - shown > 20.0:
            shown = psmdem.clock()
            print(f"[bench] serving (batched): {n_done} of {len(stream)} jobs done after {shown - t0:.0f} s",
                  file=sys.stderr, flush=True)
        now = psmdem.clock() - t0
        while k < len(stream) and stream[k][0] <= now:
            arr, cfg, parts, steps = stream[k]
            ids[S.submit(cfg, parts, steps)] = arr
            k += 1
        n_active, n_queued = S.iterate()
        if n_active == 0 and n_queued == 0 and k < len(stream):
            time.sleep(max(0.0, min(0.01, stream[k][0] - (psmdem.clock() - t0))))
        for j in list(ids):
            info = S.job(j)
            if info["state"] == "done":
                lat.append(info["t_done"] - t0 - ids.pop(j))
                S.release(j)
                n_done += 1
            elif info["state"] == "failed":
                raise RuntimeError(f"served job failed: {info}")
    wall = psmdem.clock() - t0
    S.close()
    return wall, lat


def serve_one_at_a_time(stream):
    """The same stream, one job at a time in arrival order through the
    single-domain API (create, step, synchronise)."""
    from paper_2512_04997_amd import psmdem
    import torch
    t0 = psmdem.clock()
    lat = []
    shown = t0
    for arr, cfg, parts, steps in stream:
        if psmdem.clock() - shown > 20.0:
            shown = psmdem.clock()
            print(f"[bench] serving (one at a time): {len(lat)} of {len(stream)} jobs done after {shown - t0:.0f} s",
                  file=sys.stderr, flush=True)
        wait = arr - (psmdem.clock() - t0)
        if wait > 0:
            time.sleep(wait)
        D = psmdem.Domain(cfg, parts)
        D.step(steps)
        D.sync()
        torch.cuda.synchronize()
        lat.append(psmdem.clock() - t0 - arr)
        D.close()
    return psmdem.clock() - t0, lat


def serving(a):
    from paper_2512_04997_amd import workloads
    stream = workloads.serving_stream(njobs=a.serve_jobs, rate=a.serve_rate, steps=a.serve_steps,
                                      precision="fp32")
    lups = sum(c["n"][0] * c["n"][1] * c["n"][2] * st for _, c, _, st in stream)
    # warm both paths (code objects, allocator pools) on a short prefix
    warm = [(0.0, c, p, 2) for _, c, p, _ in stream[:4]]
    serve_batched(warm, a.serve_slots, "fp32", a.serve_budget_gb)
    serve_one_at_a_time(warm)
    wb, lb = serve_batched(stream, a.serve_slots, "fp32", a.serve_budget_gb)
    ws, ls = serve_one_at_a_time(stream)
    res = {"jobs": len(stream), "steps_per_job": a.serve_steps, "arrival_rate_per_s": a.serve_rate,
           "slots": a.serve_slots, "hbm_budget_gib": a.serve_budget_gb,
           "lattices": "uniform over 32^3, 64^3, 96^3, 128^3",
           "lattice_updates": lups,
           "batched": {"mlups": round(lups / wb / 1e6, 1), "jobs_per_s": round(len(stream) / wb, 3),
                       "p50_s": round(_pct(lb, 50), 4), "p99_s": round(_pct(lb, 99), 4), "wall_s": round(wb, 3)},
           "one_at_a_time": {"mlups": round(lups / ws / 1e6, 1), "jobs_per_s": round(len(stream) / ws, 3),
                             "p50_s": round(_pct(ls, 50), 4), "p99_s": round(_pct(ls, 99), 4),
                             "wall_s": round(ws, 3)}}
    res["speedup"] = round(ws / wb, 3)
    return res


def cpu_baseline(cfg, parts, steps, name):
    """FP64 CPU oracle on a bounded sample of the workload (coupled steps of
    `cfg`, which the caller names)."""
    from oracle import oracle
    threads = min(os.cpu_count() or 1, 16)
    oracle.set_threads(threads)
    D = oracle.OracleDomain(cfg, parts)
    D.step(1)  # first step outside the clock
    t0 = time.perf_counter()
    D.step(steps)
    dt = time.perf_counter() - t0
    N = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    return {"value": N * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.get_threads(),
            "kind": "oracle",
            "sample": f"{steps} coupled steps of {name} (after one untimed step), FP64, {dt:.1f} s"}


def main():
    a = parse()
    if a.summarize:
        summarize(a.summarize, a.kernel)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): the coupled step of one "
              "domain is a single-GPU build; see the design notes for how it would shard.", file=sys.stderr)
        sys.exit(2)
    import torch

    if a.stream_probe:
        stream_probe(a.stream_probe)
        return
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    if a.lbm_sweep:
        lbm_sweep(a.lbm_sweep, a.collision or "bgk")
        return
    if a.precision_study:
        precision_study(a.precision_study)
        return
    if a.fluidized_sweep:
        fluidized_sweep(a.warmup, a.steps, a.collision)
        return
    from paper_2512_04997_amd import psmdem, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n = a.n or (512 if a.workload == "kolmogorov" else 128)
    if a.workload == "couette":
        cfg, parts, meta = workloads.couette_suspension(precision=a.precision, n=n, nsph=a.spheres)
    elif a.workload == "kolmogorov":
        cfg, parts, meta = workloads.kolmogorov_ellipsoids(n=n, precision=a.precision)
    elif a.workload == "fluidized":
        cfg, parts, meta = workloads.fluidized_bed(precision=a.precision, phi=a.phi)
    else:
        cfg, parts, meta = workloads.settling_bed_dense(precision=a.precision)
    if a.collision:
        cfg["collision"] = a.collision
    N = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    stream = torch.cuda.current_stream()
    D = psmdem.Domain(cfg, parts, stream=stream)
    info = D.info()
    print(f"[bench] {meta['workload']} {a.precision}: n_sub={info['n_sub']} particles={info['n_particles']} "
          f"device={info['device_bytes'] / 2**20:.0f} MiB", file=sys.stderr, flush=True)
    D.step(a.warmup)
    D.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    D.step(a.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    D.sync()
    ms = elapsed / a.steps * 1e3
    mlups = N * a.steps / elapsed / 1e6
    ctr = D.counters()
    print(f"[bench] {a.steps} steps in {elapsed:.3f} s: {ms:.3f} ms/step, {mlups:.0f} MLUPS; "
          f"solid tiles {ctr['n_solid_tiles']}, entries {ctr['n_entries']}, registrations {ctr['n_registrations']}, "
          f"pairs {ctr['n_pairs']}, contacts {ctr['n_contacts']}", file=sys.stderr, flush=True)

    sb = STORAGE_BYTES[a.precision]
    np_ = info["n_particles"]
    # algorithmic bytes of one coupled step: populations read and written once,
    # a solid-presence bit per cell, solid-fraction entries written and read,
    # hydrodynamic force and torque out, and per substep the particle state,
    # the cell-list keys and the pair list with history and contact outputs
    step_terms = {
        "populations": N * 2 * 19 * sb,
        "solid_presence": N / 8.0,
        "solid_entries": ctr["n_entries"] * (4 + 4 + (8 if a.precision == "fp64" else 4)) * 2,
        "hydro_out": np_ * 48,
        "dem": info["n_sub"] * (np_ * 500 + ctr["n_registrations"] * 16 + ctr["n_pairs"] * (8 + 24 * 2 + 72)),
    }
    step_bytes = sum(step_terms.values())
    step_gbs = step_bytes / (ms * 1e-3) / 1e9
    step_roof = {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(step_gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_step": int(step_bytes),
                 "terms": {k: int(v) for k, v in step_terms.items()}}

    roof = None
    parts_ms = None
    if not a.no_timing:
        # a separate pass with HIP events around every kernel family on the domain stream
        D.set_timing(True)
        D.step(min(a.steps, 50))
        D.set_timing(False)
        lbm_ms, lbm_n = D.timing("lbm")
        vox_ms, _ = D.timing("voxel")
        dem_ms, dem_n = D.timing("dem")
        hyd_ms, _ = D.timing("hydro")
        groups = dem_n / max(lbm_n, 1)
        parts_ms = {"lbm": round(lbm_ms, 4), "voxel": round(vox_ms, 4), "dem": round(dem_ms * groups, 4),
                    "hydro_and_corrector": round(hyd_ms, 4)}
        alg_bytes = N * 2 * 19 * sb
        achieved = alg_bytes / (lbm_ms * 1e-3) / 1e9
        traffic = measured_traffic(meta["workload"], a.precision)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "LBM collide-stream pass (one k_lbm_mixed launch over fluid and PSM tiles per step)",
                "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": round(lbm_ms, 5)}
        print(f"[bench] per step: lbm {lbm_ms:.4f} ms, voxel {vox_ms:.4f} ms, hydro {hyd_ms:.4f} ms, "
              f"dem {dem_ms * groups:.4f} ms ({groups:.0f} DEM launch groups)", file=sys.stderr, flush=True)

    serve = None
    if a.serve_jobs > 0:
        serve = serving(a)
        print(f"[bench] serving {serve['jobs']} jobs x {serve['steps_per_job']} steps: batched "
              f"{serve['batched']['mlups']} MLUPS p50 {serve['batched']['p50_s']} s p99 {serve['batched']['p99_s']} s; "
              f"one at a time {serve['one_at_a_time']['mlups']} MLUPS p50 {serve['one_at_a_time']['p50_s']} s "
              f"p99 {serve['one_at_a_time']['p99_s']} s", file=sys.stderr, flush=True)

    cpu = None
    cpu_steps = a.cpu_sample_steps
    if cpu_steps < 0:
        cpu_steps = 600 if a.workload == "kolmogorov" else 120
    if cpu_steps > 0:
        if a.workload == "kolmogorov" and n > 64:
            # the oracle's two FP64 population arrays of 512^3 would not finish in a
            # bounded sample: it runs the 64^3 box of the same recipe (same forcing
            # amplitude, number density of ellipsoids, contact law)
            ccfg, cparts, cmeta = workloads.kolmogorov_ellipsoids(n=64, precision="fp64")
            cpu = cpu_baseline(ccfg, cparts, cpu_steps, cmeta["workload"])
        else:
            cpu = cpu_baseline(cfg, parts, cpu_steps, meta["workload"])
        print(f"[bench] cpu oracle: {cpu['value']:.2f} MLUPS on {cpu['cores']} threads", file=sys.stderr,
              flush=True)

    out = {"metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": a.precision, "data": "synthetic",
           "config": {"workload": meta["workload"], "lattice": list(cfg["n"]), "particles": info["n_particles"],
                      "n_sub": info["n_sub"], "tau": cfg["tau"], "collision": cfg.get("collision", "bgk"),
                      "populations": a.precision, "particles_dtype": "fp64"},
           "roofline": roof, "coupled_step_roofline": step_roof, "per_step_ms": parts_ms,
           "cpu_baseline": cpu, "serving": serve}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
