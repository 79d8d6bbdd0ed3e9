#!/usr/bin/env python3
"""Benchmark of the coupled LBM-PSM-DEM time step on one MI355X.

Workload (default): bounded Couette shear, 128^3 lattice, walls beyond node
layers 0 and 127 moving at -/+0.02, periodic in x and y, tau = 0.7; 500
spheres of radius 5 at seeded non-overlapping positions, density ratio 1.5;
linear spring-dashpot k_n = 1e3, restitution 0.8, Coulomb mu = 0.3; FP32
populations (shifted storage), FP64 particles.  Synthetic seeded data.

Prints one JSON line: coupled-step MLUPS (lattice updates per second of whole
coupled steps, every phase included), the roofline of the dominant kernel (the
LBM collide-stream pass, measured with HIP events on the domain stream), and
the FP64 CPU oracle timed on a bounded sample of the same workload.
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
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--precision", default="fp32", choices=list(STORAGE_BYTES))
    p.add_argument("--n", type=int, default=128, help="lattice edge of the Couette workload")
    p.add_argument("--spheres", type=int, default=500)
    p.add_argument("--cpu-sample-steps", type=int, default=20,
                   help="coupled steps of the CPU oracle sample (0: skip the CPU baseline)")
    p.add_argument("--no-timing", action="store_true", help="skip the per-kernel event timing pass")
    return p.parse_args()


def cpu_baseline(cfg, parts, steps):
    """FP64 CPU oracle on the same workload for a bounded number of coupled steps."""
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
            "sample": f"{steps} coupled steps of the same workload (after one untimed step), FP64, "
                      f"{dt:.1f} s"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): the coupled step of one "
              "domain is a single-GPU build; see the design notes for how it would shard.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2512_04997_amd import psmdem, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg, parts, meta = workloads.couette_suspension(precision=a.precision, n=a.n, nsph=a.spheres)
    N = a.n ** 3
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
    print(f"[bench] {a.steps} steps in {elapsed:.3f} s: {ms:.3f} ms/step, {mlups:.0f} MLUPS",
          file=sys.stderr, flush=True)

    roof = None
    if not a.no_timing:
        # a separate pass with HIP events around every kernel family on the domain stream
        D.set_timing(True)
        D.step(min(a.steps, 50))
        D.set_timing(False)
        lbm_ms, lbm_n = D.timing("lbm")
        vox_ms, _ = D.timing("voxel")
        dem_ms, dem_n = D.timing("dem")
        hyd_ms, _ = D.timing("hydro")
        sb = STORAGE_BYTES[a.precision]
        alg_bytes = N * 2 * 19 * sb
        achieved = alg_bytes / (lbm_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "LBM collide-stream pass (k_lbm fluid-tile + PSM-tile kernels of one step)",
                "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": round(lbm_ms, 5)}
        print(f"[bench] per step: lbm {lbm_ms:.4f} ms, voxel {vox_ms:.4f} ms, hydro {hyd_ms:.4f} ms, "
              f"dem {dem_ms * dem_n / max(lbm_n, 1):.4f} ms ({dem_n // max(lbm_n, 1)} DEM launch groups)",
              file=sys.stderr, flush=True)

    cpu = None
    if a.cpu_sample_steps > 0:
        cpu = cpu_baseline(cfg, parts, a.cpu_sample_steps)
        print(f"[bench] cpu oracle: {cpu['value']:.2f} MLUPS on {cpu['cores']} threads", file=sys.stderr,
              flush=True)

    out = {"metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": a.precision, "data": "synthetic",
           "config": {"workload": meta["workload"], "lattice": [a.n] * 3, "particles": info["n_particles"],
                      "n_sub": info["n_sub"], "tau": cfg["tau"], "populations": a.precision,
                      "particles_dtype": "fp64"},
           "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
