#!/usr/bin/env python3
"""Throughput of the space-charge PIC step on one MI355X, in particle-steps/s.

One step = the whole hot path over the beam: box and grid geometry, charge deposition,
integrated Green's function and its FFT, zero-padded FFT Poisson solve and field, fused field
gather + space-charge kick + drifts + thin quadrupole (pic_track_n_steps).  Inputs are resident
in HBM before the timed region (the beam is generated on the device).

Workload (default): 1e8 macroparticles, 6-D Gaussian with a 10 % uniform halo out to 4 sigma,
128^3 grid (256^3 padded FFT), TSC, thin-lens FODO, float64 grid; the float32-grid variant is
timed on the same beam and reported next to it.

Prints ONE JSON line.  `--gpus N` with N > 1 exits: this build runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published peak
METRIC = "particle-steps/s, 1e8 ptcl 128^3 space-charge PIC; FP32/batched/adjoint vs plain"
# algorithmic bytes per particle per launch (float64 phase space)
ALGO_BYTES = {
    "deposit": 24,   # read x, y, z
    "gkd": 96,       # read and write the six coordinates
}
KERNEL_SOURCES = {"gkd": "paper_2208_02382_amd/csrc/particles.hip",
                  "deposit": "paper_2208_02382_amd/csrc/particles.hip"}


def _source_hash(rel):
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0].strip() in ("source_sha256_16", "bytes_per_launch"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("source_sha256_16") != _source_hash(KERNEL_SOURCES[kernel]):
        return None
    try:
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_gpu(cfg, steps, warmup, grid_fp32, X=None):
    import torch
    import paper_2208_02382_amd as pic

    beam = pic.Beam(cfg.n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV,
                    cfg.shape, cfg.nodes, grid_fp32=grid_fp32, X=X)
    beam.init(cfg.sigma_matrix, seed=cfg.seed, halo_frac=cfg.halo_frac)
    if warmup:
        beam.track(cfg.lattice, warmup)
    torch.cuda.synchronize()
    beam.profile_start()
    t0 = time.perf_counter()
    beam.track(cfg.lattice, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = beam.profile_read()
    st = beam.check()
    if st != pic.PIC_OK:
        raise RuntimeError("device error flag set: %s" % pic.STATUS_NAMES.get(st, st))
    mean, cov = beam.moments()
    return beam, t1 - t0, stages, cov


def cpu_baseline(cfg, n_sample):
    """One oracle step on a sample of the workload's particles (full grid), single thread."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import workloads
    from oracle import pic as opic

    xi = workloads.draw_xi(cfg, n=n_sample)
    prob = opic.make_problem(n_sample, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV,
                             cfg.mass_MeV, cfg.nodes, cfg.shape)
    X = opic.init_from_normals(cfg.sigma_matrix, xi)
    ks, dss = workloads.lattice_arrays(cfg)

    def go():
        t0 = time.perf_counter()
        opic.track(X, ks, dss, 1, prob)
        return time.perf_counter() - t0

    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            dt = go()
    else:
        dt = go()
    return {"value": n_sample / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "1 oracle step (NumPy float64, 1 thread) of %d particles drawn like the "
                      "%d-particle workload, on its full %dx%dx%d grid with %s; includes the "
                      "double-double IGF and the padded FFTs; %.1f s"
                      % (n_sample, cfg.n, *cfg.nodes, "TSC" if cfg.shape == 2 else "CIC", dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gausshalo-1e8-128c-tsc")
    ap.add_argument("--cpu-sample", type=int, default=200_000,
                    help="particles in the oracle's timed sample (0 disables)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32-grid variant")
    ap.add_argument("--copy-ref-bytes", type=int, default=0,
                    help="first run one device-to-device copy of this many bytes (a reference "
                         "of known traffic for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported (the multi-GPU "
              "sharding is a design in DESIGN.md, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads

    cfg = workloads.CONFIGS[args.workload]
    if args.copy_ref_bytes > 0:
        src = torch.ones(args.copy_ref_bytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    beam, dt, stages, _ = run_gpu(cfg, args.steps, args.warmup, grid_fp32=False)
    ps = cfg.n * args.steps / dt

    def roof(name, stg):
        ms, cnt = stg[name]
        avg = ms / cnt / 1e3
        achieved = ALGO_BYTES[name] * cfg.n / avg / 1e9
        t = _traffic(name, cfg.name)
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": t,
                "kernel": name, "avg_launch_ms": avg * 1e3,
                "algorithmic_bytes_per_launch": ALGO_BYTES[name] * cfg.n}

    kernels = {k: roof(k, stages) for k in ("gkd", "deposit")}
    dominant = max(kernels, key=lambda k: stages[k][0])
    stage_ms = {k: v[0] / max(v[1], 1) for k, v in stages.items()}

    variants = {}
    if not args.no_fp32:
        X = beam.X
        beam.close()
        del beam
        b32, dt32, st32, _ = run_gpu(cfg, args.steps, args.warmup, grid_fp32=True, X=X)
        variants["fp32_grid"] = {
            "value": cfg.n * args.steps / dt32, "ms_per_step": dt32 / args.steps * 1e3,
            "stage_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in st32.items()},
            "note": "charge grid, FFT, field and gather in float32; particles and push float64"}
        b32.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": ps, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "particles": cfg.n, "grid": list(cfg.nodes),
                   "shape": "TSC" if cfg.shape == 2 else "CIC", "grid_dtype": "f64",
                   "halo_frac": cfg.halo_frac, "lattice": "thin FODO k=+-1/m, 0.5 m"},
        "roofline": kernels[dominant],
        "kernels": kernels,
        "stage_ms_per_launch": stage_ms,
        "variants": variants,
    }
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
