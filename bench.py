#!/usr/bin/env python3
"""Throughput of the space-charge PIC step on one MI355X, in particle-steps/s.

One step = the whole hot path over the beam: box and grid geometry, charge deposition,
integrated Green's function and its FFT, zero-padded FFT Poisson solve and field, fused field
gather + space-charge kick + drifts + thin quadrupole.  Inputs are resident in HBM before the
timed region (the beam is generated on the device).  The timed call is pic_track_n_steps_binned
(the particles stay in the library's tile order between calls, as after the warm-up call);
the same workload through pic_track_n_steps, which starts from and returns to the caller's
particle order in every call, is reported next to it (variants.caller_order).

Workload (default): 1e8 macroparticles, 6-D Gaussian with a 10 % uniform halo out to 4 sigma,
128^3 grid (256^3 padded FFT), TSC, thin-lens FODO, float64 grid; the float32-grid variant is
timed on the same beam and reported next to it.

Prints ONE JSON line.  `--gpus N` with N > 1 exits: the library tracks a beam on one GPU.
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
# algorithmic bytes per particle per launch (float64 phase space): what the method itself must
# move, the deposit reading x, y, z and the fused gather-kick-drift reading and writing the six
# coordinates
ALGO_BYTES = {
    "deposit": 24,
    "gkd": 96,
}
# bytes per particle per launch the binned kernels move on top of that in the steady state of
# the tracking loop, reported separately: the sort permutation's source index (both kernels)
# and, where particle labels are carried (the caller's order), the id the gather-kick reads and
# writes
OVERHEAD_BYTES = {
    "deposit": 4,
    "gkd": 4,
}
ID_BYTES = {"deposit": 0, "gkd": 8}
# (file, device function) whose source text the counter figures were taken on
KERNEL_SOURCES = {"gkd": ("paper_2208_02382_amd/csrc/sort.hip", "gkd_tiles_body"),
                  "deposit": ("paper_2208_02382_amd/csrc/sort.hip", "deposit_tiles_body")}


def function_text(path, name):
    """Source text of the definition of device function `name` in `path`: from the line that
    declares it to the first closing brace in column 0 after that."""
    lines = open(path).read().split("\n")
    start = next(i for i, l in enumerate(lines)
                 if ("void %s(" % name) in l and not l.rstrip().endswith(";"))
    # include the template line above the declaration
    if start > 0 and lines[start - 1].startswith("template"):
        start -= 1
    end = next(i for i in range(start, len(lines)) if lines[i] == "}")
    return "\n".join(lines[start:end + 1])


def _source_hash(kernel):
    rel, func = KERNEL_SOURCES[kernel]
    text = function_text(os.path.join(ROOT, rel), func)
    return hashlib.sha256(text.encode()).hexdigest()[:16]


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
    if rec.get("source_sha256_16") != _source_hash(kernel):
        return None
    try:
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def tuned(cfg, grid_fp32, enabled):
    """Launch tuning of the binned kernels for this workload (cached, else searched now,
    outside any timed region)."""
    if not enabled:
        return None, None
    from paper_2208_02382_amd import autotune
    rec = autotune.tune(cfg, grid_fp32=grid_fp32, log=_log)
    t = {k: rec[k] for k in autotune.FIELDS if k in rec}
    return t, {"tuning": t, "tuned_ms_per_step": rec["s_per_step"] * 1e3,
               "default_ms_per_step": rec["default_s_per_step"] * 1e3,
               "candidates": len(rec["tried"])}


def run_gpu(cfg, steps, warmup, grid_fp32, X=None, tuning=None, direct_field=False,
            binned=True):
    """Warm-up call, then `steps` steps in one timed call: pic_track_n_steps_binned (X left in
    the library's tile order between and after the calls) or, binned=False, pic_track_n_steps
    (every call starts from and returns to the caller's particle order)."""
    import torch
    import paper_2208_02382_amd as pic

    beam = pic.Beam(cfg.n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV,
                    cfg.shape, cfg.nodes, grid_fp32=grid_fp32, X=X, tuning=tuning,
                    direct_field=direct_field)
    beam.init(cfg.sigma_matrix, seed=cfg.seed, halo_frac=cfg.halo_frac)
    if warmup:
        beam.track(cfg.lattice, warmup, binned=binned)
    torch.cuda.synchronize()
    beam.profile_start()
    t0 = time.perf_counter()
    beam.track(cfg.lattice, steps, binned=binned)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = beam.profile_read()
    st = beam.check()
    if st != pic.PIC_OK:
        raise RuntimeError("device error flag set: %s" % pic.STATUS_NAMES.get(st, st))
    mean, cov = beam.moments()
    return beam, t1 - t0, stages, cov


def measured_copy_gbs(nbytes=1 << 30, reps=5):
    """Device-to-device copy bandwidth (read + write bytes / time), best of `reps`, HIP events
    on torch's stream: the practical streaming rate next to the published peak."""
    import torch
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / best / 1e9


def lds_atomic_reference(blocks=2048, threads=1024, iters=2048):
    """Measured 64-bit LDS atomic (ds_add_u64) throughput of this GPU, in lane-atomics/s, for
    consecutive words (no bank conflict) and for hash-scattered words (libpic_probe.so), with
    the per-clock-per-CU figure it implies at the published 2.4 GHz over the device's CUs."""
    import ctypes
    import torch
    path = os.path.join(ROOT, "paper_2208_02382_amd", "libpic_probe.so")
    lib = ctypes.CDLL(path)
    lib.probe_lds_u64_atomics.restype = ctypes.c_int
    lib.probe_lds_u64_atomics.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double)]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"clock_GHz": 2.4, "compute_units": cus}
    for pattern, name in ((0, "consecutive"), (1, "scattered")):
        ms = ctypes.c_double()
        if lib.probe_lds_u64_atomics(pattern, blocks, threads, iters, ctypes.byref(ms)) != 0:
            raise RuntimeError("LDS atomic probe failed")
        rate = blocks * threads * iters / (ms.value * 1e-3)
        out[name] = {"lane_atomics_per_s": rate,
                     "per_clock_per_cu": rate / (cus * 2.4e9), "ms": ms.value}
    return out


def device_info():
    import torch
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", ""),
            "compute_units": p.multi_processor_count,
            "memory_GiB": round(p.total_memory / 2**30, 1)}


def _rms(cov):
    import math
    return [math.sqrt(cov[0][0]), math.sqrt(cov[2][2]),
            math.sqrt(cov[0][0] * cov[1][1] - cov[0][1] ** 2),
            math.sqrt(cov[2][2] * cov[3][3] - cov[2][3] ** 2)]


ORACLE_RECORD = os.path.join(ROOT, "tests", "golden", "gauss-1e6-64c-cic_oracle.json")


def fp32_accuracy(cfg, steps):
    """Relative rms size and emittance errors of the float64-grid and float32-grid paths after
    `steps` steps of `cfg` from the seeded draws, against the oracle's tracking of the same beam
    (the stored record of tests/golden/gen_medium_oracle.py, which calls only the oracle)."""
    import torch
    import workloads
    import paper_2208_02382_amd as pic

    with open(ORACLE_RECORD) as f:
        rec = json.load(f)
    if rec["workload"] != cfg.name or str(steps) not in rec["moments"]:
        raise RuntimeError("no stored oracle record for %s after %d steps" % (cfg.name, steps))
    m_oracle = rec["moments"][str(steps)]["objective"]
    xi = torch.from_numpy(workloads.draw_xi(cfg)).cuda()
    out = {}
    for fp32 in (False, True):
        b = pic.Beam(cfg.n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV,
                     cfg.shape, cfg.nodes, grid_fp32=fp32, tuning=tuned(cfg, fp32, True)[0])
        b.init_from_normals(cfg.sigma_matrix, xi)
        t0 = time.perf_counter()
        b.track(cfg.lattice, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _, cov = b.moments()
        err = [abs(a - o) / abs(o) for a, o in zip(_rms(cov), m_oracle)]
        out["f32" if fp32 else "f64"] = (err, dt)
        b.close()
    (e64, t64), (e32, t32) = out["f64"], out["f32"]
    return {"workload": cfg.name, "steps": steps,
            "reference": "FP64 oracle (stored record, tests/golden/gen_medium_oracle.py)",
            "f32_rel_err_sigx_sigy_epsx_epsy": e32, "max_rel_err": max(e32),
            "f64_rel_err_sigx_sigy_epsx_epsy": e64, "f64_max_rel_err": max(e64),
            "f64_particle_steps_per_s": cfg.n * steps / t64,
            "f32_particle_steps_per_s": cfg.n * steps / t32}


def run_batched(n_beams, steps, grid_fp32=False, tune=True, sequential=True):
    """The batched workload in one graph launch per call, against the same beams tracked one
    after another by pic_track_n_steps (the plain per-beam form)."""
    import torch
    import workloads
    import paper_2208_02382_amd as pic

    cfgs = workloads.batch_beams(n_beams=n_beams, steps=steps)
    blocks = 0
    tune_rec = None
    from paper_2208_02382_amd import autotune
    if tune:
        tune_rec = autotune.tune_batch(cfgs, grid_fp32=grid_fp32, log=_log)
        blocks = tune_rec["blocks_per_beam"]
    beams = []
    for c in cfgs:
        b = pic.Beam(c.n, c.qm_qeeV, c.charge_C, c.kin_energy_MeV, c.mass_MeV, c.shape, c.nodes,
                     grid_fp32=grid_fp32,
                     tuning=autotune.batch_tuning(c, tune_rec, grid_fp32) if tune else None)
        b.init(c.sigma_matrix, seed=c.seed)
        beams.append(b)
    total = sum(c.n for c in cfgs)
    batch = pic.Batch(beams, [c.lattice for c in cfgs], blocks_per_beam=blocks)
    t0 = time.perf_counter()
    batch.track(steps)  # captures and instantiates the graph, then runs it
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch.track(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bad = [i for i, st in enumerate(batch.check()) if st != pic.PIC_OK]
    if bad:
        raise RuntimeError("device error flag set on batched beams %s" % bad[:8])
    dt_seq = None
    if sequential:
        t0 = time.perf_counter()
        for c, b in zip(cfgs, beams):
            b.track(c.lattice, steps)
        torch.cuda.synchronize()
        dt_seq = time.perf_counter() - t0
    batch.close()
    for b in beams:
        b.close()
    return {"value": total * steps / dt, "unit": "particle-steps/s", "beams": n_beams,
            "particles_total": total, "steps": steps, "s_per_call": dt,
            "first_call_s_incl_capture": t_first,
            "grid_dtype": "f32" if grid_fp32 else "f64", "blocks_per_beam": blocks or 256,
            "autotune": None if tune_rec is None else
            {"tried": tune_rec["tried"], "chosen": tune_rec["blocks_per_beam"],
             "tile": tune_rec.get("tile", [0, 0, 0])},
            "per_beam_sequential": None if dt_seq is None else
            {"value": total * steps / dt_seq, "s": dt_seq,
             "note": "same beams, one pic_track_n_steps per beam"}}


def run_adjoint(cfg, ckpt_every=10):
    """Forward plus reverse sweep with gradients of w . (sigma_x, sigma_y, eps_x, eps_y) with
    respect to the quad strengths and the initial sigma matrix, next to the plain forward."""
    import torch
    import workloads
    import paper_2208_02382_amd as pic

    b = pic.Beam(cfg.n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, cfg.shape,
                 cfg.nodes, tuning=tuned(cfg, False, True)[0])
    xi = torch.from_numpy(workloads.draw_xi(cfg)).cuda()
    w = (1.0, 1.0, 1.0, 1.0)
    b.init_from_normals(cfg.sigma_matrix, xi)
    b.track_adjoint(cfg.lattice, 2, w, ckpt_every=2, xi=xi)  # warm-up
    b.init_from_normals(cfg.sigma_matrix, xi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m, dk, lam, dL = b.track_adjoint(cfg.lattice, cfg.steps, w, ckpt_every=ckpt_every, xi=xi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.init_from_normals(cfg.sigma_matrix, xi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.track(cfg.lattice, cfg.steps)
    torch.cuda.synchronize()
    dt_fwd = time.perf_counter() - t0
    if b.check() != pic.PIC_OK:
        raise RuntimeError("device error flag set in the reverse sweep")
    b.close()
    return {"value": cfg.n * cfg.steps / dt, "unit": "particle-steps/s (forward equivalent)",
            "workload": cfg.name, "steps": cfg.steps, "checkpoint_every": ckpt_every,
            "s_forward_plus_reverse": dt, "plain_forward": {"value": cfg.n * cfg.steps / dt_fwd,
                                                           "s": dt_fwd},
            "objective_terms": m, "dJ_dk": dk}


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
    try:
        host_cpus = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        host_cpus = os.cpu_count()
    return {"value": n_sample / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "host_cpus": host_cpus, "host_cpu_count": os.cpu_count(),
            "sample": "1 oracle step (NumPy float64, 1 thread) of %d particles drawn like the "
                      "%d-particle workload, on its full %dx%dx%d grid with %s; includes the "
                      "double-double IGF and the padded FFTs; %.1f s"
                      % (n_sample, cfg.n, *cfg.nodes, "TSC" if cfg.shape == 2 else "CIC", dt)}


def oracle_timings():
    """The oracle (NumPy float64, one thread) on every workload: the small case in full, one
    step of the others (a sample of the particles where the full count would take hours),
    extrapolated to particle-steps/s; 8 beams of the batched workload; the reverse sweep on a
    sample of the adjoint workload."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import workloads
    from oracle import adjoint as oadj
    from oracle import pic as opic

    def prob(c, n):
        return opic.make_problem(n, c.qm_qeeV, c.charge_C, c.kin_energy_MeV, c.mass_MeV,
                                 c.nodes, c.shape)

    def track_rate(c, n, steps):
        X = opic.init_from_normals(c.sigma_matrix, workloads.draw_xi(c, n=n))
        ks, dss = workloads.lattice_arrays(c)
        t0 = time.perf_counter()
        opic.track(X, ks, dss, steps, prob(c, n))
        dt = time.perf_counter() - t0
        return n * steps / dt, dt

    out = {"cores": 1, "kind": "oracle"}
    with threadpool_limits(limits=1):
        r, dt = track_rate(workloads.SMALL, workloads.SMALL.n, workloads.SMALL.steps)
        out[workloads.SMALL.name] = {"value": r, "s": dt, "sample": "full run (20 steps)"}
        r, dt = track_rate(workloads.MEDIUM, workloads.MEDIUM.n, 1)
        out[workloads.MEDIUM.name] = {"value": r, "s": dt, "sample": "1 step of all 1e6 particles"}
        r, dt = track_rate(workloads.LARGE, 1_000_000, 1)
        out[workloads.LARGE.name] = {"value": r, "s": dt,
                                     "sample": "1 step of 1e6 of the 1e8 particles, full grid"}
        beams = workloads.batch_beams()[:8]
        tot_n, tot_t = 0, 0.0
        for c in beams:
            _, dt = track_rate(c, c.n, 1)
            tot_n += c.n
            tot_t += dt
        out[workloads.BATCH_NAME] = {"value": tot_n / tot_t, "s": tot_t,
                                     "sample": "1 step of each of the first 8 beams"}
        c = workloads.ADJOINT
        n = 50_000
        X = opic.init_from_normals(c.sigma_matrix, workloads.draw_xi(c, n=n))
        ks, dss = workloads.lattice_arrays(c)
        t0 = time.perf_counter()
        oadj.adjoint(X, ks, dss, 2, prob(c, n), np.ones(4))
        dt = time.perf_counter() - t0
        out[c.name] = {"value": n * 2 / dt, "s": dt, "unit": "particle-steps/s (forward equivalent)",
                       "sample": "forward and reverse sweep, 2 steps of 5e4 particles, full grid"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gausshalo-1e8-128c-tsc")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="particles in the oracle's timed sample (0 disables)")
    ap.add_argument("--order", choices=("binned", "caller"), default="binned",
                    help="binned: pic_track_n_steps_binned (particles stay in the library's tile "
                         "order between calls); caller: pic_track_n_steps (each call returns "
                         "them to the caller's order)")
    ap.add_argument("--no-caller-order", action="store_true",
                    help="skip the caller-order variant of the headline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32-grid variant")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched variant")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint variant")
    ap.add_argument("--no-thick", action="store_true",
                    help="skip the thick-element (Listing 1 FODO) variant")
    ap.add_argument("--no-shard", action="store_true",
                    help="skip one GPU's share of the headline at 8 GPUs (n/8 particles)")
    ap.add_argument("--no-direct", action="store_true",
                    help="skip the direct-field variant (E' from the field's own IGF)")
    ap.add_argument("--batch-beams", type=int, default=256)
    ap.add_argument("--oracle-timings", action="store_true",
                    help="time the oracle on every workload (host CPU, a few minutes) and exit")
    ap.add_argument("--only", choices=("batched", "adjoint"),
                    help="run only this variant (for profiling it) and print its JSON")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched variant without the beam-by-beam comparison")
    ap.add_argument("--no-tune", action="store_true",
                    help="library default launch shapes instead of the autotuned ones")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--copy-ref-bytes", type=int, default=0,
                    help="first run one device-to-device copy of this many bytes (a reference "
                         "of known traffic for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library tracks a beam on one GPU; --gpus %d is not supported (the "
              "multi-GPU sharding is not implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.oracle_timings:
        print(json.dumps({"oracle_timings": oracle_timings()}), flush=True)
        return
    import torch
    import workloads

    cfg = workloads.CONFIGS[args.workload]
    if args.only == "batched":
        print(json.dumps(run_batched(args.batch_beams, args.batch_steps, tune=not args.no_tune,
                                     sequential=not args.no_sequential)), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(run_adjoint(workloads.ADJOINT)), flush=True)
        return
    if args.copy_ref_bytes > 0:
        src = torch.ones(args.copy_ref_bytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuning, tune_info = tuned(cfg, False, not args.no_tune)
    binned = args.order == "binned"
    beam, dt, stages, _ = run_gpu(cfg, args.steps, args.warmup, grid_fp32=False, tuning=tuning,
                                  binned=binned)
    ps = cfg.n * args.steps / dt

    def roof(name, stg):
        ms, cnt = stg[name]
        avg = ms / cnt / 1e3
        achieved = ALGO_BYTES[name] * cfg.n / avg / 1e9
        t = _traffic(name, cfg.name)
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": t,
                "kernel": name, "avg_launch_ms": avg * 1e3,
                "algorithmic_bytes_per_launch": ALGO_BYTES[name] * cfg.n,
                "overhead_bytes_per_launch":
                    (OVERHEAD_BYTES[name] + (0 if binned else ID_BYTES[name])) * cfg.n}

    kernels = {k: roof(k, stages) for k in ("gkd", "deposit")}
    # the deposit's LDS atomics: (S+1)^3 per particle, against the measured ds_add_u64 rates
    lds_ref = lds_atomic_reference()
    n_atomics = (cfg.shape + 1) ** 3 * cfg.n
    dep_rate = n_atomics / (kernels["deposit"]["avg_launch_ms"] * 1e-3)
    kernels["deposit"]["lds_atomics"] = {
        "per_launch": n_atomics, "achieved_per_s": dep_rate,
        "peak_consecutive_per_s": lds_ref["consecutive"]["lane_atomics_per_s"],
        "frac_of_consecutive": dep_rate / lds_ref["consecutive"]["lane_atomics_per_s"],
        "scattered_per_s": lds_ref["scattered"]["lane_atomics_per_s"],
        "frac_of_scattered": dep_rate / lds_ref["scattered"]["lane_atomics_per_s"],
        "reference": lds_ref}
    copy_gbs = measured_copy_gbs()
    for k in kernels.values():
        k["measured_copy_GBs"] = copy_gbs
        k["frac_of_measured_copy"] = k["achieved"] / copy_gbs
    dominant = max(kernels, key=lambda k: stages[k][0])
    stage_ms = {k: v[0] / max(v[1], 1) for k, v in stages.items()}

    variants = {}
    if binned and not args.no_caller_order:
        # the same workload with every call starting from and returning to the caller's order
        X = beam.X
        beam.close()
        del beam
        bc, dtc, stc, _ = run_gpu(cfg, args.steps, args.warmup, grid_fp32=False, X=X,
                                  tuning=tuning, binned=False)
        variants["caller_order"] = {
            "value": cfg.n * args.steps / dtc, "ms_per_step": dtc / args.steps * 1e3,
            "stage_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in stc.items()},
            "note": "pic_track_n_steps: the first step moves the caller's order into tile "
                    "order and the call ends with the return to the caller's order"}
        beam = bc
    if not args.no_fp32:
        X = beam.X
        beam.close()
        del beam
        tuning32, tune32 = tuned(cfg, True, not args.no_tune)
        b32, dt32, st32, _ = run_gpu(cfg, args.steps, args.warmup, grid_fp32=True, X=X,
                                     tuning=tuning32, binned=binned)
        variants["fp32_grid"] = {
            "value": cfg.n * args.steps / dt32, "ms_per_step": dt32 / args.steps * 1e3,
            "stage_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in st32.items()},
            "autotune": tune32,
            "note": "charge grid, FFT, field and gather in float32; particles and push float64"}
        b32.close()
        del X
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_thick:
        # the same beam through the paper's FODO cell of thick elements (Listing 1), one step
        # per slice (125 per cell)
        cfg_t = cfg.with_(lattice=workloads.THICK_FODO)
        bt, dtt, stt, _ = run_gpu(cfg_t, args.steps, args.warmup, grid_fp32=False, tuning=tuning,
                                  binned=binned)
        variants["thick_fodo"] = {
            "value": cfg.n * args.steps / dtt, "ms_per_step": dtt / args.steps * 1e3,
            "stage_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in stt.items()},
            "lattice": "Listing 1 FODO: Drift 0.25, Quad(1.0, k=+1), Drift 0.5, Quad(1.0, k=-1), "
                       "Drift 0.25, 25 slices each; steps are slices",
            "note": "float64; same beam, grid, shape and launch shapes as the headline"}
        bt.close()
        del bt
        torch.cuda.empty_cache()
    if not args.no_thick:
        # slice-step diagnostics (moments after every step) on the headline workload
        import paper_2208_02382_amd as pic
        bd = pic.Beam(cfg.n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV,
                      cfg.shape, cfg.nodes, tuning=tuning)
        bd.init(cfg.sigma_matrix, seed=cfg.seed, halo_frac=cfg.halo_frac)
        bd.track(cfg.lattice, args.warmup, diagnostics=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        diag = bd.track(cfg.lattice, args.steps, diagnostics=True)
        torch.cuda.synchronize()
        dtd = time.perf_counter() - t0
        variants["slice_step_diagnostics"] = {
            "value": cfg.n * args.steps / dtd, "ms_per_step": dtd / args.steps * 1e3,
            "note": "headline workload with the 27 moments recorded after every step",
            "last_step_rms_x_y": [float(diag[-1, 6] ** 0.5), float(diag[-1, 6 + 11] ** 0.5)]}
        bd.close()
        del bd, diag
        torch.cuda.empty_cache()
    if not args.no_shard:
        # one GPU's share of the headline over 8 GPUs: n/8 particles on the full 128^3 grid
        # (the sharded design replicates the grid work and all-reduces rho each step)
        cfg_s = cfg.with_(n=cfg.n // 8)
        bs, dts, sts, _ = run_gpu(cfg_s, args.steps, args.warmup, grid_fp32=False,
                                  tuning=tuning, binned=binned)
        st_s = {k: v[0] / max(v[1], 1) for k, v in sts.items()}
        grid_bytes = 8 * cfg.nodes[0] * cfg.nodes[1] * cfg.nodes[2]
        variants["one_gpu_share_of_8"] = {
            "value": cfg_s.n * args.steps / dts, "ms_per_step": dts / args.steps * 1e3,
            "particles": cfg_s.n, "stage_ms_per_launch": st_s,
            "gkd_GBs": ALGO_BYTES["gkd"] * cfg_s.n / (st_s["gkd"] * 1e-3) / 1e9,
            "deposit_GBs": ALGO_BYTES["deposit"] * cfg_s.n / (st_s["deposit"] * 1e-3) / 1e9,
            "rho_allreduce_bytes": grid_bytes,
            "note": "measured on one GPU: the per-GPU work of the particle-sharded design at 8 "
                    "GPUs (same grid, 1/8 of the particles); the all-reduce of rho is not run"}
        bs.close()
        del bs
        torch.cuda.empty_cache()
    if not args.no_direct:
        # the headline workload with E' from the integrated Green's functions of the field
        bf, dtf, stf, _ = run_gpu(cfg, args.steps, args.warmup, grid_fp32=False, tuning=tuning,
                                  direct_field=True, binned=binned)
        variants["direct_field"] = {
            "value": cfg.n * args.steps / dtf, "ms_per_step": dtf / args.steps * 1e3,
            "stage_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in stf.items()},
            "note": "headline workload; three field-kernel spectra and three convolutions "
                    "instead of the potential's, no differencing"}
        bf.close()
        del bf
        torch.cuda.empty_cache()
    if not args.no_fp32:
        variants["fp32_grid_accuracy"] = fp32_accuracy(workloads.MEDIUM, workloads.MEDIUM.steps)
    if not args.no_batched:
        variants["batched"] = run_batched(args.batch_beams, args.batch_steps,
                                          tune=not args.no_tune)
        torch.cuda.empty_cache()
        if not args.no_fp32:
            variants["batched_fp32_grid"] = run_batched(args.batch_beams, args.batch_steps,
                                                        grid_fp32=True, tune=not args.no_tune)
            torch.cuda.empty_cache()
    if not args.no_adjoint:
        variants["adjoint"] = run_adjoint(workloads.ADJOINT)
        torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": ps, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "device": device_info(),
        "config": {"workload": cfg.name, "particles": cfg.n, "grid": list(cfg.nodes),
                   "shape": "TSC" if cfg.shape == 2 else "CIC", "grid_dtype": "f64",
                   "halo_frac": cfg.halo_frac, "lattice": "thin FODO k=+-1/m, 0.5 m",
                   "particle_order": "binned between calls (pic_track_n_steps_binned), no "
                   "labels" if binned else "caller's order (pic_track_n_steps)"},
        "roofline": kernels[dominant],
        "autotune": tune_info,
        "kernels": kernels,
        "stage_ms_per_launch": stage_ms,
        "variants": variants,
    }
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
