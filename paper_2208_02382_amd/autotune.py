"""Autotuner of the binned deposit and gather: tile edge, particles per work item, workgroup
count and size (pic_beam_desc.tile / chunk / blocks / threads), and the workgroups per beam of
a batch.

Each candidate is timed on the device with the library's own tracking loop
(pic_track_n_steps_binned in steady state: after a one-step call has moved the particles into
tile order, the wall time of a call less its once-per-call stages; pic_track_batch for a batch:
the whole call) over a few steps of a beam of the problem's size, re-initialised to the same
seeded state before every candidate.  The search is
coordinate-wise: tile shape with the default work items, then the work-item size at the best
tile, then the workgroup count, then the workgroup size.  Tile shapes are cubes and slabs: a
slab is thin along one axis and wide along the other two, so that particles moving mostly
across the wide axes (the transverse planes of a focusing lattice, where the longitudinal
position hardly changes within a step) leave their tile less often, and the gather reads fewer
of them from outside the tile's own stretch of the previous order.  Only launch shapes within the
library's documented limits are tried (tile count <= 4096, the gather's
field window within the 156 KB of dynamic LDS a workgroup may use).  Results go into a JSON
cache keyed by problem class: particle count rounded to a power of two, grid, shape and
grid precision.  Results depend on the tuning only through the rounding of the deposit's
fixed-point contributions, whose scale each tile takes from its own particle count.
"""
import json
import math
import os
import time

import torch

from . import Batch, Beam, PIC_OK, STATUS_NAMES

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
TILES = (4, 5, 6, 8, 10, 12, 16)
# slabs (wide, wide, thin), with the thin axis put on each of x, y and z in turn
SLABS = ((24, 24, 2), (32, 16, 2), (16, 32, 2), (32, 32, 2), (16, 16, 4), (20, 20, 4),
         (24, 24, 4), (32, 32, 1))
CHUNKS = (2048, 4096, 8192, 16384, 32768)
BLOCKS = (0, 1024, 2048, 8192)          # 0: min(work items, 4096)
THREADS = (256, 512, 1024)
DEPOSIT_THREADS = (0, 128, 256, 512, 1024)  # 0: that of `threads`
FIELDS = ("tile", "chunk", "blocks", "threads", "deposit_threads")
LDS_BYTES = 163840 - 4096               # dynamic LDS one workgroup may allocate
BATCH_BLOCKS = (32, 64, 128, 256, 512)
BATCH_TILES = (8, 12, 16)                # one tile edge for every beam of a batch


def key(n, nodes, shape, grid_fp32):
    return "n2^%d-%dx%dx%d-%s-%s" % (round(math.log2(max(int(n), 1))), *nodes,
                                     "tsc" if shape == 2 else "cic",
                                     "f32" if grid_fp32 else "f64")


def load(cache=DEFAULT_CACHE):
    if cache and os.path.exists(cache):
        with open(cache) as f:
            return json.load(f)
    return {}


def save(table, cache=DEFAULT_CACHE):
    tmp = cache + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, cache)


def lookup(n, nodes, shape, grid_fp32, cache=DEFAULT_CACHE):
    """The cached tuning dict (tile, chunk, blocks, threads, deposit_threads) of this problem
    class, or None."""
    rec = load(cache).get(key(n, nodes, shape, grid_fp32))
    return None if rec is None else {k: rec[k] for k in FIELDS if k in rec}


def _tile_ok(tile, nodes, shape, grid_fp32):
    es = 4 if grid_fp32 else 8
    ntiles = 1
    win = 3 * es
    for t, n in zip(tile, nodes):
        ntiles *= -(-n // t)
        win *= t + shape
    return ntiles <= 4096 and win <= LDS_BYTES


# stages that run once per call, alone on the caller's stream
CALL_STAGES = ("prologue", "unpermute")


def _time_single(cfg, tuning, grid_fp32, steps, X):
    """Mean time of one steady-state step over `steps` steps: a binned call of one step moves
    the particles into tile order, then a binned call of `steps` steps (every step only ranks)
    is timed, less its once-per-call stages (timed by the library's HIP events).  Stage times
    are not summed, because the Green spectrum overlaps the binning and deposit."""
    b = Beam(cfg.n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV, cfg.mass_MeV, cfg.shape,
             cfg.nodes, grid_fp32=grid_fp32, X=X, tuning=tuning)
    try:
        b.init(cfg.sigma_matrix, seed=cfg.seed, halo_frac=cfg.halo_frac)
        b.track(cfg.lattice, 1, binned=True)
        torch.cuda.synchronize()
        b.profile_start()
        t0 = time.perf_counter()
        b.track(cfg.lattice, steps, binned=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stages = b.profile_read()
        dt = (wall - sum(stages[k][0] for k in CALL_STAGES) / 1e3) / steps
        st = b.check()
        if st != PIC_OK:
            raise RuntimeError("device error during tuning: %s" % STATUS_NAMES.get(st, st))
        return dt
    finally:
        b.close()


def tune(cfg, grid_fp32=False, steps=6, cache=DEFAULT_CACHE, force=False, log=None):
    """Tune one problem class (cfg: n, nodes, shape, sigma_matrix, seed, halo_frac, lattice,
    species fields); returns the cache record {tile, chunk, blocks, s_per_step,
    default_s_per_step, tried}."""
    k = key(cfg.n, cfg.nodes, cfg.shape, grid_fp32)
    table = load(cache) if cache else {}
    if not force and k in table:
        return table[k]
    X = torch.empty((6, cfg.n), dtype=torch.float64, device="cuda")
    tried = []

    def run(tuning):
        dt = _time_single(cfg, tuning, grid_fp32, steps, X)
        tried.append({"tuning": tuning, "s_per_step": dt})
        if log:
            log("tune %s %s: %.3f ms/step" % (k, tuning, dt * 1e3))
        return dt

    default = run({})
    best, best_t = {}, default
    shapes = [(t, t, t) for t in TILES]
    for thin in (2, 1, 0):
        for sl in SLABS:
            wide = list(sl[:2])
            shapes.append(tuple(sl[2] if a == thin else wide.pop(0) for a in range(3)))
    seen = set()
    for shp in shapes:
        tile = [min(t, n) for t, n in zip(shp, cfg.nodes)]
        if tuple(tile) in seen or not _tile_ok(tile, cfg.nodes, cfg.shape, grid_fp32):
            continue
        seen.add(tuple(tile))
        cand = {"tile": tile}
        dt = run(cand)
        if dt < best_t:
            best, best_t = cand, dt
    for c in CHUNKS:
        cand = dict(best, chunk=c)
        dt = run(cand)
        if dt < best_t:
            best, best_t = cand, dt
    for bl in BLOCKS[1:]:
        cand = dict(best, blocks=bl)
        dt = run(cand)
        if dt < best_t:
            best, best_t = cand, dt
    for th in THREADS[1:]:
        cand = dict(best, threads=th)
        dt = run(cand)
        if dt < best_t:
            best, best_t = cand, dt
    # the deposit's workgroup size apart from the gather's (the two kernels' best sizes differ)
    for th in DEPOSIT_THREADS[1:]:
        if th == best.get("threads", THREADS[0]):
            continue
        cand = dict(best, deposit_threads=th)
        dt = run(cand)
        if dt < best_t:
            best, best_t = cand, dt
    del X
    rec = {"tile": list(best.get("tile", (0, 0, 0))), "chunk": int(best.get("chunk", 0)),
           "blocks": int(best.get("blocks", 0)), "threads": int(best.get("threads", 0)),
           "deposit_threads": int(best.get("deposit_threads", 0)),
           "s_per_step": best_t,
           "default_s_per_step": default, "steps_timed": steps, "tried": tried}
    if cache:
        table = load(cache)
        table[k] = rec
        save(table, cache)
    return rec


def batch_tuning(c, rec, grid_fp32, cache=DEFAULT_CACHE):
    """The launch tuning of one beam of a tuned batch: the batch-wide tile edge of the record
    where the tuner chose one, else the cached tuning of the beam's class (or None)."""
    if rec and any(rec.get("tile", (0, 0, 0))):
        return {"tile": list(rec["tile"])}
    return lookup(c.n, c.nodes, c.shape, grid_fp32, cache) if cache else None


def tune_batch(cfgs, grid_fp32=False, steps=10, cache=DEFAULT_CACHE, force=False, log=None):
    """Workgroups per beam of the batched deposit and gather, then one tile edge for every
    beam (BATCH_TILES, against the beams' own tuning or default), timed on the batch itself
    (every beam re-initialised before each candidate).  Returns {blocks_per_beam, tile,
    s_per_step, tried}; tile [0, 0, 0]: each beam keeps its class's cached tuning or the
    default."""
    k = "batch-%d-beams-n%d-%s-%s" % (len(cfgs), sum(c.n for c in cfgs),
                                      "tsc" if cfgs[0].shape == 2 else "cic",
                                      "f32" if grid_fp32 else "f64")
    table = load(cache) if cache else {}
    if not force and k in table:
        return table[k]
    tried = []

    def run(bl, tile):
        trec = {"tile": tile} if tile else None
        beams = [Beam(c.n, c.qm_qeeV, c.charge_C, c.kin_energy_MeV, c.mass_MeV, c.shape,
                      c.nodes, grid_fp32=grid_fp32,
                      tuning=batch_tuning(c, trec, grid_fp32, cache))
                 for c in cfgs]
        try:
            batch = Batch(beams, [c.lattice for c in cfgs], blocks_per_beam=bl)
            for c, b in zip(cfgs, beams):
                b.init(c.sigma_matrix, seed=c.seed)
            batch.track(steps)  # capture
            torch.cuda.synchronize()
            for c, b in zip(cfgs, beams):
                b.init(c.sigma_matrix, seed=c.seed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            batch.track(steps)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            batch.close()
        finally:
            for b in beams:
                b.close()
        tried.append({"blocks_per_beam": bl, "tile": tile or [0, 0, 0], "s_per_step": dt})
        if log:
            log("tune %s blocks_per_beam=%d tile=%s: %.3f ms/step" % (k, bl, tile, dt * 1e3))
        return dt

    best_bl, best_tile, best_t = None, None, float("inf")
    for bl in BATCH_BLOCKS:
        dt = run(bl, None)
        if dt < best_t:
            best_bl, best_t = bl, dt
    for t in BATCH_TILES:
        tile = [t, t, t]
        if not all(_tile_ok(tile, c.nodes, c.shape, grid_fp32) for c in cfgs):
            continue
        dt = run(best_bl, tile)
        if dt < best_t:
            best_tile, best_t = tile, dt
    rec = {"blocks_per_beam": best_bl, "tile": best_tile or [0, 0, 0], "s_per_step": best_t,
           "steps_timed": steps, "tried": tried}
    if cache:
        table = load(cache)
        table[k] = rec
        save(table, cache)
    return rec
