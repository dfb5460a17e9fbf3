"""Write tests/golden/gauss-1e6-64c-cic_oracle.json: the oracle's tracking of the workload
gauss-1e6-64c-cic (1e6 particles of the seeded Gaussian beam, 64^3 nodes, CIC, the thin FODO,
200 steps) from the seeded host draws, recorded every 10 steps as the 6 means, the 6x6 centred
second moments and (sigma_x, sigma_y, eps_x, eps_y), plus the final coordinates of 256 sampled
particles.

Calls only oracle/ and the seeded input generators of workloads.py.  About 20 minutes of one
CPU core.  Usage: python tests/golden/gen_medium_oracle.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import pic as opic  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gauss-1e6-64c-cic_oracle.json")
RECORD_EVERY = 10
N_SAMPLE = 256
SAMPLE_SEED = 17


def main():
    cfg = workloads.MEDIUM
    prob = opic.make_problem(cfg.n, cfg.qm_qeeV, cfg.charge_C, cfg.kin_energy_MeV,
                             cfg.mass_MeV, cfg.nodes, cfg.shape)
    ks, dss = workloads.lattice_arrays(cfg)
    X = opic.init_from_normals(cfg.sigma_matrix, workloads.draw_xi(cfg))
    rec = {}
    t0 = time.time()
    for j in range(cfg.steps):
        X = opic.step(X, ks[j % len(ks)], dss[j % len(ks)], prob)
        if (j + 1) % RECORD_EVERY == 0:
            mean, cov, m = opic.moments(X)
            rec[str(j + 1)] = {"mean": mean.tolist(), "cov": cov.tolist(), "objective": m.tolist()}
            print("step %d  %.0f s  sigma_x %.9e" % (j + 1, time.time() - t0, m[0]), flush=True)
    S = np.sort(np.random.default_rng(SAMPLE_SEED).choice(cfg.n, N_SAMPLE, replace=False))
    out = {
        "workload": cfg.name, "particles": cfg.n, "nodes": list(cfg.nodes), "shape": "CIC",
        "steps": cfg.steps, "record_every": RECORD_EVERY,
        "initial_state": "workloads.draw_xi(MEDIUM) through oracle.pic.init_from_normals",
        "written_by": "tests/golden/gen_medium_oracle.py (oracle/ only)",
        "moments": rec,
        "sample_index": S.tolist(),
        "sample_final": X[:, S].tolist(),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
