"""Seeded synthetic workloads shared by the oracle-side tests and the GPU-side tests and bench.

This module holds configuration data and random draws only -- none of the method's
arithmetic.  Both the oracle (``oracle/``) and the HIP path (``paper_2208_02382_amd``) take
their inputs from here; neither imports the other.

The beams stand in for the paper's workloads (its lattices and data artifact are not
available): electrons (mass 0.510998950 MeV and charge -e, as in Listing 1 of the paper) of
1 nC total charge, here at 20 MeV kinetic energy, with uncorrelated 6-D Gaussian phase space
(x, px, y, py, z, delta): sigma_x = sigma_y = 1 mm, sigma_px = sigma_py = sigma_delta = 1e-3
and sigma_z = 2 mm (small case) or 5 mm (others).  The lattice is a thin-lens FODO: every step
is a thin quadrupole of integrated strength +-1 /m followed by a 0.5 m space-charge drift.
"""
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

ELECTRON_MASS_MEV = 0.510998950


@dataclass(frozen=True)
class Beam:
    """One beam and its tracking problem."""
    name: str
    n: int                                   # macroparticles
    sigma: Tuple[float, ...]                 # rms of (x, px, y, py, z, delta)
    nodes: Tuple[int, int, int]              # grid nodes (nx, ny, nz)
    shape: int                               # B-spline order: 1 = CIC, 2 = TSC
    steps: int
    lattice: Tuple[Tuple[float, float], ...]  # per step (k [1/m], ds [m]), cycled
    seed: int
    halo_frac: float = 0.0                   # trailing fraction drawn uniform in [-4, 4]^6
    kin_energy_MeV: float = 20.0
    mass_MeV: float = ELECTRON_MASS_MEV
    charge_C: float = 1.0e-9
    charge_sign: float = -1.0

    @property
    def qm_qeeV(self):
        """Species charge over mass in e/eV (the paper's `qm_qeeV` argument)."""
        return self.charge_sign * 1.0e-6 / self.mass_MeV

    @property
    def sigma_matrix(self):
        """Initial 6x6 second-moment matrix (uncorrelated)."""
        return np.diag(np.asarray(self.sigma, dtype=np.float64) ** 2)

    def with_(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Beam(**d)


FODO = ((1.0, 0.5), (-1.0, 0.5))

# The paper's FODO cell of Listing 1 with thick elements: (kind, k [1/m^2], ds [m], nslice),
# kinds 1 = drift, 2 = quadrupole (0 is the thin-lens step of FODO above)
THICK_FODO = ((1, 0.0, 0.25, 25), (2, 1.0, 1.0, 25), (1, 0.0, 0.5, 25), (2, -1.0, 1.0, 25),
              (1, 0.0, 0.25, 25))

SMALL = Beam("gauss-1e4-32c-cic", 10_000, (1e-3, 1e-3, 1e-3, 1e-3, 2e-3, 1e-3),
             (32, 32, 32), 1, 20, FODO, seed=1)
MEDIUM = Beam("gauss-1e6-64c-cic", 1_000_000, (1e-3, 1e-3, 1e-3, 1e-3, 5e-3, 1e-3),
              (64, 64, 64), 1, 200, FODO, seed=2)
LARGE = Beam("gausshalo-1e8-128c-tsc", 100_000_000, (1e-3, 1e-3, 1e-3, 1e-3, 5e-3, 1e-3),
             (128, 128, 128), 2, 50, FODO, seed=3, halo_frac=0.1)
ADJOINT = Beam("gauss-1e6-64c-cic-8quads", 1_000_000, (1e-3, 1e-3, 1e-3, 1e-3, 5e-3, 1e-3),
               (64, 64, 64), 1, 100,
               tuple((1.0 if i % 2 == 0 else -1.0, 0.5) for i in range(8)), seed=5)

CONFIGS = {b.name: b for b in (SMALL, MEDIUM, LARGE, ADJOINT)}

BATCH_NAME = "batch-256-loguniform-1e4-1e6-cic"
BATCH_GRIDS = (32, 48, 64)


def batch_beams(n_beams=256, seed=4, n_range=(1e4, 1e6), grids=BATCH_GRIDS, k_range=(0.5, 2.0),
                steps=100):
    """Independent beams of the batched workload: particle counts round(10^U[log10 lo,
    log10 hi]), cubic grids drawn uniformly from `grids`, and a thin FODO of strength
    +-k_b with k_b ~ U[k_range] (0.5 m drifts).  The beam family is MEDIUM's (sigma_z 5 mm,
    CIC); beam b draws its coordinates with seed 1000 + b."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = np.log10(n_range[0]), np.log10(n_range[1])
    ns = np.rint(10.0 ** rng.uniform(lo, hi, n_beams)).astype(np.int64)
    gs = rng.integers(0, len(grids), n_beams)
    ks = rng.uniform(k_range[0], k_range[1], n_beams)
    out = []
    for b in range(n_beams):
        g = int(grids[gs[b]])
        k = float(ks[b])
        out.append(MEDIUM.with_(name="%s-b%d" % (BATCH_NAME, b), n=int(ns[b]), nodes=(g, g, g),
                                steps=steps, lattice=((k, 0.5), (-k, 0.5)), seed=1000 + b))
    return out


def n_halo(n, halo_frac):
    """Number of trailing halo particles."""
    return int(np.floor(halo_frac * n + 0.5))


def draw_xi(beam: Beam, n=None, seed=None):
    """Unit-free random draws xi, shape (6, n), float64, rows (x, px, y, py, z, delta).

    The first n - n_halo columns are standard normal, the trailing n_halo columns uniform in
    [-4, 4].  numpy's PCG64 generator, seeded with `seed` (default: the beam's seed).
    """
    n = beam.n if n is None else int(n)
    rng = np.random.Generator(np.random.PCG64(beam.seed if seed is None else seed))
    nh = n_halo(n, beam.halo_frac)
    xi = np.empty((6, n), dtype=np.float64)
    xi[:, : n - nh] = rng.standard_normal((6, n - nh))
    if nh:
        xi[:, n - nh:] = rng.uniform(-4.0, 4.0, (6, nh))
    return xi


def lattice_arrays(beam: Beam):
    """The lattice as two float64 arrays (k, ds)."""
    lat = np.asarray(beam.lattice, dtype=np.float64)
    return lat[:, 0].copy(), lat[:, 1].copy()
