"""Pins of the oracle's thick elements and sliced tracking (the paper's Drift / Quad elements)
against the paper's FODO benchmark: its printed phase advance, the rms-matched beam of its
Listing 1, and closed-form properties of the quadrupole map."""
import json
import os

import numpy as np

from oracle import pic

HERE = os.path.dirname(__file__)
CELL = json.load(open(os.path.join(HERE, "golden", "fodo_thick_cell.json")))
BEAM = json.load(open(os.path.join(HERE, "golden", "fodo_listing_emittance.json")))


def _cell_matrix(plane_sign):
    M = np.eye(2)
    for kind, k, ds, _ in CELL["lattice"]:
        M = pic.quad_matrix(plane_sign * k if kind == pic.QUAD else 0.0, ds) @ M
    return M


def _twiss(M):
    mu = np.arccos(0.5 * np.trace(M))
    return np.degrees(mu), M[0, 1] / np.sin(mu), (M[0, 0] - M[1, 1]) / (2 * np.sin(mu))


def _listing_sigma():
    # the Listing's Waterbag parameters (sigmaT = 1e-3, sigmaPt = 2e-3, mutpt = 0 as printed)
    return pic.sigma_from_params(BEAM["sigmaX"], BEAM["sigmaY"], 1.0e-3, BEAM["sigmaPx"],
                                 BEAM["sigmaPy"], 2.0e-3, BEAM["muxpx"], BEAM["muypy"], 0.0)


def _problem():
    return pic.make_problem(1, -1e-6 / CELL["mass_MeV"], 0.0, CELL["energy_MeV"],
                            CELL["mass_MeV"], (8, 8, 8), 2)


def test_phase_advance_matches_the_printed_value():
    for sign in (1.0, -1.0):
        mu, _, _ = _twiss(_cell_matrix(sign))
        assert abs(mu - CELL["printed_phase_advance_deg"]) < 0.05


def test_matched_twiss_equals_the_listing_beam():
    # the Waterbag parameters of Listing 1 describe the beam matched to this lattice: its
    # beta = <x^2>/eps and alpha = -<x px>/eps equal the cell's periodic Twiss functions
    S = _listing_sigma()
    for i, sign in ((0, 1.0), (2, -1.0)):
        eps = np.sqrt(S[i, i] * S[i + 1, i + 1] - S[i, i + 1] ** 2)
        _, beta, alpha = _twiss(_cell_matrix(sign))
        assert abs(S[i, i] / eps - beta) < 1e-8 * beta
        assert abs(-S[i, i + 1] / eps - alpha) < 1e-8 * abs(alpha)


def test_matched_beam_keeps_its_second_moments_through_a_sliced_cell():
    S = _listing_sigma()
    L = np.linalg.cholesky(S)
    pts = np.sqrt(6) * L
    X = np.concatenate([pts, -pts], axis=1)       # centred second moments exactly S
    Y = pic.track_elements(X, CELL["lattice"], 125, _problem(), space_charge=False)
    _, cov, _ = pic.moments(Y)
    # Listing 1 prints the Waterbag parameters to 11 significant digits, and the beam they
    # describe is matched to the cell to about 1e-8 (previous test): the moments return to
    # themselves within that precision
    T = np.ix_([0, 1, 2, 3], [0, 1, 2, 3])
    assert np.abs(cov[T] - S[T]).max() < 2e-8 * np.abs(S[T]).max()


def test_quad_matrix_closed_forms():
    rng = np.random.default_rng(3)
    for k in (1.7, -0.6, 0.0):
        s1, s2 = rng.uniform(0.05, 0.9, 2)
        M1, M2 = pic.quad_matrix(k, s1), pic.quad_matrix(k, s2)
        assert abs(np.linalg.det(M1) - 1) < 1e-14                     # symplectic
        assert np.allclose(M2 @ M1, pic.quad_matrix(k, s1 + s2), rtol=1e-13, atol=1e-14)
    # short-element limit: strength K/s over length s -> thin quad K plus a drift s
    K, s = 0.8, 1e-5
    M = pic.quad_matrix(K / s, s)
    thin = np.array([[1.0, 0.0], [-K, 1.0]])
    assert np.abs(M - np.array([[1.0, s], [0.0, 1.0]]) @ thin).max() < 5 * K * s


def test_slicing_does_not_change_the_zero_current_map():
    X = np.random.default_rng(4).standard_normal((6, 50)) * 1e-3
    one = [[kind, k, ds, 1] for kind, k, ds, _ in CELL["lattice"]]
    Y1 = pic.track_elements(X, one, 5, _problem(), space_charge=False)
    Y25 = pic.track_elements(X, CELL["lattice"], 125, _problem(), space_charge=False)
    assert np.abs(Y25 - Y1).max() < 1e-15 * 50 + 1e-14 * np.abs(Y1).max()
