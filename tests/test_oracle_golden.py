"""Golden pin from the paper's printed example: the FODO beam's 2 nm rms emittance."""
import json
import os

import numpy as np

from oracle import pic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fodo_listing_emittance.json")


def _exact_sample(sigma):
    """2n points +-sqrt(n) L e_k whose centred second moments equal sigma exactly."""
    n = sigma.shape[0]
    L = np.linalg.cholesky(sigma)
    pts = np.sqrt(n) * L
    return np.concatenate([pts, -pts], axis=1)


def test_listing_beam_has_the_printed_emittance():
    g = json.load(open(GOLDEN))
    S = np.zeros((6, 6))
    for (i, s, sp, mu) in ((0, g["sigmaX"], g["sigmaPx"], g["muxpx"]),
                           (2, g["sigmaY"], g["sigmaPy"], g["muypy"])):
        rx = s / np.sqrt(1 - mu ** 2)
        rp = sp / np.sqrt(1 - mu ** 2)
        S[i, i], S[i + 1, i + 1] = rx ** 2, rp ** 2
        S[i, i + 1] = S[i + 1, i] = -mu * rx * rp
    S[4, 4] = S[5, 5] = 1e-6
    X = _exact_sample(S)
    _, cov, m = pic.moments(X)
    assert np.allclose(cov, S, rtol=1e-12, atol=1e-30)
    eps_x, eps_y = m[2], m[3]
    # the paper prints one significant digit ("2 nm"); the parameters give it to 1e-9
    for e in (eps_x, eps_y):
        assert abs(e - g["printed_emittance_m"]) < 1e-9 * g["printed_emittance_m"]


def test_parameter_mapping_gives_the_printed_emittance():
    # oracle.pic.sigma_from_params on the Listing's numbers: the 2 nm emittance printed in the
    # text, rms sizes from the parameters, correlation -mu, and the Waterbag of that covariance
    g = json.load(open(GOLDEN))
    S = pic.sigma_from_params(g["sigmaX"], g["sigmaY"], 1.0e-3, g["sigmaPx"], g["sigmaPy"],
                              2.0e-3, g["muxpx"], g["muypy"], 0.0)
    for i, mu in ((0, g["muxpx"]), (2, g["muypy"])):
        eps = np.sqrt(np.linalg.det(S[i:i + 2, i:i + 2]))
        assert abs(eps - g["printed_emittance_m"]) < 1e-9 * g["printed_emittance_m"]
        rho = S[i, i + 1] / np.sqrt(S[i, i] * S[i + 1, i + 1])
        assert abs(rho + mu) < 1e-15
    assert S[4, 5] == 0.0 and S[4, 4] == 1e-6 and abs(S[5, 5] - 4e-6) < 1e-21
    # a Waterbag beam of that covariance: second moments within sampling error
    from oracle import rng
    n = 200_000
    X = pic.init_waterbag(S, rng.waterbag_xi(n, seed=9))
    _, cov, m = pic.moments(X)
    d = np.sqrt(np.diag(S))
    assert np.all(np.abs(cov - S) / np.outer(d, d) < 5.0 / np.sqrt(n))
    # inside the ellipsoid x^T S^-1 x <= 8
    q = np.einsum("in,ij,jn->n", X, np.linalg.inv(S), X)
    assert q.max() <= 8.0 * (1 + 1e-9)
    for bad in ((0.0, 1.0, 0.1), (1.0, 1.0, 1.0)):
        try:
            pic.sigma_from_params(bad[0], 1, 1, bad[1], 1, 1, bad[2], 0, 0)
            assert False
        except ValueError:
            pass
