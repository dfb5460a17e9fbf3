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
