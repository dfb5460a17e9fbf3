"""The cold, uniformly charged ellipsoid of test_oracle_envelope.py tracked by the library:
equal to the oracle within 1e-12 of each coordinate's rms (both field paths), and its rms sizes
grow by the factors of the envelope equations integrated independently with scipy (bar 2 %).
"""
import numpy as np
import pytest
import torch

import test_oracle_envelope as env
from oracle import pic as opic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2208_02382_amd as p
    return p


@pytest.mark.parametrize("direct_field", [False, True])
def test_cold_uniform_ellipsoid_on_the_gpu(lib, direct_field):
    qm, charge, ke, mass = -1.0 / 0.51099895e6, 1e-9, 20.0, 0.51099895
    X0 = env._cold_uniform_ellipsoid(env.N, seed=3)
    b = lib.Beam(env.N, qm, charge, ke, mass, 2, env.NODES, direct_field=direct_field)
    b.X.copy_(torch.from_numpy(X0))
    b.track([(0.0, env.LENGTH / env.STEPS)], env.STEPS)
    torch.cuda.synchronize()
    assert b.check() == lib.PIC_OK
    Xg = b.X.cpu().numpy()
    prob = opic.make_problem(env.N, qm, charge, ke, mass, env.NODES, 2, direct_field=direct_field)
    Xo = opic.track(X0, [0.0], [env.LENGTH / env.STEPS], env.STEPS, prob)
    assert (np.abs(Xg - Xo).max(axis=1) / Xo.std(axis=1)).max() < 1e-12
    c0, c = np.cov(X0, bias=True), np.cov(Xg, bias=True)
    grown = np.sqrt(np.diag(c)[[0, 2, 4]] / np.diag(c0)[[0, 2, 4]])
    ratio = env._envelope(prob, -charge)  # the configured bunch charge, electron sign
    assert np.all(np.abs((grown - 1.0) / (ratio - 1.0) - 1.0) < 0.02), (grown, ratio)
