"""torch.autograd.Function over the tracking: (Sigma0, k) -> (sigma_x, sigma_y, eps_x, eps_y).

The forward pass initialises X0 = L xi on the device (L = chol(Sigma0), from torch so that
torch's Cholesky backward carries dJ/dL to dJ/dSigma0) and runs pic_track_n_steps; the backward
pass re-initialises X0 and runs the library's reverse sweep (pic_track_adjoint), which returns
dJ/dk and dJ/dL = sum_i lam0_i xi_i^T: the gradient of the tracking itself, including the terms
through every step's grid geometry, which follows the particles' box.  Argument marshalling only: the tracking, the moments, the
objective terms (pic_objective) and both reductions run in the library's kernels.
"""
import torch

from . import Beam


class _Track(torch.autograd.Function):
    @staticmethod
    def forward(ctx, L, k, beam, xi, ds, n_steps, ckpt_every):
        sigma = (L @ L.T).detach().cpu()
        beam.init_from_normals(sigma, xi)
        beam.track([(float(kk), float(d)) for kk, d in zip(k.tolist(), ds)], n_steps)
        m = beam.objective()
        ctx.beam, ctx.xi, ctx.ds, ctx.n_steps, ctx.ck = beam, xi, ds, n_steps, ckpt_every
        ctx.save_for_backward(L, k)
        return torch.tensor(m, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gm):
        L, k = ctx.saved_tensors
        beam = ctx.beam
        beam.init_from_normals((L @ L.T).detach().cpu(), ctx.xi)
        lattice = [(float(kk), float(d)) for kk, d in zip(k.tolist(), ctx.ds)]
        _, dk, _, dL = beam.track_adjoint(lattice, ctx.n_steps, gm.tolist(), ctx.ck, xi=ctx.xi)
        gL = torch.tril(torch.tensor(dL, dtype=torch.float64))
        return gL, torch.tensor(dk, dtype=torch.float64), None, None, None, None, None


def track_moments(sigma0, k, beam: Beam, xi, ds, n_steps, ckpt_every=10):
    """Differentiable (sigma_x, sigma_y, eps_x, eps_y) after n_steps steps of the lattice
    (k_j, ds_j) from X0 = chol(sigma0) xi.  sigma0: (6, 6) float64 CPU tensor; k: (n_el,)
    float64 CPU tensor; xi: (6, n) float64 device tensor; ds: n_el drift lengths."""
    L = torch.linalg.cholesky(sigma0)
    return _Track.apply(L, k, beam, xi, list(ds), int(n_steps), int(ckpt_every))
