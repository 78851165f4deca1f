"""Differentiation pattern (sfm-1m scene, render-proxy loss): gradients from
DipoleSum (GPU forward + two-stage GPU adjoint) against central finite
differences of the same loss evaluated with the FP64 oracle.

The sums are linear in the attributes, so perturbing mu_m,c by +-h changes f
by exactly +-h times the response to a one-hot attribute; that response is
evaluated in FP64 and the FD quotient is exact up to O(h^2) of the renderer.
"""
import math

import numpy as np
import pytest

import workloads
from workloads.render import fd_linear, fd_position, loss_numpy, loss_torch

pytestmark = pytest.mark.gpu

EPS = math.sqrt(2.0) * 0.01
BETA = 2.0
H = 1e-4        # position step
H_FIELD = 1e-3  # largest field change of an attribute step (Richardson-extrapolated)


def test_sfm_1m_autograd_matches_fd(orc):
    import torch
    import paper_2405_16788_amd as P
    P.load()
    p, n, A, mu = workloads.sfm_cloud(workloads.SFM_1M_SURFACE, workloads.SFM_1M_OUTLIERS, 10)
    R, S = 64, 128
    pix, x = workloads.pixel_ray_samples(workloads.sfm_camera(11), 512, 512, S, 12, R, 14)
    target = np.random.default_rng(13).uniform(size=(R, 3))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tree = P.dps_build(dev(p), dev(n), dev(A), dev(mu), leaf_size=16)
    attrs_t = dev(mu).requires_grad_(True)
    x_t = dev(x).requires_grad_(True)
    f, g = P.dipole_sum(attrs_t, x_t, tree, BETA, EPS)
    L = loss_torch(f.double(), R, S, dev(target))
    L.backward()
    ga = attrs_t.grad.cpu().numpy().astype(np.float64)
    gx = x_t.grad.cpu().numpy().astype(np.float64)

    T = orc.Tree(p, n, A, mu, 16)
    base = T.query(x, BETA, EPS)
    assert abs(L.item() - loss_numpy(base["f"], R, S, target)) <= 1e-4 * abs(L.item())
    # linearise the finite differences at the GPU forward values, so that the
    # comparison isolates the adjoint (the FP32 forward moves dL/df slightly)
    f0 = f.detach().cpu().numpy().astype(np.float64)
    L0 = loss_numpy(f0, R, S, target)
    # dL/df in FP64 for the error scales of the oracle adjoint
    f0t = torch.tensor(f0, dtype=torch.float64, requires_grad=True)
    loss_torch(f0t, R, S, torch.tensor(target)).backward()
    df64 = f0t.grad.numpy()
    adj = T.adjoint(x, BETA, EPS, df64.astype(np.float32))

    # attributes: 64 points x 4 channels
    pts = np.random.default_rng(15).choice(p.shape[0], 64, replace=False)
    worst = 0.0
    for m in pts:
        e = np.zeros_like(mu)
        e[m, :] = 1.0
        T.set_attrs(e)
        fe = T.query(x, BETA, EPS, want_grad=False)["f"]
        for c in range(mu.shape[1]):
            # the attribute step is scaled so the field moves by at most H:
            # a step of H on mu itself moves the FP64 loss of points far from
            # the rays by less than its rounding
            fd = fd_linear(f0, fe[:, c], c, lambda ff: loss_numpy(ff, R, S, target), H_FIELD)
            scale = adj["sdmu"][m, c] + 1e-12 * abs(L0)
            worst = max(worst, abs(ga[m, c] - fd) / scale)
    T.set_attrs(mu)
    print(f"[autograd] dattrs vs FD, max normalised error {worst:.3g}", flush=True)
    assert worst < 1e-5

    # sample positions: 64 samples x 3 coordinates, skipping samples whose
    # visited set changes within +-h (the Barnes-Hut sum is discontinuous there)
    qs = np.random.default_rng(16).choice(x.shape[0], 64, replace=False)
    worst, used = 0.0, 0
    for q in qs:
        for k in range(3):
            fd = fd_position(T, x, f0, base["counts"], q, k, S, target, H, BETA, EPS)
            if fd is None:
                continue
            scale = np.sum(np.abs(df64[q]) * base["sg"][q]) + 1e-12 * abs(L0)
            worst = max(worst, abs(gx[q, k] - fd) / scale)
            used += 1
    print(f"[autograd] dx vs FD on {used} coordinates, max normalised error {worst:.3g}", flush=True)
    assert used >= 96
    assert worst < 1e-4
    P.dps_destroy(tree)
