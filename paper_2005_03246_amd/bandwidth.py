"""Bandwidth selection by leave-one-out likelihood cross-validation, with a
learned proposal.

Host orchestration only: every number comes from the library (exact LCV
scores of the Laplacian KDE, on-device features, the network's forward,
backward and Adam kernels).  The selected bandwidth is always the grid point
with the best exactly evaluated score in the window the proposal opened, so
the kernel values never depend on the network.
"""
from __future__ import annotations

import numpy as np
import torch

from . import datagen, mecdf


def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-style initial parameters (float32 vector in the C-ABI layout)."""
    g = np.random.default_rng(seed)
    w1 = g.normal(0.0, np.sqrt(2.0 / 32), (128, 32))
    w2 = g.normal(0.0, np.sqrt(2.0 / 128), (128, 128))
    w3 = g.normal(0.0, np.sqrt(1.0 / 128), 128) * 0.1
    p = np.concatenate([w1.ravel(), np.zeros(128), w2.ravel(), np.zeros(128), w3, [0.0]])
    assert p.size == mecdf.MLP_PARAMS
    return torch.tensor(p, dtype=torch.float32, device=device)


def to_device(sets):
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in sets]


def grid_search(dsets, hgrid):
    """Exact LCV at every grid bandwidth; returns (argmax index, score matrix)."""
    res = mecdf.kde_lcv_batched(dsets, [hgrid] * len(dsets))
    mat = torch.stack(res).cpu().numpy()
    return np.argmax(mat, axis=1), mat


def targets(feat, hidx, hgrid):
    """Network target: log of the grid optimum minus the rule-of-thumb log h0."""
    return torch.tensor(np.log(np.asarray(hgrid))[hidx], dtype=torch.float32,
                        device=feat.device) - feat[:, 12]


def train(dsets, hgrid, steps: int = 2000, lr: float = 1e-3, wd: float = 1.0, seed: int = 0,
          hidx=None):
    """Labels from the exact grid search, then full-batch Adam with decoupled
    weight decay on the device.  Returns (params, losses, labels)."""
    feat = mecdf.bw_features(dsets)
    if hidx is None:
        hidx, _ = grid_search(dsets, hgrid)
    t = targets(feat, hidx, hgrid)
    params = init_params(seed)
    adam = torch.zeros((2 * mecdf.MLP_PARAMS,), dtype=torch.float32, device="cuda")
    losses = mecdf.mlp_train(feat, t, params, adam, steps, lr, wd)
    return params, losses.cpu().numpy(), hidx


def select(dsets, params, hgrid, mode=mecdf.BW_EXTEND):
    return mecdf.bw_select(dsets, params, hgrid, mode)


def hgrid64():
    return datagen.bandwidths(64)
