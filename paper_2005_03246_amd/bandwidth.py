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


def grid_search_device(dsets, hgrid):
    """Exact LCV at every grid bandwidth: (best index per dataset as an int32
    GPU tensor, the score rows as a list of GPU tensors)."""
    res, best = mecdf.kde_lcv_batched(dsets, [hgrid] * len(dsets), want_best=True)
    return best, res


def grid_search(dsets, hgrid):
    """Exact LCV at every grid bandwidth; returns (best index, score matrix)
    as numpy arrays copied from the library's outputs."""
    best, res = grid_search_device(dsets, hgrid)
    return best.cpu().numpy().astype(np.int64), torch.stack(res).cpu().numpy()


def train(dsets, hgrid, steps: int = 2000, lr: float = 1e-3, wd: float = 1.0, seed: int = 0,
          hidx=None, checkpoint=None):
    """Labels from the exact grid search (the library's device argmax), then
    full-batch Adam with decoupled weight decay, all in the library
    (mecdf_bw_train; with a checkpoint path, training resumes from the file
    and rewrites it).  Returns (params, losses, labels)."""
    feat = mecdf.bw_features(dsets)
    if hidx is None:
        label, _ = grid_search_device(dsets, hgrid)
    else:
        label = torch.as_tensor(np.asarray(hidx), dtype=torch.int32).cuda()
    params, _, losses, _ = mecdf.bw_train(feat, label, hgrid, steps, lr, wd, seed,
                                          checkpoint=checkpoint)
    return params, losses.cpu().numpy(), label.cpu().numpy().astype(np.int64)


def select(dsets, params, hgrid, mode=mecdf.BW_EXTEND):
    return mecdf.bw_select(dsets, params, hgrid, mode)


def hgrid64():
    return datagen.bandwidths(64)
