"""Bandwidth selection on the GPU: features, the network's forward and
gradient against the float64 reference, training, the batched LCV scores
against the oracle, and the learned selection against the full grid search."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp
from paper_2005_03246_amd import bandwidth, datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2005_03246_amd import mecdf

    return mecdf


def test_features_match_numpy(lib):
    sets = datagen.config5(count=6, log2n_lo=9, log2n_hi=12, seed=11)
    feat = lib.bw_features(bandwidth.to_device(sets)).cpu().numpy()
    for i, x in enumerate(sets):
        d, n = x.shape
        m = x.mean(1)
        sd = x.std(1)
        c = x - m[:, None]
        f = feat[i]
        np.testing.assert_allclose(f[0], np.log(n) / 10, rtol=1e-6)
        np.testing.assert_allclose(f[1], d / 3, rtol=1e-6)
        np.testing.assert_allclose(f[2:2 + d], np.log(sd), rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(f[5:5 + d], (c ** 3).mean(1) / sd ** 3, rtol=1e-4, atol=1e-5)
        np.testing.assert_allclose(f[8:8 + d], ((c ** 4).mean(1) / sd ** 4 - 3) / 10,
                                   rtol=1e-4, atol=1e-5)
        lg = np.log(sd).mean()
        np.testing.assert_allclose(f[12], lg - np.log(n) / (d + 4), rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(f[14:14 + d], np.abs(c).mean(1) / sd, rtol=1e-5)
        np.testing.assert_allclose(f[17:17 + d], (np.abs(c) <= 0.5 * sd[:, None]).mean(1),
                                   rtol=1e-6, atol=1e-6)
        for k in range(d):
            a = np.abs(c[k]) / sd[k]
            np.testing.assert_allclose(f[20 + 3 * k:23 + 3 * k],
                                       [np.mean(a <= 0.25), np.mean(a <= 1.0), np.mean(a <= 2.0)],
                                       rtol=1e-6, atol=1e-6)
        assert np.all(f[20 + 3 * d:] == 0)


def _rand_problem(B, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(B, 32)).astype(np.float32)
    T = g.normal(size=B).astype(np.float32)
    p = bandwidth.init_params(seed).cpu().numpy().astype(np.float64)
    p[omlp.OW3:omlp.OB3] = g.normal(0, 0.3, 128)   # non-trivial last layer
    p[omlp.OB1:omlp.OW2] = g.normal(0, 0.1, 128)
    return X, T, p.astype(np.float32)


@pytest.mark.parametrize("B", [1, 16, 37, 300])
def test_mlp_forward_and_grad_vs_reference(lib, B):
    X, T, p = _rand_problem(B, 3 + B)
    Xt, Tt, pt = (torch.from_numpy(a).cuda() for a in (X, T, p))
    out = lib.mlp_forward(Xt, pt).cpu().numpy()
    ref, _ = omlp.forward(X.astype(np.float64), p.astype(np.float64), emulate=True)
    exact, _ = omlp.forward(X.astype(np.float64), p.astype(np.float64), emulate=False)
    scale = np.max(np.abs(ref)) + 1e-6
    assert np.max(np.abs(out - ref)) <= 1e-2 * scale
    assert np.median(np.abs(out - ref)) <= 1e-5 * scale
    assert np.max(np.abs(out - exact)) <= 3e-2 * scale
    G, loss = lib.mlp_grad(Xt, Tt, pt)
    G = G.cpu().numpy()
    Gr, Lr = omlp.grad(X.astype(np.float64), T.astype(np.float64), p.astype(np.float64),
                       emulate=True)
    assert abs(float(loss.cpu()) - Lr) <= 1e-3 * max(Lr, 1e-6)
    Gx, _ = omlp.grad(X.astype(np.float64), T.astype(np.float64), p.astype(np.float64),
                      emulate=False)
    blocks = [(omlp.OW1, omlp.OB1), (omlp.OB1, omlp.OW2), (omlp.OW2, omlp.OB2),
              (omlp.OB2, omlp.OW3), (omlp.OW3, omlp.OB3), (omlp.OB3, omlp.NPARAMS)]
    loose_exact = []
    for a, b in blocks:
        s = np.max(np.abs(Gr[a:b])) + 1e-12
        err = np.abs(G[a:b] - Gr[a:b]) / s
        # most entries differ from the bf16-emulating reference only by the
        # float32 accumulation order; an activation whose bf16 rounding falls
        # the other way (an accumulation error straddling a rounding boundary)
        # moves the entries it feeds by up to a bf16 step, hence the loose max
        assert np.max(err) <= 2e-2, (a, b)
        assert np.quantile(err, 0.99) <= 1e-4, (a, b)
        loose_exact.append(np.quantile(np.abs(Gx[a:b] - Gr[a:b]) / s, 0.99))
    # the bound above separates the emulation from plain float64: without
    # the bf16 roundings the reference gradient misses it in the weight blocks
    assert max(loose_exact[0], loose_exact[2]) > 1e-4


def test_training_reduces_loss(lib):
    g = np.random.default_rng(5)
    X = g.normal(size=(512, 32)).astype(np.float32)
    T = (np.tanh(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3).astype(np.float32)
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    p = bandwidth.init_params(1)
    adam = torch.zeros((2 * lib.MLP_PARAMS,), dtype=torch.float32, device="cuda")
    losses = lib.mlp_train(Xt, Tt, p, adam, 400, 2e-3).cpu().numpy()
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.2 * losses[0]
    # the trained parameters keep the low loss
    _, l_now = lib.mlp_grad(Xt, Tt, p)
    assert float(l_now.cpu()) < 0.2 * losses[0]


def test_adamw_first_step(lib):
    """One step from a zero state: the bias-corrected moments are g and g^2,
    so the update is p - lr (g / (|g| + eps) + wd p)."""
    X, T, p = _rand_problem(40, 8)
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    p0 = torch.from_numpy(p).cuda()
    G, _ = lib.mlp_grad(Xt, Tt, p0)
    g = G.cpu().numpy().astype(np.float64)
    lr, wd = 1e-3, 0.7
    p1 = p0.clone()
    adam = torch.zeros((2 * lib.MLP_PARAMS,), dtype=torch.float32, device="cuda")
    lib.mlp_train(Xt, Tt, p1, adam, 1, lr, wd)
    want = p.astype(np.float64) - lr * (g / (np.abs(g) + 1e-8) + wd * p.astype(np.float64))
    np.testing.assert_allclose(p1.cpu().numpy(), want, rtol=1e-5, atol=1e-7)


def test_lcv_batched_matches_oracle(lib):
    sets = datagen.config5(count=5, log2n_lo=8, log2n_hi=10, seed=21)
    hs = [[0.05, 0.2], [0.1], [0.03, 0.3, 1.0], [0.5], [0.2, 0.4]]
    got = lib.kde_lcv_batched(bandwidth.to_device(sets), hs)
    for x, h, r in zip(sets, hs, got):
        ref = oracle.lcv(x, np.asarray(h))
        assert np.allclose(r.cpu().numpy(), ref, rtol=1e-12, atol=1e-12)


def test_learned_selection_vs_grid_search(lib):
    """Train on separately seeded datasets, then select on others: every
    returned score is exact, each choice is a local maximum of the grid
    scores, and the mean LCV gap to the grid optimum is within log(1/0.99)."""
    hgrid = bandwidth.hgrid64()
    train = bandwidth.to_device(datagen.config5(count=160, log2n_lo=9, log2n_hi=12, seed=99))
    params, losses, _ = bandwidth.train(train, hgrid, steps=1500, lr=2e-3)
    assert losses[-1] < losses[0]
    test = bandwidth.to_device(datagen.config5(count=40, log2n_lo=9, log2n_hi=12, seed=7))
    gidx, mat = bandwidth.grid_search(test, hgrid)
    hidx, lcv, evals = bandwidth.select(test, params, hgrid)
    rows = np.arange(len(test))
    np.testing.assert_allclose(lcv, mat[rows, hidx], rtol=1e-12, atol=1e-12)
    for i in rows:
        j = hidx[i]
        if j > 0:
            assert mat[i, j] >= mat[i, j - 1]
        if j < len(hgrid) - 1:
            assert mat[i, j] >= mat[i, j + 1]
    gap = mat[rows, gidx] - lcv
    assert np.all(gap >= -1e-12)
    assert gap.mean() <= np.log(1 / 0.99)
    assert evals.mean() < 16
    # the single-window mode: four exact evaluations around the same proposal
    widx, wlcv, wev = bandwidth.select(test, params, hgrid, lib.BW_WINDOW)
    np.testing.assert_allclose(wlcv, mat[rows, widx], rtol=1e-12, atol=1e-12)
    assert np.all(wev == 4)
    # the extension only adds evaluations, so its choice is at least as good
    assert np.all(lcv >= wlcv - 1e-12)
    # what the network adds: the same four-point window opened at the
    # rule-of-thumb bandwidth alone (network output 0) lands further from the
    # grid optimum, on average and in the share of datasets within 1 %
    zero = torch.zeros_like(params)
    ridx, rlcv, _ = bandwidth.select(test, zero, hgrid, lib.BW_WINDOW)
    lim = np.log(1 / 0.99)
    gap_learned = mat[rows, gidx] - wlcv
    gap_rot = mat[rows, gidx] - rlcv
    assert gap_learned.mean() < gap_rot.mean()
    assert np.mean(gap_learned <= lim) >= np.mean(gap_rot <= lim)


def test_batched_best_index_is_the_argmax(lib):
    sets = datagen.config5(count=7, log2n_lo=8, log2n_hi=10, seed=23)
    hs = [bandwidth.hgrid64()[::3]] * 6 + [[0.3]]
    rows, best = lib.kde_lcv_batched(bandwidth.to_device(sets), hs, want_best=True)
    best = best.cpu().numpy()
    for r, b in zip(rows, best):
        r = r.cpu().numpy()
        assert b == int(np.argmax(r))


def test_bw_train_from_seed_and_checkpoint_resume(lib, tmp_path):
    """Training through the C ABI: fresh parameters come from the seed alone;
    60 steps in one call equal 25 steps written to a checkpoint and 35 more
    resumed from it, bit for bit (parameters, moments and losses); the first
    loss is the network's loss on the targets log h[label] - log h0."""
    hgrid = bandwidth.hgrid64()
    dsets = bandwidth.to_device(datagen.config5(count=48, log2n_lo=9, log2n_hi=11, seed=31))
    feat = lib.bw_features(dsets)
    label, _ = bandwidth.grid_search_device(dsets, hgrid)
    p0, a0, _, n0 = lib.bw_train(feat, label, hgrid, 0, 1e-3, 0.5, seed=9)
    q0, _, _, _ = lib.bw_train(feat, label, hgrid, 0, 1e-3, 0.5, seed=9)
    r0, _, _, _ = lib.bw_train(feat, label, hgrid, 0, 1e-3, 0.5, seed=10)
    assert n0 == 0 and torch.equal(p0, q0) and not torch.equal(p0, r0)
    assert torch.all(a0 == 0)
    w1 = p0[omlp.OW1:omlp.OB1].cpu().numpy()
    assert abs(w1.std() / np.sqrt(2.0 / 32) - 1) < 0.05
    assert torch.all(p0[omlp.OB1:omlp.OW2] == 0) and float(p0[omlp.OB3]) == 0.0
    # the targets the library forms on the device
    t = (np.log(hgrid)[label.cpu().numpy()] - feat[:, 12].cpu().numpy().astype(np.float64))
    _, l_ref = lib.mlp_grad(feat, torch.from_numpy(t.astype(np.float32)).cuda(), p0)

    pf, af, lf, nf = lib.bw_train(feat, label, hgrid, 60, 2e-3, 0.5, seed=9)
    assert nf == 60
    assert float(lf[0]) == pytest.approx(float(l_ref), rel=1e-6)
    assert float(lf[-1]) < float(lf[0])
    ck = str(tmp_path / "bw.ckpt")
    _, _, l1, n1 = lib.bw_train(feat, label, hgrid, 25, 2e-3, 0.5, seed=9, checkpoint=ck)
    assert n1 == 25
    p2, a2, l2, n2 = lib.bw_train(feat, label, hgrid, 35, 2e-3, 0.5, seed=9, checkpoint=ck)
    assert n2 == 60
    assert torch.equal(p2, pf) and torch.equal(a2, af)
    assert torch.equal(torch.cat([l1, l2]), lf)
    # resuming from memory (no file) continues the same way
    p3, a3, _, n3 = lib.bw_train(feat, label, hgrid, 25, 2e-3, 0.5, seed=9)
    p3, a3, _, n3 = lib.bw_train(feat, label, hgrid, 35, 2e-3, 0.5, seed=9, params=p3,
                                 adam=a3, step=n3)
    assert n3 == 60 and torch.equal(p3, pf)
    # a checkpoint of another seed, or a damaged one, is refused
    with pytest.raises(lib.MecdfError) as e:
        lib.bw_train(feat, label, hgrid, 1, 2e-3, 0.5, seed=8, checkpoint=ck)
    assert e.value.code == lib.MECDF_EINVAL
    raw = bytearray(open(ck, "rb").read())
    raw[100] ^= 0xFF
    bad = str(tmp_path / "bad.ckpt")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(lib.MecdfError) as e:
        lib.bw_train(feat, label, hgrid, 1, 2e-3, 0.5, seed=9, checkpoint=bad)
    assert e.value.code == lib.MECDF_EIO
    # labels outside the grid are refused
    with pytest.raises(lib.MecdfError) as e:
        lib.bw_train(feat, label + 64, hgrid, 1, 2e-3, 0.5, seed=9)
    assert e.value.code == lib.MECDF_EINVAL


def _mixed_sets(qn, rn, seed):
    """Datasets on both sides of the queue sizes qn / rn per dimension, with
    bandwidth lists of different lengths (one empty)."""
    g = np.random.default_rng(seed)
    sets, hs = [], []
    for d in (1, 2, 3):
        for n in (qn[d - 1], rn[d - 1], 2, 257):
            sets.append(datagen.mixture_dataset(g, n, d))
            hs.append(list(np.sort(g.uniform(0.004, 1.5, size=int(g.integers(1, 7))))))
    hs[3] = []
    return sets, hs


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_batched_queue_and_recursion_match_oracle(lib, prec):
    """The work queue (small datasets, every pair) and the recursion (larger
    ones) in one batched call, against the oracle's leave-one-out scores;
    bandwidths down to 0.004 put some sums below the float ranges."""
    old, _ = lib.tuning()
    lib.tuning_set({"f64": [1500, 1000, 800], "f32c": [1500, 1000, 800]})
    try:
        sets, hs = _mixed_sets([1400, 900, 700], [2100, 1300, 1100], 41)
        got, best = lib.kde_lcv_batched(bandwidth.to_device(sets), hs, prec=prec,
                                        want_best=True)
        tol = 1e-12 if prec == "f64" else 1e-5
        for x, h, r, b in zip(sets, hs, got, best.cpu().numpy()):
            if not h:
                assert b == -1
                continue
            ref = oracle.lcv(x, np.asarray(h))
            r = r.cpu().numpy()
            assert np.all(np.abs(r - ref) <= tol * np.maximum(1.0, np.abs(ref))), (x.shape, h)
            assert b == int(np.argmax(r))
    finally:
        lib.tuning_set(old)


def test_lcv_plan_replays_the_batch(lib):
    """A recorded plan gives the eager call's scores bit for bit, on every
    replay, and follows in-place changes of the data's values."""
    old, _ = lib.tuning()
    lib.tuning_set({"f64": [1500, 1000, 800], "f32c": [1500, 1000, 800]})
    try:
        sets, hs = _mixed_sets([1400, 900, 700], [2100, 1300, 1100], 43)
        dev = bandwidth.to_device(sets)
        want, wbest = lib.kde_lcv_batched(dev, hs, want_best=True)
        plan = lib.LcvPlan(dev, hs)
        for _ in range(3):
            got, best = plan.run()
            torch.cuda.synchronize()
            for a, b in zip(want, got):
                assert torch.equal(a, b)
            assert torch.equal(best, wbest)
            # eager work between replays
            lib.kde_lcv_batched(dev[:2], hs[:2])
        for x in dev:
            x.mul_(1.25)
        want2, _ = lib.kde_lcv_batched(dev, hs, want_best=True)
        got2, _ = plan.run()
        torch.cuda.synchronize()
        for a, b in zip(want2, got2):
            assert torch.equal(a, b)
        plan.close()
    finally:
        lib.tuning_set(old)


def test_autotune_writes_its_choice(lib, tmp_path):
    import json

    old, _ = lib.tuning()
    path = str(tmp_path / "tune.json")
    try:
        lib.autotune(path)
        doc = json.load(open(path))
        assert doc["arch"].startswith("gfx")
        sizes = {0, 512, 1024, 2048, 4096, 8192, 16384, 32768}
        for p in ("f64", "f32c"):
            assert len(doc["kde_queue_max_n"][p]) == 3
            assert all(v in sizes for v in doc["kde_queue_max_n"][p])
        now, src = lib.tuning()
        assert src == path and now == doc["kde_queue_max_n"]
        assert len(doc["ms_64_bandwidths"]) == 2 * 3 * 7
    finally:
        lib.tuning_set(old)
