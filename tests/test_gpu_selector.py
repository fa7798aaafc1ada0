"""GPU parity of the learned format selector: features against the oracle,
the MLP's forward pass, loss gradient and Adam steps against the FP64
oracle, model persistence, selection, and a small end-to-end training run
that must beat always using CSR."""
import math
import os

import numpy as np
import pytest

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2011_08879_amd as g
    return g


def feature_cases(gen_mod):
    yield "stencil27", gen_mod.stencil27(12), None
    yield "laplace1d", gen_mod.laplace1d(10), None
    yield "lognormal", gen_mod.random_lognormal(4, 30000, max_len=3000), None
    yield "banded", gen_mod.banded(5, 5000, 20, 3, 30), None
    yield "blockdiag", gen_mod.blockdiag(6, 3000, 4, 40), None
    yield "uniform0", gen_mod.uniform_random(7, 4000, 0, 9), None
    A = (np.array([0, 2, 2, 5], np.int32), np.array([1, 4, 0, 1, 2], np.int32), np.ones(5))
    yield "rect", A, 5


def test_features_match_oracle(g, orc, gen_mod):
    for name, A, m in feature_cases(gen_mod):
        M = g.Matrix.from_csr(*A, n_cols=m)
        fg = g.features(M).astype(np.float64)
        fo = orc.features(A, n_cols=m).astype(np.float32).astype(np.float64)
        err = np.abs(fg - fo)
        assert np.all(err <= 1e-6 * np.maximum(1.0, np.abs(fo))), (name, np.nonzero(err > 1e-6 * np.maximum(1, np.abs(fo))), fg, fo)
        for fmt in ("coo", "hybrid"):       # features do not depend on the stored format
            M.convert(fmt)
            assert np.array_equal(g.features(M).astype(np.float64), fg), (name, fmt)


def params(seed):
    import paper_2011_08879_amd.selector as sel
    return sel.he_uniform(seed)


def test_mlp_forward_and_gradient_match_oracle(g, orc):
    import torch
    rng = np.random.default_rng(3)
    P = params(1)
    assert P.size == g.N_PARAMS == orc.N_PARAMS and g.N_CLASSES == orc.N_CLASSES == 6
    b2 = 64 * 32 + 64 + 64 * 64
    P[b2:b2 + 64] = rng.uniform(-0.1, 0.1, 64)   # nonzero b2
    X = rng.standard_normal((300, 32)).astype(np.float32)
    Y = rng.standard_normal((300, g.N_CLASSES)).astype(np.float32)
    M = (rng.random((300, g.N_CLASSES)) > 0.25).astype(np.float32)
    model = g.Mlp(P)
    out = host(model.forward(dev(X)))
    ref = orc.mlp_forward(P.astype(np.float64), X.astype(np.float64))
    assert np.abs(out - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    loss, grad = model.loss_grad(dev(X), dev(Y), dev(M))
    lo, go = orc.mlp_loss_grad(P.astype(np.float64), X, Y, M)
    assert abs(float(host(loss)) - lo) <= 1e-5 * abs(lo)
    gg = host(grad).astype(np.float64)
    off = 0
    for shp in orc.MLP_SHAPES:
        k = int(np.prod(shp))
        a, b = gg[off:off + k], go[off:off + k]
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-7, (shp, np.linalg.norm(a - b), np.linalg.norm(b))
        off += k


def test_mlp_adam_steps_match_oracle(g, orc):
    rng = np.random.default_rng(4)
    P = params(2)
    X = rng.standard_normal((100, 32)).astype(np.float32)
    Y = np.tanh(X[:, :g.N_CLASSES]).astype(np.float32)
    M = np.ones((100, g.N_CLASSES), np.float32)
    model = g.Mlp(P)
    hist = host(model.train(dev(X), dev(Y), dev(M), 5, 1e-3))
    Pg, _ = model.params()
    Po = P.astype(np.float64)
    m, v = np.zeros_like(Po), np.zeros_like(Po)
    losses = []
    for t in range(1, 6):
        loss, G = orc.mlp_loss_grad(Po, X, Y, M)
        losses.append(loss)
        orc.adam_step(Po, G, m, v, t)
    assert np.allclose(hist, losses, rtol=1e-5, atol=0)
    assert np.abs(Pg - Po).max() <= 1e-5


def test_mlp_training_decreases_and_persists(g, tmp_path):
    import torch
    rng = np.random.default_rng(5)
    X = rng.standard_normal((400, 32)).astype(np.float32) * 3 + 1
    Y = np.stack([np.abs(X[:, k]) for k in range(g.N_CLASSES)], 1).astype(np.float32)
    M = np.ones((400, g.N_CLASSES), np.float32)
    model = g.Mlp(params(3))
    model.fit_normalization(dev(X))
    _, norm = model.params()
    assert np.allclose(norm[0], X.mean(0), atol=1e-4) and np.allclose(norm[1], X.std(0), rtol=1e-4)
    hist = host(model.train(dev(X), dev(Y), dev(M), 400, 3e-3))
    assert hist[-1] < 0.1 * hist[0]
    path = str(tmp_path / "sel.bin")
    model.save(path)
    other = g.Mlp.load(path)
    assert np.array_equal(host(other.forward(dev(X))), host(model.forward(dev(X))))


def test_autotune_select_and_auto_convert(g, orc, gen_mod):
    Ah = gen_mod.random_lognormal(4, 20000, max_len=5000)
    w, sets, _, _ = orc.csr_to_sellp(Ah)
    assert sets[-1] * 12 > 4 * (len(Ah[1]) * 12 + len(Ah[0]) * 4)   # SELL-P infeasible too
    A = g.Matrix.from_csr(*Ah)
    best, ms = g.autotune_format(A)
    assert g.SELECTOR_FORMATS[3] == "ell" and g.SELECTOR_FORMATS[5] == "sellp"
    assert np.isinf(ms[3]) and np.isinf(ms[5]) and np.all(np.isfinite(ms[[0, 1, 2, 4]]))
    assert best == g.SELECTOR_FORMATS[int(np.argmin(ms))]
    assert A.describe().format == "csr"                             # A untouched
    model = g.Mlp(params(4))
    fmt, scores = model.select(A)
    assert fmt in g.SELECTOR_FORMATS and fmt not in ("ell", "sellp") and scores.shape == (6,)
    g.set_selector(model)
    try:
        A.convert("auto")
        assert A.describe().format == fmt
    finally:
        g.set_selector(None)
    # a regular matrix: every format feasible and timed
    S = g.Matrix.from_csr(*gen_mod.stencil27(24))
    best, ms = g.autotune_format(S)
    assert np.all(np.isfinite(ms)) and best == g.SELECTOR_FORMATS[int(np.argmin(ms))]


def test_corpus_training_meets_regret_target(g):
    """400 generated matrices (320 train, 80 test): the trained network's picks
    stay within 10% of exhaustive autotuning in total SpMV time on the test
    matrices, and beat always using CSR (whose own regret is the headroom:
    about 1.07 on this corpus since CSR's kernels improved)."""
    import paper_2011_08879_amd.selector as sel
    res, model = sel.run(n_matrices=400, n_lo=1e4, n_hi=3e5, steps=3000, lr=3e-3, workers=8)
    model.close()
    assert res["loss_last"] < 0.5 * res["loss_first"]
    assert res["test"]["regret_total"] <= 1.10, res["test"]
    assert res["test"]["regret_total"] < res["test"]["csr_regret_total"], res["test"]
    assert res["test"]["gain_vs_csr_total"] > 1.0, res["test"]
