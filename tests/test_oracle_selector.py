"""Pins for the oracle's selector arithmetic: the 32 structural features on
matrices worked by hand, and the MLP's loss gradient against central finite
differences, a hand-set forward pass and Adam's first step in closed form."""
import math

import numpy as np
import pytest


def test_features_tridiagonal_by_hand(orc, gen_mod):
    f = orc.features(gen_mod.laplace1d(10))   # lengths 2, 3 x 8, 2; nnz 28
    hand = {0: 1.0, 1: math.log10(28), 2: 2.8, 3: 0.4, 4: 0.4 / 2.8, 5: 2, 6: 3, 7: 3, 8: 3, 9: 3,
            10: 3 / 2.8, 11: 0.0, 12: 1.0, 13: 30 / 28, 14: 3 / 2.8,   # K* = 3: 360 B < 368 B
            15: 0.0, 16: 2 / 35,            # sum |l_i - l_j| = 32 over ordered pairs
            17: -(0.2 * math.log(0.2) + 0.8 * math.log(0.8)), 18: 3 / 28,
            19: math.log10(12 * 28 + 4 * 11 + 80 + 80), 20: 64 * 3 / 28, 21: 1.0,   # one slice
            22: 18 / 28 / 10, 23: 0.1, 24: 10 / 28, 25: 1.0, 26: 1.0, 27: math.log10(2),
            28: 1.0, 29: 12 / 28,           # rows 7 and 8 straddle the column-8 boundary
            30: 1.0, 31: math.log10(1 + 28 / 10)}
    for k, v in hand.items():
        assert abs(f[k] - v) <= 1e-12 * max(1.0, abs(v)), (k, f[k], v)


def test_features_identity_and_rectangular(orc):
    n = 100
    I = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    f = orc.features(I)
    assert f[2] == 1 and f[3] == 0 and f[16] == 0 and f[17] == 0 and f[24] == 1
    assert f[27] == 0 and f[28] == 0 and f[29] == 1 and f[30] == 1 and f[18] == 1 / 100
    assert f[20] == 128 / 100      # two 64-row slices of width 1
    # 3 x 5 with an empty row: rows {0: [1, 4]}, {1: []}, {2: [0, 1, 2]}
    A = (np.array([0, 2, 2, 5], np.int32), np.array([1, 4, 0, 1, 2], np.int32), np.ones(5))
    f = orc.features(A, n_cols=5)
    assert f[11] == 1 / 3 and f[21] == 5 / 3 and f[30] == 0.0 and f[5] == 0 and f[6] == 3
    assert f[22] == (1 + 4 + 2 + 1 + 0) / 5 / 5 and f[23] == 4 / 5
    assert abs(f[27] - math.log10(1 + (3 + 1 + 1) / 3)) < 1e-15 and f[28] == 2 / 3
    assert abs(f[31] - math.log10(1 + (4 + 3) / 2)) < 1e-15
    assert f[20] == 64 * 3 / 5
    # no entries: every padding ratio is 1 by convention
    f = orc.features((np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0)))
    assert f[13] == 1.0 and f[20] == 1.0


def test_sellp_padding_feature_matches_layout(orc, gen_mod):
    """Feature 20 against the slot count of the (separately pinned) SELL-P layout."""
    for A in (gen_mod.random_lognormal(41, 5000, mean=8.0, sigma=1.2, max_len=500),
              gen_mod.banded(42, 3001, 30, 1, 40), gen_mod.blockdiag(43, 2000, 4, 40),
              gen_mod.stencil27(9)):
        w, sets, sc, sv = orc.csr_to_sellp(A, 64)
        assert orc.features(A)[20] == sets[-1] / len(A[1])


def init_params(seed):
    rng = np.random.default_rng(seed)
    P = []
    for shp in orc_shapes():
        if len(shp) == 2:
            lim = math.sqrt(6.0 / shp[1])
            P.append(rng.uniform(-lim, lim, shp).ravel())
        else:
            P.append(rng.uniform(-0.1, 0.1, shp))
    return np.concatenate(P)


def orc_shapes():
    return [(64, 32), (64,), (64, 64), (64,), (6, 64), (6,)]


def test_mlp_gradient_matches_central_differences(orc):
    rng = np.random.default_rng(3)
    P = init_params(1)
    assert P.size == orc.N_PARAMS == 6662 and orc.N_CLASSES == 6
    X = rng.standard_normal((40, 32))
    Y = rng.standard_normal((40, 6))
    M = (rng.random((40, 6)) > 0.2).astype(float)
    loss, G = orc.mlp_loss_grad(P, X, Y, M)
    h = 1e-6
    for i in rng.choice(P.size, 60, replace=False):
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (orc.mlp_loss_grad(Pp, X, Y, M)[0] - orc.mlp_loss_grad(Pm, X, Y, M)[0]) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * max(1.0, abs(G[i])) + 1e-9, (i, fd, G[i])


def test_mlp_forward_by_hand(orc):
    # W1 = [I_32; 0], W2 = I_64, W3 picks units 0..5 (unit 5 twice), b3 set:
    # o = relu(x)[0:6] * (1, 1, 1, 1, 1, 2) + b3
    W1 = np.zeros((64, 32))
    W1[:32, :32] = np.eye(32)
    W3 = np.zeros((6, 64))
    W3[np.arange(6), np.arange(6)] = 1.0
    W3[5, 5] = 2.0
    b3 = np.array([0.0, 1.0, 0.0, 0.0, -2.0, 0.5])
    P = np.concatenate([W1.ravel(), np.zeros(64), np.eye(64).ravel(), np.zeros(64), W3.ravel(), b3])
    x = np.linspace(-2, 2, 32)
    o = orc.mlp_forward(P, x[None])[0]
    assert np.array_equal(o, np.maximum(x[:6], 0) * np.array([1, 1, 1, 1, 1, 2]) + b3)


def test_adam_first_step_closed_form_and_training_decreases(orc):
    P = np.array([1.0, -2.0, 3.0])
    G = np.array([0.5, -4.0, 0.0])
    m, v = np.zeros(3), np.zeros(3)
    orc.adam_step(P, G, m, v, 1, lr=0.01)
    # t = 1: mhat = g, vhat = g^2, so the step is lr g / (|g| + eps)
    assert np.allclose(P, [1.0 - 0.01 * 0.5 / (0.5 + 1e-8), -2.0 + 0.01 * 4 / (4 + 1e-8), 3.0],
                       rtol=0, atol=1e-15)
    rng = np.random.default_rng(5)
    P = init_params(2)
    X = rng.standard_normal((64, 32))
    Y = np.tanh(X[:, :6]) + 0.1
    M = np.ones((64, 6))
    m, v = np.zeros_like(P), np.zeros_like(P)
    losses = []
    for t in range(1, 201):
        loss, G = orc.mlp_loss_grad(P, X, Y, M)
        losses.append(loss)
        orc.adam_step(P, G, m, v, t)
    assert losses[-1] < 0.2 * losses[0]
    assert all(b <= a * 1.05 for a, b in zip(losses[:20], losses[1:21]))
