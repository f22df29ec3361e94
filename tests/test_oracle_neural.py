"""Pins for the oracle of the neural acoustic transfer field (Sections
3.2-3.4): bfloat16 rounding against torch's conversion, trilinear
interpolation exact on linear data, hash indices in the table, positional
encoding values, gradients against central differences, the first Adam
step and the learning-rate schedule in closed form, and a short training
run that fits a smooth target."""
import math

import numpy as np
import pytest

from oracle import neural as NF

torch = pytest.importorskip("torch")


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -2.5, 0.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(NF.bf16(x), ref)
    assert NF.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0          # tie to even


def test_trilinear_exact_on_linear_features_and_hash_in_range():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((3, NF.FEATURES))
    grid = []
    for l in range(NF.LEVELS):
        n = NF.level_res(l)
        g = np.zeros((NF.level_size(l), NF.FEATURES))
        if not NF.level_hashed(l):
            ii, jj, kk = np.meshgrid(*[np.arange(n + 1)] * 3, indexing="ij")
            ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
            pos = np.stack([ii, jj, kk], 1) / n
            g[NF.vertex_index(l, ii, jj, kk)] = pos @ a
        grid.append(g)
    u = rng.uniform(0.0, 1.0, (500, 3))
    enc = NF.grid_encode(u, grid)
    for l in range(NF.LEVELS):
        if not NF.level_hashed(l):
            assert np.allclose(enc[:, l * NF.FEATURES:(l + 1) * NF.FEATURES], u @ a, atol=1e-12)
    assert NF.level_hashed(3) and not NF.level_hashed(2)
    big = np.arange(0, 65, dtype=np.int64)
    idx = NF.vertex_index(3, big, big[::-1], (big * 7) % 65)
    assert idx.min() >= 0 and idx.max() < NF.TABLE
    assert NF.vertex_index(3, np.array([0]), np.array([1]), np.array([0]))[0] == 2654435761 % NF.TABLE


def test_positional_encoding_values():
    e = NF.pe(np.array([[0.0], [0.5], [0.25]]))
    assert e.shape == (3, 12)
    assert np.allclose(e[0], np.tile([0.0, 1.0], 6))
    # c = 1/2: sin(pi/2) = 1, cos(pi/2) = 0; k = 1: sin(pi) = 0, cos(pi) = -1
    assert np.allclose(e[1, :4], [1.0, 0.0, 0.0, -1.0], atol=1e-15)
    assert np.allclose(e[2, :2], [math.sqrt(0.5), math.sqrt(0.5)])


def _batch(B, n_v, seed):
    rng = np.random.default_rng(seed)
    th = np.arccos(1 - 2 * rng.uniform(0, 1, B))
    ph = rng.uniform(0, 2 * np.pi, B)
    r = rng.uniform(1.5, 3.0, B)
    v = rng.uniform(0, 1, (B, n_v))
    f = rng.uniform(0, 1, B)
    return th, ph, r, v, f


def test_gradients_against_central_differences():
    n_v, n_out, B = 2, 3, 64
    p = NF.init_params(n_v, n_out, 3)
    p["grid"] = [g * 1e3 for g in p["grid"]]          # make the grid matter
    th, ph, r, v, f = _batch(B, n_v, 4)
    tgt = np.random.default_rng(5).standard_normal((B, n_out))
    loss, g = NF.loss_and_grad(th, ph, r, v, f, tgt, p, 1.5, 3.0)
    rng = np.random.default_rng(6)
    for key, i in [("W", 0), ("W", 2), ("W", 4), ("b", 1), ("b", 4)]:
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p[key][i].shape)
            h = 1e-6
            p[key][i][idx] += h
            lp, _ = NF.loss_and_grad(th, ph, r, v, f, tgt, p, 1.5, 3.0)
            p[key][i][idx] -= 2 * h
            lm, _ = NF.loss_and_grad(th, ph, r, v, f, tgt, p, 1.5, 3.0)
            p[key][i][idx] += h
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[key][i][idx]) <= 1e-6 * max(1.0, abs(fd)), (key, i, idx, fd, g[key][i][idx])
    for l in range(NF.LEVELS):
        touched = np.flatnonzero(np.abs(g["grid"][l]).sum(axis=1))
        for e in touched[:3]:
            h = 1e-5
            p["grid"][l][e, 1] += h
            lp, _ = NF.loss_and_grad(th, ph, r, v, f, tgt, p, 1.5, 3.0)
            p["grid"][l][e, 1] -= 2 * h
            lm, _ = NF.loss_and_grad(th, ph, r, v, f, tgt, p, 1.5, 3.0)
            p["grid"][l][e, 1] += h
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g["grid"][l][e, 1]) <= 1e-6 * max(1.0, abs(fd)), (l, e)


def test_adam_first_step_and_schedule():
    p = {"W": [np.array([[2.0, -3.0]])], "b": [np.array([0.5])], "grid": [np.array([[1.0]])]}
    g = {"W": [np.array([[4.0, -0.1]])], "b": [np.array([0.0])], "grid": [np.array([[-7.0]])]}
    NF.adam_step(p, g, {}, 0, 9)
    # first step: m_hat = g, v_hat = g^2, so the move is lr g / (|g| + eps)
    assert np.allclose(p["W"][0], [[2.0 - 1e-3 * 4 / (4 + 1e-8), -3.0 + 1e-3 * 0.1 / (0.1 + 1e-8)]])
    assert p["b"][0][0] == 0.5
    assert np.isclose(p["grid"][0][0, 0], 1.0 + 1e-3 * 7 / (7 + 1e-8))
    assert [NF.lr_at(s, 9) for s in (0, 2, 3, 5, 6, 8)] == pytest.approx([1e-3, 1e-3, 3.3e-4, 3.3e-4,
                                                                          1.089e-4, 1.089e-4])


@pytest.mark.parametrize("bf", [False, True])
def test_training_fits_a_smooth_field(bf):
    """200 Adam steps on 1024 points of a smooth positive field of (theta,
    phi, r, v, f) bring the MSE below a tenth of its start (also with the
    bfloat16 storage rounding)."""
    n_v, B = 1, 1024
    th, ph, r, v, f = _batch(B, n_v, 7)
    tgt = (1.0 + 0.5 * np.cos(th) * np.sin(ph + 2 * v[:, 0]) + 0.3 * f) / r
    p = NF.init_params(n_v, 1, 8)
    st = {}
    first = None
    for s in range(200):
        loss, g = NF.loss_and_grad(th, ph, r, v, f, tgt, p, 1.5, 3.0, bf=bf)
        first = loss if first is None else first
        NF.adam_step(p, g, st, s, 200)
    assert loss < 0.1 * first, (first, loss)


def test_frequency_only_input_layout():
    """With no condition variables the input is [G (16) | P(f) (12) | 0 (4)]:
    width 32, P(f) the closed-form sines and cosines of 2^k pi f, the pad
    zero."""
    B = 5
    th, ph, r, v, f = _batch(B, 0, 11)
    p = NF.init_params(0, 1, 2)
    x = NF.encode(th, ph, r, v, f, p["grid"], 1.5, 3.0)
    assert NF.input_dim(0) == 32 and x.shape == (B, 32)
    for k in range(6):
        a = (2.0 ** k) * np.pi * f
        assert np.allclose(x[:, 16 + 2 * k], np.sin(a), atol=1e-15)
        assert np.allclose(x[:, 17 + 2 * k], np.cos(a), atol=1e-15)
    assert np.all(x[:, 28:] == 0.0)
    y, _ = NF.forward(x, p)
    assert y.shape == (B, 1)
