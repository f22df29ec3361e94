"""Plain numpy oracle of the neural acoustic transfer field (Section 3: the
network that the Monte-Carlo BEM's data trains).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  It shares no code with
the GPU library.

Definition (the paper's Sections 3.2-3.4; readings in the design notes):
  * inputs: listener point in spherical coordinates about the scene's centre,
    polar angle theta in [0, pi], azimuth phi in [0, 2 pi), radius r in the
    training shell [r_lo, r_hi]; condition variables v in [0, 1]^n_v; the
    frequency normalised to [0, 1];
  * grid encoding G (Section 3.3): L = 4 lattices over the unit cube of
    (theta/pi, phi/(2 pi), (r - r_lo)/(r_hi - r_lo)), lattice l with
    8 * 2^l cells per axis, F = 4 features per lattice vertex, the features
    of a point the trilinear interpolation of its cell's 8 corners; a
    lattice with more than 2^16 vertices stores them in a table of 2^16
    entries indexed by the spatial hash (i * 1) xor (j * 2654435761) xor
    (k * 805459861) mod 2^16 (instant-NGP), the others densely;
  * positional encoding P (Section 3.2): sin(2^k pi c), cos(2^k pi c) for
    k = 0..5 and every scalar c of v and f;
  * MLP: input [G | P(v) | P(f)] padded with zeros to a multiple of 16,
    4 hidden layers of 128 with ReLU, a linear output layer; weights and
    biases;
  * loss: mean squared error against |p| (Section 3.2);
  * Adam (beta1 0.9, beta2 0.999, eps 1e-8), learning rate 1e-3 times 0.33
    after each third of the steps (Section 3.4).
Everything is float64.  With bf16=True the values the GPU form stores in
bfloat16 (the MLP's inputs, weights and hidden activations, and the
back-propagated gradients it multiplies and sums for the weights and the
biases) are rounded to bfloat16 (round to nearest even) at the same
points, with all sums in float64.
"""
from __future__ import annotations

import numpy as np

LEVELS = 4
BASE_RES = 8
FEATURES = 4
TABLE = 1 << 16
PE_FREQS = 6
HIDDEN = 128
N_HIDDEN = 4
PRIMES = (1, 2654435761, 805459861)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return out.reshape(np.shape(x))


def level_res(l):
    return BASE_RES << l


def level_size(l):
    n = (level_res(l) + 1) ** 3
    return n if n <= TABLE else TABLE


def level_hashed(l):
    return (level_res(l) + 1) ** 3 > TABLE


def vertex_index(l, i, j, k):
    """Table index of lattice vertex (i, j, k) of level l (arrays of int64)."""
    n1 = level_res(l) + 1
    if not level_hashed(l):
        return (i * n1 + j) * n1 + k
    h = (i.astype(np.uint64) * np.uint64(PRIMES[0])) ^ (j.astype(np.uint64) * np.uint64(PRIMES[1])) ^ \
        (k.astype(np.uint64) * np.uint64(PRIMES[2]))
    return (h & np.uint64(0xFFFFFFFF) & np.uint64(TABLE - 1)).astype(np.int64)


def unit_coords(theta, phi, r, r_lo, r_hi):
    return np.stack([theta / np.pi, phi / (2.0 * np.pi), (r - r_lo) / (r_hi - r_lo)], -1)


def grid_corners(u, l):
    """For unit-cube points u (B, 3): corner table indices (B, 8) and
    trilinear weights (B, 8) on level l."""
    n = level_res(l)
    p = np.clip(u, 0.0, 1.0) * n
    c = np.minimum(np.floor(p), n - 1).astype(np.int64)
    t = p - c
    idx, wts = [], []
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                idx.append(vertex_index(l, c[:, 0] + dx, c[:, 1] + dy, c[:, 2] + dz))
                wts.append((t[:, 0] if dx else 1.0 - t[:, 0]) * (t[:, 1] if dy else 1.0 - t[:, 1]) *
                           (t[:, 2] if dz else 1.0 - t[:, 2]))
    return np.stack(idx, 1), np.stack(wts, 1)


def grid_encode(u, grid):
    """G(u): (B, LEVELS * FEATURES)."""
    out = []
    for l in range(LEVELS):
        idx, w = grid_corners(u, l)
        out.append((grid[l][idx] * w[:, :, None]).sum(axis=1))
    return np.concatenate(out, axis=1)


def pe(c):
    """Positional encoding of scalars c (B, m) -> (B, 12 m): per scalar
    sin(2^k pi c), cos(2^k pi c), k = 0..5."""
    c = np.atleast_2d(np.asarray(c, dtype=np.float64))
    if c.shape[1] == 0:
        return np.zeros((c.shape[0], 0))
    cols = []
    for s in range(c.shape[1]):
        for k in range(PE_FREQS):
            a = (2.0 ** k) * np.pi * c[:, s]
            cols += [np.sin(a), np.cos(a)]
    return np.stack(cols, 1)


def input_dim(n_v):
    d = LEVELS * FEATURES + 2 * PE_FREQS * (n_v + 1)
    return (d + 15) // 16 * 16


def encode(theta, phi, r, v, f, grid, r_lo, r_hi):
    """The MLP input (B, input_dim): [G | P(v) | P(f) | zero padding]."""
    u = unit_coords(theta, phi, r, r_lo, r_hi)
    v = np.atleast_2d(v)
    x = np.concatenate([grid_encode(u, grid), pe(v), pe(np.asarray(f)[:, None])], axis=1)
    d = input_dim(v.shape[1])
    return np.concatenate([x, np.zeros((len(x), d - x.shape[1]))], axis=1)


def init_params(n_v, n_out, seed):
    """Glorot-uniform weights, zero biases, grid features uniform in +-1e-4."""
    rng = np.random.default_rng([seed, 11])
    d = input_dim(n_v)
    dims = [d] + [HIDDEN] * N_HIDDEN + [n_out]
    W = [rng.uniform(-1.0, 1.0, (dims[i + 1], dims[i])) * np.sqrt(6.0 / (dims[i] + dims[i + 1]))
         for i in range(len(dims) - 1)]
    b = [np.zeros(dims[i + 1]) for i in range(len(dims) - 1)]
    grid = [rng.uniform(-1e-4, 1e-4, (level_size(l), FEATURES)) for l in range(LEVELS)]
    return {"W": W, "b": b, "grid": grid}


def forward(x, params, bf=False):
    """Returns the output (B, n_out) and the per-layer inputs/pre-activations
    kept for the backward pass."""
    q = bf16 if bf else (lambda a: a)
    h = q(x)
    acts, pre = [h], []
    n = len(params["W"])
    for i in range(n):
        z = h @ q(params["W"][i]).T + params["b"][i]
        pre.append(z)
        if i < n - 1:
            h = q(np.maximum(z, 0.0))
            acts.append(h)
        else:
            h = z
    return h, (acts, pre)


def loss_and_grad(theta, phi, r, v, f, target, params, r_lo, r_hi, bf=False):
    """MSE loss and its gradient with respect to every parameter."""
    q = bf16 if bf else (lambda a: a)
    u = unit_coords(theta, phi, r, r_lo, r_hi)
    x = encode(theta, phi, r, v, f, params["grid"], r_lo, r_hi)
    y, (acts, pre) = forward(x, params, bf)
    target = np.asarray(target, dtype=np.float64).reshape(y.shape)
    diff = y - target
    loss = float(np.mean(diff * diff))
    dz = 2.0 * diff / diff.size
    n = len(params["W"])
    gW, gb = [None] * n, [None] * n
    for i in range(n - 1, -1, -1):
        gW[i] = q(dz).T @ acts[i]
        gb[i] = q(dz).sum(axis=0)
        dh = q(dz) @ q(params["W"][i])
        if i > 0:
            dz = dh * (pre[i - 1] > 0.0)
    # dh: gradient of the loss with respect to the MLP input x
    gg = [np.zeros_like(g) for g in params["grid"]]
    for l in range(LEVELS):
        idx, w = grid_corners(u, l)
        dxl = dh[:, l * FEATURES:(l + 1) * FEATURES]
        for c in range(8):
            np.add.at(gg[l], idx[:, c], w[:, c:c + 1] * dxl)
    return loss, {"W": gW, "b": gb, "grid": gg}


def lr_at(step, total, lr0=1e-3):
    """1e-3, times 0.33 after each third of the training."""
    return lr0 * 0.33 ** min(2, (3 * step) // max(total, 1))


def adam_step(params, grads, state, step, total, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of every parameter, step = 0, 1, ..."""
    lr = lr_at(step, total)
    t = step + 1
    for key in ("W", "b", "grid"):
        for i, g in enumerate(grads[key]):
            m = state.setdefault(("m", key, i), np.zeros_like(g))
            s = state.setdefault(("v", key, i), np.zeros_like(g))
            m *= beta1
            m += (1.0 - beta1) * g
            s *= beta2
            s += (1.0 - beta2) * g * g
            mh = m / (1.0 - beta1 ** t)
            sh = s / (1.0 - beta2 ** t)
            params[key][i] = params[key][i] - lr * mh / (np.sqrt(sh) + eps)
    return params
