"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these checks re-types an oracle formula: each compares the oracle
with a printed value, a library routine, a closed form or an invariant, chosen
so that a dropped term, a wrong sign or index or a transposed operand fails.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def small_model(L=3, F=2, log2T=12, res=(5, 9, 17), width=16, n_hidden=2):
    return oracle.Model(L, F, log2T, list(res), width, n_hidden)


def rand_params(m, seed=7, table_scale=0.5):
    rng = np.random.default_rng(seed)
    p = np.concatenate([rng.uniform(-table_scale, table_scale, m.n_table),
                        rng.uniform(-0.6, 0.6, m.n_mlp)])
    return p


# ---------------------------------------------------------------- RNG -----

def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLD, "splitmix64_seed0.json")))
    # stream 0, seed 0 is the plain generator started from state 0
    for n, hx in enumerate(g["outputs_hex"]):
        assert oracle.rng_u64(0, 0, n) == int(hx, 16)


def test_rng_two_implementations_agree():
    # the NumPy input generator and the C oracle implement the same definition
    idx = np.arange(0, 5000, 7, dtype=np.uint64)
    a = synth.rng_u64(2207_11620, 3, idx)
    b = np.array([oracle.rng_u64(2207_11620, 3, int(i)) for i in idx], dtype=np.uint64)
    assert np.array_equal(a, b)
    u = oracle.batch_coords(99, 5, 300)
    ref = synth.rng_u01(99, synth.STREAM_BATCH, np.arange(5 * 300 * 3, 6 * 300 * 3)).reshape(300, 3)
    assert np.array_equal(u, ref)
    assert u.min() >= 0.0 and u.max() < 1.0
    # uniformity sanity: mean of 2^16 draws within 5 sigma of 1/2
    v = synth.rng_u01_f64(1, 4, np.arange(1 << 16))
    assert abs(v.mean() - 0.5) < 5 * math.sqrt(1 / 12 / (1 << 16))


# --------------------------------------------------- layout / counts -----

def test_resolution_lists():
    # growth 1.5 from 4 (8 levels) and 16 -> 2048 geometric (16 levels)
    assert oracle.resolutions(8, 4, 1.5) == [4, 6, 9, 14, 21, 31, 46, 69]
    r = oracle.resolutions(16, 16, 0.0, 2048)
    assert r[0] == 16 and r[-1] == 2048 and len(r) == 16
    b = 128 ** (1 / 15)
    for l, n in enumerate(r):  # ceil of the real resolution, exact ends
        assert n == (round(16 * b ** l) if l in (0, 15) else math.ceil(16 * b ** l))
    assert oracle.resolutions(5, 4, 2.0) == [4, 8, 16, 32, 64]


def test_param_counts_match_paper():
    g = json.load(open(os.path.join(GOLD, "param_counts.json")))
    for mdl in g["models"]:
        res = oracle.resolutions(mdl["L"], mdl["base"], 2.0)
        m = oracle.Model(mdl["L"], mdl["F"], mdl["log2T"], res, mdl["width"], mdl["n_hidden"])
        w, nin = mdl["width"], mdl["L"] * mdl["F"]
        nin_pad = -(-nin // 16) * 16
        mlp_padded = nin_pad * w + (mdl["n_hidden"] - 1) * w * w + w * 16
        # unpadded storage: the last layer has a single output row
        assert m.n_mlp == nin * w + (mdl["n_hidden"] - 1) * w * w + w
        total = m.n_table + mlp_padded
        assert total == mdl["printed_params"], mdl["name"]
        assert round(total * 2 / 2 ** 20, 1) == mdl["table1_size_mb"], mdl["name"]


def test_level_sizes_dense_then_capped():
    m = oracle.Model(8, 2, 14, oracle.resolutions(8, 4, 1.5), 32, 2)
    assert list(m.level_size) == [64, 216, 729, 2744, 9261, 16384, 16384, 16384]
    assert list(np.diff(m.level_offset)) == list(m.level_size)
    assert m.n_params == 125900


# ------------------------------------------------------------ hash -----

def test_hash_vectors():
    # Mueller et al. spatial hash with primes (1, 2654435761, 805459861),
    # evaluated by hand: 2654435761 = 0x9E3779B1, 805459861 = 0x30025795.
    # level with N=64 vertices (64^3 > 2^14: hashed)
    m = oracle.Model(1, 1, 14, [64], 8, 1)
    s = 1.0 / 63.0
    pts = np.array([[0.5 * s, 1.5 * s, 0.5 * s],     # cell (0,1,0): corner 0 = (0,1,0)
                    [0.5 * s, 0.5 * s, 1.5 * s],     # cell (0,0,1): corner 0 = (0,0,1)
                    [0.5 * s, 0.5 * s, 0.5 * s],     # cell (0,0,0): corner 7 = (1,1,1)
                    [5.5 * s, 7.5 * s, 11.5 * s]],   # cell (5,7,11): corner 0
                   dtype=np.float32)
    idx, _ = oracle.encode_debug(m, pts)
    assert idx[0, 0, 0] == 0x39B1 == 14769          # 0x9E3779B1 & 0x3FFF
    assert idx[1, 0, 0] == 0x1795 == 6037           # 0x30025795 & 0x3FFF
    assert idx[2, 0, 7] == 11813                    # (1 ^ 0x9E3779B1 ^ 0x30025795) & 0x3FFF
    assert idx[2, 0, 0] == 0                        # vertex (0,0,0) hashes to 0
    assert idx[3, 0, 0] == 4277
    # T = 2^19 on the finest cfg1 level (N = 2048)
    m2 = oracle.Model(1, 1, 19, [2048], 8, 1)
    t = 1.0 / 2047.0
    p2 = np.array([[1.5 * t, 1.5 * t, 1.5 * t], [1.0, 1.0, 1.0]], dtype=np.float32)
    idx2, w2 = oracle.encode_debug(m2, p2)
    assert idx2[0, 0, 0] == 339493                  # vertex (1,1,1)
    assert idx2[1, 0, 7] == 285147                  # vertex (2047,2047,2047): x=1 -> last cell, w=1
    assert w2[1, 0, 7] == 1.0 and np.all(w2[1, 0, :7] == 0.0)


def test_dense_index_and_corner_order():
    # a dense level: slot = vx + N*(vy + N*vz); corner k has delta (k&1, k>>1&1, k>>2&1)
    N = 9
    m = oracle.Model(1, 1, 12, [N], 8, 1)
    c = np.array([3, 5, 7])
    p = ((c + 0.25) / (N - 1)).astype(np.float32)[None]
    idx, w = oracle.encode_debug(m, p)
    for k in range(8):
        d = np.array([k & 1, (k >> 1) & 1, (k >> 2) & 1])
        v = c + d
        assert idx[0, 0, k] == v[0] + N * (v[1] + N * v[2])
    # weights for fractional offset 0.25 on every axis
    for k in range(8):
        n1 = bin(k).count("1")
        assert w[0, 0, k] == pytest.approx(0.25 ** n1 * 0.75 ** (3 - n1), abs=1e-12)


# ---------------------------------------------------- interpolation -----

def test_collision_free_equals_dense_trilinear_library():
    # cfg0 resolutions with T = 2^19: every level dense (69^3 < 2^19)
    res = oracle.resolutions(8, 4, 1.5)
    m = oracle.Model(8, 2, 19, res, 16, 1)
    assert all(s == n ** 3 for s, n in zip(m.level_size, res))
    rng = np.random.default_rng(3)
    params = rng.normal(size=m.n_params)
    xyz = rng.random((500, 3)).astype(np.float32)
    xyz[:5] = [[0, 0, 0], [1, 1, 1], [1, 0, 0.5], [0.999999, 1e-7, 0.5], [0.5, 0.5, 0.5]]
    e = oracle.encode(m, params, xyz)
    for l, N in enumerate(res):
        off = int(m.level_offset[l])
        g = np.linspace(0.0, 1.0, N)
        for f in range(2):
            tab = params[2 * off + f: 2 * (off + N ** 3): 2].reshape(N, N, N)  # [vz][vy][vx]
            interp = RegularGridInterpolator((g, g, g), tab, method="linear")
            ref = interp(xyz[:, ::-1].astype(np.float64))
            np.testing.assert_allclose(e[:, 2 * l + f], ref, rtol=0, atol=1e-12)


def test_affine_field_reproduced_exactly():
    res = [5, 9, 17, 33]
    m = oracle.Model(4, 1, 17, res, 8, 1)  # all dense (33^3 < 2^17)
    a = np.array([0.3, -1.7, 2.5])
    b = 0.125
    params = np.zeros(m.n_params)
    for l, N in enumerate(res):
        v = np.arange(N) / (N - 1)
        vz, vy, vx = np.meshgrid(v, v, v, indexing="ij")
        params[m.level_offset[l]: m.level_offset[l + 1]] = (a[0] * vx + a[1] * vy + a[2] * vz + b).ravel()
    xyz = np.random.default_rng(5).random((1000, 3)).astype(np.float32)
    e = oracle.encode(m, params, xyz)
    exact = xyz.astype(np.float64) @ a + b
    for l in range(4):
        np.testing.assert_allclose(e[:, l], exact, atol=2e-15 * 8)


def test_partition_of_unity_and_vertex_values():
    m = oracle.Model(8, 2, 14, oracle.resolutions(8, 4, 1.5), 32, 2)
    xyz = np.random.default_rng(11).random((2000, 3)).astype(np.float32)
    idx, w = oracle.encode_debug(m, xyz)
    assert np.all(w >= 0.0) and np.all(w <= 1.0)
    np.testing.assert_allclose(w.sum(axis=2), 1.0, atol=1e-14)
    # at a vertex the feature equals that vertex's table entry
    params = rand_params(m)
    for l, N in enumerate(m.res):
        v = np.array([[2, 1, N - 1]])
        p = (v / (N - 1)).astype(np.float32)
        exact = np.all(p.astype(np.float64) * (N - 1) == v)
        if not exact:
            continue
        i, ww = oracle.encode_debug(m, p)
        k = int(np.argmax(ww[0, l]))
        assert ww[0, l, k] == 1.0
        e = oracle.encode(m, params, p)
        slot = int(m.level_offset[l]) + int(i[0, l, k])
        assert e[0, 2 * l] == params[2 * slot] and e[0, 2 * l + 1] == params[2 * slot + 1]


def test_clamp_outside_unit_cube():
    m = small_model()
    params = rand_params(m)
    a = np.array([[-0.5, 0.3, 1.5], [2.0, -1.0, 0.5]], np.float32)
    b = np.clip(a, 0, 1)
    np.testing.assert_array_equal(oracle.encode(m, params, a), oracle.encode(m, params, b))


# --------------------------------------------------------------- MLP -----

def test_mlp_equals_blas_chain():
    m = oracle.Model(16, 2, 19, oracle.resolutions(16, 16, 0, 2048), 64, 2)
    rng = np.random.default_rng(1)
    W = rng.normal(size=m.n_mlp) * 0.2
    feat = rng.normal(size=(300, 32))
    out = oracle.mlp_fwd(m, W, feat)
    W1 = W[:64 * 32].reshape(64, 32)
    W2 = W[64 * 32: 64 * 32 + 64 * 64].reshape(64, 64)
    W3 = W[64 * 32 + 64 * 64:].reshape(1, 64)
    h = np.maximum(feat @ W1.T, 0)
    h = np.maximum(h @ W2.T, 0)
    ref = (h @ W3.T)[:, 0]
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_forward_is_encode_then_mlp():
    m = small_model()
    params = rand_params(m)
    xyz = np.random.default_rng(2).random((100, 3)).astype(np.float32)
    a = oracle.forward(m, params, xyz)
    b = oracle.mlp_fwd(m, params[m.n_table:], oracle.encode(m, params, xyz))
    np.testing.assert_allclose(a, b, rtol=1e-14, atol=1e-15)


# ---------------------------------------------------------- gradient -----

def _loss(m, params, xyz, y):
    out = oracle.forward(m, params, xyz)
    return float(np.mean((out - y) ** 2))


def test_gradient_central_differences():
    m = small_model(L=3, F=2, log2T=10, res=(5, 9, 17), width=16, n_hidden=2)
    params = rand_params(m, seed=4)
    rng = np.random.default_rng(8)
    xyz = rng.random((64, 3)).astype(np.float32)
    y = rng.random(64)
    loss, g = oracle.loss_grad(m, params, xyz, y)
    assert loss == pytest.approx(_loss(m, params, xyz, y), rel=1e-13)
    h = 1e-3
    # every MLP weight, and the table entries the batch touches plus some it does not
    idx, _ = oracle.encode_debug(m, xyz)
    touched = set()
    for l in range(m.L):
        for s in np.unique(idx[:, l, :]):
            touched.update({2 * (int(m.level_offset[l]) + int(s)) + f for f in range(2)})
    cand = sorted(touched)[::7] + list(range(m.n_table, m.n_params))
    cand += [i for i in range(0, m.n_table, 97) if i not in touched][:10]
    checked = 0
    for i in cand:
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        fd = (_loss(m, p1, xyz, y) - _loss(m, p2, xyz, y)) / (2 * h)
        # piecewise quadratic in one parameter: FD exact unless a ReLU flips
        # within +-h; detect flips by comparing one-sided second differences
        l0 = _loss(m, params, xyz, y)
        c2a = (_loss(m, p1, xyz, y) - l0)
        c2b = (l0 - _loss(m, p2, xyz, y))
        p3 = params.copy()
        p3[i] += 2 * h
        c2c = (_loss(m, p3, xyz, y) - _loss(m, p1, xyz, y))
        if abs((c2c - c2a) - (c2a - c2b)) > 1e-9 * max(1.0, abs(c2a)):
            continue
        assert fd == pytest.approx(g[i], rel=1e-7, abs=1e-11), i
        checked += 1
    assert checked > 0.8 * len(cand)
    # untouched table entries have exactly zero gradient
    un = [i for i in range(m.n_table) if i not in touched]
    assert np.all(g[un] == 0.0)


def test_gradient_matches_torch_autograd_for_mlp_block():
    torch = pytest.importorskip("torch")
    m = small_model(L=3, F=2, log2T=10, res=(5, 9, 17), width=16, n_hidden=3)
    params = rand_params(m, seed=9)
    rng = np.random.default_rng(10)
    xyz = rng.random((128, 3)).astype(np.float32)
    y = rng.random(128)
    _, g = oracle.loss_grad(m, params, xyz, y)
    e = torch.tensor(oracle.encode(m, params, xyz), dtype=torch.float64, requires_grad=True)
    Ws = []
    pos = m.n_table
    for (o, i) in synth.mlp_shapes(m.n_in, m.width, m.n_hidden):
        Ws.append(torch.tensor(params[pos:pos + o * i].reshape(o, i), dtype=torch.float64, requires_grad=True))
        pos += o * i
    h = e
    for W in Ws[:-1]:
        h = torch.relu(torch.nn.functional.linear(h, W))
    out = torch.nn.functional.linear(h, Ws[-1])[:, 0]
    loss = torch.mean((out - torch.tensor(y)) ** 2)
    loss.backward()
    gm = np.concatenate([W.grad.numpy().ravel() for W in Ws])
    np.testing.assert_allclose(g[m.n_table:], gm, rtol=1e-12, atol=1e-15)
    # table gradient = scatter of dL/de through the corner weights
    idx, w = oracle.encode_debug(m, xyz)
    de = e.grad.numpy()
    gt = np.zeros(m.n_table)
    for l in range(m.L):
        for f in range(m.F):
            slots = 2 * (m.level_offset[l] + idx[:, l, :].astype(np.int64)) + f
            np.add.at(gt, slots.ravel(), (w[:, l, :] * de[:, 2 * l + f][:, None]).ravel())
    np.testing.assert_allclose(g[:m.n_table], gt, rtol=1e-12, atol=1e-15)


def test_l1_gradient_central_differences():
    # L1 (the paper's default loss, Section 3.1): mean |Phi - y|.  Targets sit
    # at least 0.05 away from the model so no residual changes sign within +-h
    m = small_model(L=3, F=2, log2T=10, res=(5, 9, 17), width=16, n_hidden=2)
    params = rand_params(m, seed=14)
    rng = np.random.default_rng(15)
    xyz = rng.random((48, 3)).astype(np.float32)
    out0 = oracle.forward(m, params, xyz)
    y = out0 + rng.choice([-1.0, 1.0], 48) * rng.uniform(0.05, 0.3, 48)

    def l1(p):
        return float(np.mean(np.abs(oracle.forward(m, p, xyz) - y)))

    loss, g = oracle.loss_grad(m, params, xyz, y, loss="l1")
    assert loss == pytest.approx(l1(params), rel=1e-13)
    # the L2 gradient of the same batch differs (a swapped loss kind fails here)
    _, g2 = oracle.loss_grad(m, params, xyz, y)
    assert np.max(np.abs(g2 - g)) > 1e-3
    h = 1e-4
    checked = 0
    cand = list(range(0, m.n_table, 13)) + list(range(m.n_table, m.n_params, 3))
    for i in cand:
        p1, p2, p3 = params.copy(), params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        p3[i] += 2 * h
        la, lb, l0, lc = l1(p1), l1(p2), l1(params), l1(p3)
        # piecewise polynomial in one parameter: skip where a ReLU flips
        if abs((lc - la) - (la - l0)) > 1e-9 or abs((la - l0) - (l0 - lb)) > 1e-9:
            continue
        assert (la - lb) / (2 * h) == pytest.approx(g[i], rel=1e-6, abs=1e-10), i
        checked += 1
    assert checked > 0.8 * len(cand)


def test_l1_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    m = small_model(L=3, F=2, log2T=10, res=(5, 9, 17), width=16, n_hidden=3)
    params = rand_params(m, seed=16)
    rng = np.random.default_rng(17)
    xyz = rng.random((128, 3)).astype(np.float32)
    y = rng.random(128)
    _, g = oracle.loss_grad(m, params, xyz, y, loss="l1")
    e = torch.tensor(oracle.encode(m, params, xyz), dtype=torch.float64, requires_grad=True)
    Ws = []
    pos = m.n_table
    for (o, i) in synth.mlp_shapes(m.n_in, m.width, m.n_hidden):
        Ws.append(torch.tensor(params[pos:pos + o * i].reshape(o, i), dtype=torch.float64, requires_grad=True))
        pos += o * i
    h = e
    for W in Ws[:-1]:
        h = torch.relu(torch.nn.functional.linear(h, W))
    out = torch.nn.functional.linear(h, Ws[-1])[:, 0]
    torch.nn.functional.l1_loss(out, torch.tensor(y)).backward()
    gm = np.concatenate([W.grad.numpy().ravel() for W in Ws])
    np.testing.assert_allclose(g[m.n_table:], gm, rtol=1e-12, atol=1e-15)
    idx, w = oracle.encode_debug(m, xyz)
    de = e.grad.numpy()
    gt = np.zeros(m.n_table)
    for l in range(m.L):
        for f in range(m.F):
            slots = 2 * (m.level_offset[l] + idx[:, l, :].astype(np.int64)) + f
            np.add.at(gt, slots.ravel(), (w[:, l, :] * de[:, 2 * l + f][:, None]).ravel())
    np.testing.assert_allclose(g[:m.n_table], gt, rtol=1e-12, atol=1e-15)


# -------------------------------------------------------------- Adam -----

def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    n = 1000
    theta = rng.normal(size=n)
    th0 = theta.copy()
    g = rng.normal(size=n) * 10 ** rng.uniform(-8, 2, n)
    g[::10] = 0.0
    mm, vv = np.zeros(n), np.zeros(n)
    oracle.adam(theta, mm, vv, g, 1, 1e-2, 0.9, 0.99, 1e-15)
    step = theta - th0
    # step 1: m_hat = g, v_hat = g^2, so the move is -lr g / (|g| + eps): -lr sign(g) up to eps/|g|
    gz = g[g != 0]
    np.testing.assert_allclose(step[g != 0], -1e-2 * gz / (np.abs(gz) + 1e-15), rtol=1e-12)
    np.testing.assert_allclose(step[g != 0], -1e-2 * np.sign(gz), rtol=1e-4)
    assert np.all(step[g == 0] == 0.0)


def test_adam_matches_torch_optim():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    n = 257
    theta = rng.normal(size=n)
    tp = torch.tensor(theta.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.99), eps=1e-15)
    mm, vv = np.zeros(n), np.zeros(n)
    for t in range(1, 21):
        g = rng.normal(size=n)
        g[rng.random(n) < 0.3] = 0.0
        oracle.adam(theta, mm, vv, g, t, 1e-2, 0.9, 0.99, 1e-15)
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(theta, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_l2_reg_matches_torch_weight_decay():
    # L2 regularisation of the network weights = torch Adam's (coupled)
    # weight_decay on the MLP block only
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(18)
    n_table, n = 300, 420
    theta = rng.normal(size=n)
    tt = torch.tensor(theta[:n_table].copy(), requires_grad=True)
    tw = torch.tensor(theta[n_table:].copy(), requires_grad=True)
    opt = torch.optim.Adam([{"params": [tt], "weight_decay": 0.0}, {"params": [tw], "weight_decay": 0.05}],
                           lr=5e-3, betas=(0.9, 0.999), eps=1e-15)
    mm, vv = np.zeros(n), np.zeros(n)
    for t in range(1, 16):
        g = rng.normal(size=n)
        g[rng.random(n) < 0.3] = 0.0
        oracle.adam(theta, mm, vv, g, t, 5e-3, 0.9, 0.999, 1e-15, l2_reg=0.05, reg_from=n_table)
        tt.grad = torch.tensor(g[:n_table])
        tw.grad = torch.tensor(g[n_table:])
        opt.step()
    np.testing.assert_allclose(theta[:n_table], tt.detach().numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(theta[n_table:], tw.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_lr_decay_paper_default_values():
    # appendix default optimiser: lr 5e-3, decay start 2000, interval 1000, base 0.99
    d = (2000, 1000, 0.99)
    assert oracle.lr_at(5e-3, 0, d) == 5e-3
    assert oracle.lr_at(5e-3, 1999, d) == 5e-3
    assert oracle.lr_at(5e-3, 2999, d) == 5e-3
    assert oracle.lr_at(5e-3, 3000, d) == pytest.approx(5e-3 * 0.99, rel=1e-15)
    assert oracle.lr_at(5e-3, 12999, d) == pytest.approx(5e-3 * 0.99 ** 10, rel=1e-14)
    assert oracle.lr_at(5e-3, 10 ** 6, None) == 5e-3


def test_lr_decay_matches_torch_schedulers():
    # constant for `start` steps, then a staircase decay: torch's ConstantLR
    # (factor 1) followed by StepLR
    torch = pytest.importorskip("torch")
    start, interval, base = 5, 3, 0.5
    rng = np.random.default_rng(19)
    n = 64
    theta = rng.normal(size=n)
    tp = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.99), eps=1e-15)
    sch = torch.optim.lr_scheduler.SequentialLR(
        opt, [torch.optim.lr_scheduler.ConstantLR(opt, factor=1.0, total_iters=start),
              torch.optim.lr_scheduler.StepLR(opt, step_size=interval, gamma=base)], milestones=[start])
    mm, vv = np.zeros(n), np.zeros(n)
    for k in range(20):
        assert oracle.lr_at(1e-2, k, (start, interval, base)) == pytest.approx(opt.param_groups[0]["lr"], rel=1e-14)
        g = rng.normal(size=n)
        oracle.adam(theta, mm, vv, g, k + 1, oracle.lr_at(1e-2, k, (start, interval, base)), 0.9, 0.99, 1e-15)
        tp.grad = torch.tensor(g)
        opt.step()
        sch.step()
    np.testing.assert_allclose(theta, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------- sampler -----

def test_sampler_voxel_centres_affine_and_library():
    rng = np.random.default_rng(4)
    D = (7, 5, 6)  # x, y, z
    vol = rng.random((D[2], D[1], D[0])).astype(np.float32)
    # exact at voxel centres
    zz, yy, xx = np.meshgrid(*[np.arange(d) for d in D[::-1]], indexing="ij")
    ctr = np.stack([(xx + 0.5) / D[0], (yy + 0.5) / D[1], (zz + 0.5) / D[2]], -1).reshape(-1, 3).astype(np.float32)
    y = oracle.sample_volume(vol, ctr)
    # (i+1/2)/D is not binary32-exact for D=7: error bounded by slope * ulp
    np.testing.assert_allclose(y, vol.ravel().astype(np.float64), atol=1e-6)
    # power-of-two dims: voxel centres are exact in binary32, so the sample is exact
    D2 = (8, 4, 16)
    vol2 = rng.random((D2[2], D2[1], D2[0])).astype(np.float32)
    z2, y2, x2 = np.meshgrid(*[np.arange(d) for d in D2[::-1]], indexing="ij")
    c2 = np.stack([(x2 + 0.5) / D2[0], (y2 + 0.5) / D2[1], (z2 + 0.5) / D2[2]], -1).reshape(-1, 3)
    assert np.array_equal(oracle.sample_volume(vol2, c2.astype(np.float32)), vol2.ravel().astype(np.float64))
    # interior points: scipy trilinear on the cell-centre grid
    pts = rng.uniform(0.0, 1.0, (400, 3)).astype(np.float32)
    g = [(np.arange(d) + 0.5) / d for d in D]
    interp = RegularGridInterpolator((g[2], g[1], g[0]), vol.astype(np.float64), method="linear",
                                     bounds_error=False, fill_value=None)
    clamp = np.stack([np.clip(pts[:, a], g[a][0], g[a][-1]) for a in range(3)], -1)
    ref = interp(clamp[:, ::-1])
    np.testing.assert_allclose(oracle.sample_volume(vol, pts), ref, atol=1e-6)
    # affine volume is reproduced inside the centre hull
    a = np.array([0.2, -0.1, 0.3])
    lin = (a[0] * (xx + 0.5) / D[0] + a[1] * (yy + 0.5) / D[1] + a[2] * (zz + 0.5) / D[2]).astype(np.float32)
    inside = rng.uniform(0.2, 0.8, (200, 3)).astype(np.float32)
    np.testing.assert_allclose(oracle.sample_volume(lin, inside), inside.astype(np.float64) @ a, atol=1e-7)


# -------------------------------------------------------------- PSNR -----

def test_psnr_closed_form():
    # volume = 0.25 + 0.5 x; a one-level affine table reproduces it, the MLP
    # passes the feature through (positive values) and adds no bias.
    D = 16
    xs = (np.arange(D) + 0.5) / D
    vol = np.broadcast_to((0.25 + 0.5 * xs)[None, None, :], (D, D, D)).astype(np.float32).copy()
    N = 17
    m = oracle.Model(1, 1, 14, [N], 1, 1)
    delta = 1e-2
    v = np.arange(N) / (N - 1)
    vz, vy, vx = np.meshgrid(v, v, v, indexing="ij")
    params = np.zeros(m.n_params)
    params[:N ** 3] = (0.25 + 0.5 * vx + delta).ravel()
    params[m.n_table:] = [1.0, 1.0]  # W1 = [[1]], W_out = [[1]]
    mse = oracle.mse_grid(m, params, vol)
    assert oracle.psnr_from_mse(mse) == pytest.approx(-20 * math.log10(delta), abs=1e-5)


# ---------------------------------------------------------- renderer -----

def _const_model():
    m = oracle.Model(1, 1, 10, [5], 4, 1)
    return m, np.zeros(m.n_params)  # all weights 0 -> Phi = 0 everywhere


def test_ray_count_axis_aligned():
    # every pixel looks along +z through the cube: t in [1, 2], 1024 steps of 2^-10
    cam = np.array([0.3, 0.6, -1.0, 0, 0, 0, 0, 0, 0, 0, 0, 1], np.float32)
    for seed in range(5):
        n = oracle.ray_counts(cam, 8, 8, seed, 2.0 ** -10)
        assert np.all(n == 1024)
    cam_miss = np.array([1.5, 0.6, -1.0, 0, 0, 0, 0, 0, 0, 0, 0, 1], np.float32)
    assert np.all(oracle.ray_counts(cam_miss, 4, 4, 0, 2.0 ** -10) == 0)


def test_render_constant_alpha_closed_form():
    m, params = _const_model()
    lut = np.zeros((256, 4), np.float32)
    lut[:] = [0.2, 0.4, 0.8, 0.05]
    cam = np.array([0.3, 0.6, -1.0, 0, 0, 0, 0, 0, 0, 0, 0, 1], np.float32)
    rgba, ng, nu = oracle.render_pixels(m, params, cam, lut, 4, 4, 2.0 ** -10, 3, np.arange(16))
    n_stop = math.ceil(math.log(0.01) / math.log(0.95))
    assert n_stop == 90
    assert np.all(ng == 1024) and np.all(nu == n_stop)
    a = float(np.float32(0.05))  # the table holds binary32 alpha
    A = 1 - (1 - a) ** n_stop
    np.testing.assert_allclose(rgba[:, 3], A, rtol=1e-13)
    np.testing.assert_allclose(rgba[:, :3], np.broadcast_to(np.array([0.2, 0.4, 0.8], np.float32) * A, (16, 3)),
                               rtol=1e-7)
    # short rays (fewer samples than needed to stop): A = 1 - (1-a)^n
    cam2 = np.array([0.3, 0.6, 0.96, 0, 0, 0, 0, 0, 0, 0, 0, 1], np.float32)  # 40/1024 of the cube left
    rgba2, ng2, nu2 = oracle.render_pixels(m, params, cam2, lut, 2, 2, 2.0 ** -10, 0, np.arange(4))
    assert np.all(nu2 == ng2)
    for q in range(4):
        np.testing.assert_allclose(rgba2[q, 3], 1 - (1 - a) ** int(ng2[q]), rtol=1e-13)


def test_device_volume_generators_match_numpy():
    # the torch generators (used for the large batched targets) draw the same volumes
    torch = pytest.importorskip("torch")
    a = synth.gaussian_blobs(24, 3)
    b = synth.gaussian_blobs_torch(24, 3, "cpu", dtype=torch.float32, chunk=7).numpy()
    np.testing.assert_allclose(a, b, atol=2e-6)
    c = synth.fractal_value_noise(20, 5)
    d = synth.fractal_value_noise_torch(20, 5, "cpu", dtype=torch.float32, chunk=6).numpy()
    np.testing.assert_allclose(c, d, atol=2e-6)
    assert len(synth.multi_volume_specs()) == 16


# ------------------------------------------------------------ macro-cells -----

def test_mc_cells_voxel_centres_and_edges():
    # voxel centres fall in cell voxel // cell; the grid extends past a
    # volume that is not a multiple of the cell size; p = 1 is in the last cell
    dims, cell = (100, 64, 130), 64
    assert oracle.mc_grid(dims, cell) == (2, 1, 3)
    rng = np.random.default_rng(30)
    vox = np.stack([rng.integers(0, d, 500) for d in dims], 1)
    ctr = ((vox + 0.5) / np.array(dims)).astype(np.float32)
    M = oracle.mc_grid(dims, cell)
    c = vox // cell
    want = (c[:, 2] * M[1] + c[:, 1]) * M[0] + c[:, 0]
    np.testing.assert_array_equal(oracle.mc_cells(dims, cell, ctr), want)
    edge = np.array([[0, 0, 0], [1, 1, 1], [-0.5, 2.0, np.nan]], np.float32)
    np.testing.assert_array_equal(oracle.mc_cells(dims, cell, edge), [0, 5, 0])


def test_mc_update_matches_grouped_min_max():
    dims, cell = (64, 48, 80), 16
    rng = np.random.default_rng(31)
    xyz = rng.random((5000, 3)).astype(np.float32)
    v = rng.normal(size=5000).astype(np.float32)
    ids = oracle.mc_cells(dims, cell, xyz)
    n = int(np.prod(oracle.mc_grid(dims, cell)))
    lo, hi = np.full(n, np.inf), np.full(n, -np.inf)
    np.minimum.at(lo, ids, v.astype(np.float64))
    np.maximum.at(hi, ids, v.astype(np.float64))
    # in two batches: ranges carry over
    r = oracle.mc_update(dims, cell, xyz[:2000], v[:2000])
    r = oracle.mc_update(dims, cell, xyz[2000:], v[2000:], ranges=r)
    np.testing.assert_array_equal(r[0], lo)
    np.testing.assert_array_equal(r[1], hi)


def test_mc_opacity_is_max_of_interpolated_alpha():
    rng = np.random.default_rng(32)
    lut = rng.random((256, 4)).astype(np.float32)
    lut[:100, 3] = 0.0  # transparent below v = 100/255
    lut[180, 3] = 1.0   # a spike at a node
    nodes = np.arange(256) / 255.0
    lo = rng.random(300)
    hi = lo + rng.random(300) * 0.3
    lo[:3] = [0.1, 0.70, 0.7059]
    hi[:3] = [0.3, 0.72, 0.71]
    mu = oracle.mc_opacity((lo, hi), lut)
    for c in range(300):
        v = np.linspace(lo[c], hi[c], 4001)
        ref = max(np.interp(v, nodes, lut[:, 3]).max(),
                  max((lut[i, 3] for i in range(256) if lo[c] < nodes[i] < hi[c]), default=0.0))
        assert mu[c] == pytest.approx(ref, abs=2e-6), c
    assert mu[0] == 0.0 and mu[1] == 1.0 and mu[2] < 1.0
    # empty cells (no sample yet) are transparent
    assert oracle.mc_opacity((np.array([np.inf]), np.array([-np.inf])), lut)[0] == 0.0


def test_mc_skipping_invariants():
    m = small_model(L=3, F=2, log2T=10, res=(5, 9, 17), width=16, n_hidden=2)
    params = rand_params(m, seed=33, table_scale=0.5)
    cam = np.array([0.5, 0.5, -1.5, 0.002, 0, 0, 0, 0.002, 0, -0.064, -0.064, 1.0], np.float32)
    lut = np.random.default_rng(34).random((256, 4)).astype(np.float32) * 0.2
    W = H = 64
    pix = np.arange(W * H)
    dims, cell = (64, 64, 64), 16
    plain = oracle.render_pixels(m, params, cam, lut, W, H, 1 / 64, 7, pix)
    n = int(np.prod(oracle.mc_grid(dims, cell)))
    full = oracle.render_pixels_mc(m, params, cam, lut, W, H, 1 / 64, 7, pix, dims, cell, np.ones(n))
    for a, b in zip(plain, full):
        np.testing.assert_array_equal(a, b)
    empty = oracle.render_pixels_mc(m, params, cam, lut, W, H, 1 / 64, 7, pix, dims, cell, np.zeros(n))
    assert np.all(empty[0] == 0) and np.all(empty[2] == 0)
    np.testing.assert_array_equal(empty[1], plain[1])
    # skipping the cells with x >= 1/2 leaves the rays that stay in x < 1/2 unchanged
    mu = np.ones(n)
    M = oracle.mc_grid(dims, cell)
    ids = np.arange(n)
    mu[(ids % M[0]) >= M[0] // 2] = 0.0
    half = oracle.render_pixels_mc(m, params, cam, lut, W, H, 1 / 64, 7, pix, dims, cell, mu)
    left = (pix % W) < W // 2 - 2
    np.testing.assert_array_equal(half[0][left], plain[0][left])
    assert np.all(half[2] <= plain[2]) and np.any(half[2] < plain[2])


# ------------------------------------------------------- output ReLU -----
# Reading of Section 3.1 (ReLU activations for the MLP layers) and of the
# appendix's time-varying network listing (output activation ReLU): the
# output neuron may be followed by a ReLU, with ReLU'(0) = 0.

def test_output_relu_forward_equals_blas_chain():
    res = oracle.resolutions(16, 16, 0, 2048)
    m = oracle.Model(16, 2, 19, res, 64, 2, out_relu=True)
    m_lin = oracle.Model(16, 2, 19, res, 64, 2)
    rng = np.random.default_rng(40)
    W = rng.normal(size=m.n_mlp) * 0.2
    feat = rng.normal(size=(400, 32))
    W1 = W[:64 * 32].reshape(64, 32)
    W2 = W[64 * 32: 64 * 32 + 64 * 64].reshape(64, 64)
    W3 = W[64 * 32 + 64 * 64:].reshape(1, 64)
    z = (np.maximum(np.maximum(feat @ W1.T, 0) @ W2.T, 0) @ W3.T)[:, 0]
    assert (z < 0).sum() > 50 and (z > 0).sum() > 50  # both signs occur
    np.testing.assert_allclose(oracle.mlp_fwd(m, W, feat), np.maximum(z, 0), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.mlp_fwd(m_lin, W, feat), z, rtol=1e-13, atol=1e-13)


def test_output_relu_gradient_central_differences():
    m = oracle.Model(3, 2, 10, [5, 9, 17], 16, 2, out_relu=True)
    params = rand_params(m, seed=43)
    rng = np.random.default_rng(42)
    xyz = rng.random((64, 3)).astype(np.float32)
    y = rng.random(64) * 0.3
    out = oracle.forward(m, params, xyz)
    assert (out == 0).sum() > 5 and (out > 0).sum() > 5
    loss, g = oracle.loss_grad(m, params, xyz, y)
    assert loss == pytest.approx(float(np.mean((out - y) ** 2)), rel=1e-13)
    h = 1e-4
    checked = 0
    cand = list(range(0, m.n_table, 13)) + list(range(m.n_table, m.n_params))
    for i in cand:
        ls = []
        for k in (-2, -1, 0, 1, 2):
            p = params.copy()
            p[i] += k * h
            ls.append(float(np.mean((oracle.forward(m, p, xyz) - y) ** 2)))
        # piecewise quadratic: skip parameters where a ReLU (hidden or output)
        # changes state within +-2h (the second differences disagree)
        d2 = [ls[k + 1] - 2 * ls[k] + ls[k - 1] for k in (1, 2, 3)]
        if max(d2) - min(d2) > 1e-9 * max(1e-12, abs(ls[2])) + 1e-15:
            continue
        fd = (ls[3] - ls[1]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-11), i
        checked += 1
    assert checked > 0.7 * len(cand)


def test_output_relu_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    m = oracle.Model(3, 2, 10, [5, 9, 17], 16, 3, out_relu=True)
    params = rand_params(m, seed=43)
    rng = np.random.default_rng(44)
    xyz = rng.random((128, 3)).astype(np.float32)
    y = rng.random(128) * 0.3
    for loss_kind in ("l2", "l1"):
        _, g = oracle.loss_grad(m, params, xyz, y, loss=loss_kind)
        e = torch.tensor(oracle.encode(m, params, xyz), dtype=torch.float64)
        Ws = []
        pos = m.n_table
        for (o, i) in synth.mlp_shapes(m.n_in, m.width, m.n_hidden):
            Ws.append(torch.tensor(params[pos:pos + o * i].reshape(o, i), dtype=torch.float64, requires_grad=True))
            pos += o * i
        hh = e
        for W in Ws[:-1]:
            hh = torch.relu(torch.nn.functional.linear(hh, W))
        out = torch.relu(torch.nn.functional.linear(hh, Ws[-1])[:, 0])
        r = out - torch.tensor(y)
        loss = torch.mean(r ** 2) if loss_kind == "l2" else torch.mean(torch.abs(r))
        loss.backward()
        gm = np.concatenate([W.grad.numpy().ravel() for W in Ws])
        np.testing.assert_allclose(g[m.n_table:], gm, rtol=1e-12, atol=1e-15)


def test_output_relu_negative_outputs_give_zero_gradient():
    # every output's input negative: Phi = 0, loss = mean(y^2), and no
    # parameter receives any gradient
    m = oracle.Model(2, 2, 10, [5, 9], 8, 1, out_relu=True)
    params = np.zeros(m.n_params)
    params[:m.n_table] = 0.5                     # features 0.5 everywhere
    params[m.n_table:m.n_table + 8 * 4] = 1.0    # hidden = relu(sum) = 2
    params[m.n_table + 8 * 4:] = -1.0            # output input = -16
    xyz = np.random.default_rng(45).random((32, 3)).astype(np.float32)
    y = np.linspace(0.1, 0.9, 32)
    assert np.all(oracle.forward(m, params, xyz) == 0.0)
    loss, g = oracle.loss_grad(m, params, xyz, y)
    assert loss == pytest.approx(float(np.mean(y ** 2)), rel=1e-14)
    assert np.all(g == 0.0)


# ---------------------------------------------- renderer: shading -----

def _const_phi_model(c):
    # Phi = c everywhere: every table entry 1 (so every level feature is 1 by
    # the partition of unity), one hidden neuron with weight 1, output weight c
    m = oracle.Model(1, 1, 10, [5], 1, 1)
    params = np.zeros(m.n_params)
    params[:m.n_table] = 1.0
    params[m.n_table:] = [1.0, c]
    return m, params


def _ramp_lut():
    # distinct RGBA at every node, alpha increasing: a wrong node, a swapped
    # blend weight or an uncapped index all change the result
    i = np.arange(256, dtype=np.float64)
    return np.stack([i / 255, 1 - i / 255, 0.25 + 0.5 * (i % 7) / 6, 0.001 + 0.0002 * i], 1).astype(np.float32)


@pytest.mark.parametrize("c", [0.25, 0.6013, 0.999, 1.0, 1.7, -0.3])
def test_render_transfer_function_blend_closed_form(c):
    m, params = _const_phi_model(c)
    lut = _ramp_lut().astype(np.float64)
    cam = np.array([0.3, 0.6, -1.0, 0, 0, 0, 0, 0, 0, 0, 0, 1], np.float32)  # +z through the cube: 1024 samples
    rgba, ng, nu = oracle.render_pixels(m, params, cam, _ramp_lut(), 2, 2, 2.0 ** -10, 11, np.arange(4))
    v = min(max(c, 0.0), 1.0)
    u = 255.0 * v
    i0 = min(math.floor(u), 254)
    f = u - i0
    rgba_tf = (1 - f) * lut[i0] + f * lut[i0 + 1]   # linear interpolation between table nodes
    a = rgba_tf[3]
    n_stop = math.ceil(math.log(0.01) / math.log(1 - a))
    n = min(n_stop, 1024)
    assert np.all(ng == 1024) and np.all(nu == n)
    A = 1 - (1 - a) ** n          # identical samples: A_n = 1 - (1 - a)^n
    # Phi is c up to FP64 rounding of the partition of unity (1e-16), hence the atol
    np.testing.assert_allclose(rgba[:, 3], A, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(rgba[:, :3], np.broadcast_to(rgba_tf[:3] * A, (4, 3)), rtol=1e-11, atol=1e-13)


# --------------------------------------------- renderer: ray geometry -----

def _cam_axis(o, d):
    # every pixel's ray: origin o, direction d (du = dv = 0)
    return np.array(list(o) + [0, 0, 0, 0, 0, 0] + list(d), np.float32)


def test_ray_counts_negative_directions():
    dt = 2.0 ** -10
    for o, d in [((0.3, 0.6, 2.0), (0, 0, -1)), ((1.5, 0.25, 0.75), (-1, 0, 0)), ((0.5, 3.0, 0.5), (0, -1, 0))]:
        n = oracle.ray_counts(_cam_axis(o, d), 8, 8, 3, dt)
        assert np.all(n == 1024), (o, d)
    # the same rays pointing away from the cube miss it
    for o, d in [((0.3, 0.6, 2.0), (0, 0, 1)), ((1.5, 0.25, 0.75), (1, 0, 0))]:
        assert np.all(oracle.ray_counts(_cam_axis(o, d), 4, 4, 3, dt) == 0)


@pytest.mark.parametrize("sign", [1, -1])
def test_ray_counts_and_points_on_the_diagonal(sign):
    # the main diagonal, entered at one corner: chord sqrt(3), so
    # n = ceil(sqrt(3) * 1024 - j); samples lie on the diagonal at t_k
    dt = 2.0 ** -10
    o = (-0.5, -0.5, -0.5) if sign > 0 else (1.5, 1.5, 1.5)
    cam = _cam_axis(o, (sign, sign, sign))
    W = H = 16
    n = oracle.ray_counts(cam, W, H, 7, dt).ravel()
    q = math.sqrt(3.0) * 1024
    checked = 0
    for p in range(W * H):
        j = oracle.rng_u01(7, 5, p)
        want = math.ceil(q - j)
        if abs((q - j) - round(q - j)) < 1e-3:
            continue  # binary32 span rounding may decide these
        assert n[p] == want, p
        checked += 1
        if p % 37 == 0:
            pts = oracle.ray_points(cam, W, H, 7, dt, p, 0, 3).astype(np.float64)
            start = 0.0 if sign > 0 else 1.0
            for k in range(3):
                t_in = (k + j) * dt / math.sqrt(3.0)   # distance along each axis from the entry corner
                np.testing.assert_allclose(pts[k], start + sign * t_in, atol=2e-7)
    assert checked > 200


def test_ray_counts_oblique_against_exact_intersection():
    # pinhole camera looking at the cube from an oblique position; counts
    # against the exact FP64 slab intersection (pixels within 1e-3 of a
    # ceiling boundary are skipped)
    dt = 2.0 ** -10
    o = np.array([1.7, -0.4, -1.1])
    look = np.array([0.5, 0.5, 0.5]) - o
    fwd = look / np.linalg.norm(look)
    right = np.cross(fwd, [0.0, 1.0, 0.0])
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    W = H = 24
    s = math.tan(math.radians(20)) * 2 / H
    du, dv = right * s, -up * s
    d00 = fwd - du * W / 2 - dv * H / 2
    cam = np.concatenate([o, du, dv, d00]).astype(np.float32)
    n = oracle.ray_counts(cam, W, H, 9, dt).ravel()
    c32 = cam.astype(np.float64)
    checked = hits = 0
    for p in range(W * H):
        px, py = p % W, p // W
        d = c32[9:12] + (px + 0.5) * c32[3:6] + (py + 0.5) * c32[6:9]
        d /= np.linalg.norm(d)
        with np.errstate(divide="ignore"):
            inv = 1.0 / d
        t1, t2 = (0 - c32[:3]) * inv, (1 - c32[:3]) * inv
        tn, tf = max(np.max(np.minimum(t1, t2)), 0.0), np.min(np.maximum(t1, t2))
        j = oracle.rng_u01(9, 5, p)
        want = max(0, math.ceil((tf - tn) / dt - j)) if tn < tf else 0
        x = (tf - tn) / dt - j
        if tn < tf and abs(x - round(x)) < 1e-2:
            continue
        assert n[p] == want, p
        checked += 1
        hits += want > 0
    assert checked > 500 and hits > 100


# ------------------------------------------------ training loop wiring -----

def test_train_loop_equals_composed_steps():
    # oracle.train = for each step k: batch k (stream 3), trilinear targets,
    # loss gradient, Adam at t = k + 1 with the step-k learning rate.  Compose
    # the same from the individually pinned pieces, starting at step 3 with a
    # decay that changes the rate every step (a wrong step, rate or t index
    # changes the result).
    m = small_model(L=3, F=2, log2T=10, res=(5, 9, 17), width=16, n_hidden=2)
    params = rand_params(m, seed=46, table_scale=0.1)
    vol = synth.gaussian_blobs(12, 47)
    decay = (4, 1, 0.5)
    am, av = np.zeros(m.n_params), np.zeros(m.n_params)
    rng = np.random.default_rng(48)
    am[:] = rng.normal(size=m.n_params) * 1e-3   # state as after earlier steps
    av[:] = rng.random(m.n_params) * 1e-5
    got, (gm, gv), losses = oracle.train(m, params, vol, 5, 3, 200, 1e-2, 0.9, 0.99, 1e-15, step0=3,
                                         state=(am, av), loss="l1", l2_reg=1e-3, decay=decay)
    theta, mm, vv = params.copy(), am.copy(), av.copy()
    for s in range(3):
        k = 3 + s
        xyz = oracle.batch_coords(5, k, 200)
        y = oracle.sample_volume(vol, xyz)
        loss, g = oracle.loss_grad(m, theta, xyz, y, loss="l1")
        assert losses[s] == pytest.approx(loss, rel=1e-15)
        oracle.adam(theta, mm, vv, g, k + 1, oracle.lr_at(1e-2, k, decay), 0.9, 0.99, 1e-15, l2_reg=1e-3,
                    reg_from=m.n_table)
    np.testing.assert_array_equal(got, theta)
    np.testing.assert_array_equal(gm, mm)
    np.testing.assert_array_equal(gv, vv)
    # the rate of steps 3, 4, 5 is lr, lr/2, lr/4: the run is not the constant-rate one
    flat, _, _ = oracle.train(m, params, vol, 5, 3, 200, 1e-2, 0.9, 0.99, 1e-15, step0=3, state=(am, av),
                              loss="l1", l2_reg=1e-3)
    assert np.max(np.abs(flat - got)) > 1e-4


# ------------------------------------------- adaptive marching (Section 5.3) -----

def test_adaptive_step_closed_form():
    # sbar = max(1 + 63 |min(mu,1) - 1|^2, 1): 1 at mu >= 1, 64 at mu = 0
    assert oracle.adaptive_steps(1.0) == 1 and oracle.adaptive_steps(3.5) == 1
    assert oracle.adaptive_steps(0.0) == 64
    assert oracle.adaptive_steps(0.5) == 16       # 1 + 63/4 = 16.75
    assert oracle.adaptive_steps(0.5, p=1) == 32  # 1 + 63/2 = 32.5
    assert oracle.adaptive_steps(0.75, s2=9.0) == 1  # 1 + 8/16 = 1.5
    mus = np.linspace(0, 1.2, 241)
    steps = [oracle.adaptive_steps(float(u)) for u in mus]
    assert all(a >= b for a, b in zip(steps, steps[1:]))  # more opaque cells, smaller steps
    for u, n in zip(mus, steps):
        sb = max(1 + 63 * abs(min(u, 1) - 1) ** 2, 1)
        assert n == math.floor(sb) or abs(sb - round(sb)) < 1e-5


def _cells_by_scan(cam, W, seed, dt, pix, dims, cell):
    """Cell of every sample of a pixel's ray, from the sample points."""
    n = int(oracle.ray_counts(cam, W, max(1, pix // W + 1), seed, dt).ravel()[pix])
    pts = oracle.ray_points(cam, W, 1, seed, dt, pix, 0, n)
    return oracle.mc_cells(dims, cell, pts)


@pytest.mark.parametrize("o,d", [((0.3, 0.6, -1.0), (0, 0, 1)), ((0.4, 0.55, 2.0), (0, 0, -1)),
                                 ((-0.5, -0.5, -0.5), (1, 1, 1)), ((1.5, 1.4, 1.3), (-1, -1, -1)),
                                 ((-0.2, 0.3, 0.1), (1, 0.35, 0.2))])
def test_dda_traversal_equals_sample_scan(o, d):
    dt, dims, cell = 2.0 ** -10, (64, 48, 80), 16
    cam = np.array(list(o) + [0, 0, 0, 0, 0, 0] + list(d), np.float32)
    for seed in (1, 2, 3):
        lab = _cells_by_scan(cam, 1, seed, dt, 0, dims, cell)
        assert lab.size > 0
        starts = np.flatnonzero(np.r_[True, lab[1:] != lab[:-1]])
        cells, first = oracle.mc_traverse(cam, 1, seed, dt, 0, dims, cell, dda=True)
        np.testing.assert_array_equal(first, starts)
        np.testing.assert_array_equal(cells, lab[starts])
        c2, f2 = oracle.mc_traverse(cam, 1, seed, dt, 0, dims, cell, dda=False)
        np.testing.assert_array_equal(c2, cells)
        np.testing.assert_array_equal(f2, first)
        assert len(set(cells.tolist())) == len(cells)  # a convex cell is entered once


def test_dda_cell_sequence_on_an_axis_ray():
    # +z through a 64^3 volume with 16-voxel cells: cells change at z = 1/4,
    # 1/2, 3/4, i.e. at the first sample with (k + j) dt >= z - t_near
    dt, dims, cell = 2.0 ** -10, (64, 64, 64), 16
    cam = np.array([0.3, 0.6, -1.0, 0, 0, 0, 0, 0, 0, 0, 0, 1], np.float32)
    for seed in range(4):
        j = oracle.rng_u01(seed, 5, 0)
        cells, first = oracle.mc_traverse(cam, 1, seed, dt, 0, dims, cell)
        cx, cy = int(0.3 * 64) // 16, int(0.6 * 64) // 16
        np.testing.assert_array_equal(cells, [(cz * 4 + cy) * 4 + cx for cz in range(4)])
        np.testing.assert_array_equal(first, [0] + [math.ceil(z * 1024 - j) for z in (0.25, 0.5, 0.75)])


def test_adaptive_render_at_full_opacity_is_the_fixed_step_render():
    # mu >= 1 everywhere: one grid step per sample and no correction, so the
    # image is the fixed-step one bit for bit
    m = small_model(L=3, F=2, log2T=10, res=(5, 9, 17), width=16, n_hidden=2)
    params = rand_params(m, seed=50, table_scale=0.5)
    cam = np.array([0.5, 0.5, -1.5, 0.002, 0, 0, 0, 0.002, 0, -0.064, -0.064, 1.0], np.float32)
    lut = np.random.default_rng(51).random((256, 4)).astype(np.float32) * 0.2
    W = H = 48
    pix = np.arange(W * H)
    dims, cell = (64, 64, 64), 16
    n = int(np.prod(oracle.mc_grid(dims, cell)))
    plain = oracle.render_pixels(m, params, cam, lut, W, H, 1 / 64, 7, pix)
    ad = oracle.render_pixels_adaptive(m, params, cam, lut, W, H, 1 / 64, 7, pix, dims, cell, np.full(n, 1.5))
    for a, b in zip(plain, ad):
        np.testing.assert_array_equal(a, b)
    # every cell transparent: nothing is evaluated
    none = oracle.render_pixels_adaptive(m, params, cam, lut, W, H, 1 / 64, 7, pix, dims, cell, np.zeros(n))
    assert np.all(none[0] == 0) and np.all(none[2] == 0)
    np.testing.assert_array_equal(none[1], plain[1])


def test_adaptive_render_constant_alpha_closed_form():
    # constant Phi (constant alpha a per grid step) through cells whose mu
    # gives 16-step samples: the corrected opacities compose to the same
    # 1 - (1 - a)^n as n single steps; samples = one per 16 steps, restarted
    # at every cell boundary
    m, params = _const_phi_model(0.25)
    lut = np.zeros((256, 4), np.float32)
    lut[:] = [0.3, 0.5, 0.7, 0.001]
    dt, dims, cell = 2.0 ** -10, (64, 64, 64), 16
    nc = int(np.prod(oracle.mc_grid(dims, cell)))
    mu = np.full(nc, 0.5, np.float32)                   # 16 steps
    assert oracle.adaptive_steps(0.5) == 16
    cam = np.array([0.3, 0.6, -1.0, 0, 0, 0, 0, 0, 0, 0, 0, 1], np.float32)
    rgba, ng, nu = oracle.render_pixels_adaptive(m, params, cam, lut, 2, 2, dt, 5, np.arange(4), dims, cell, mu)
    a = float(np.float32(0.001))
    assert np.all(ng == 1024)
    np.testing.assert_allclose(rgba[:, 3], 1 - (1 - a) ** 1024, rtol=1e-12)
    rgb = np.array([0.3, 0.5, 0.7], np.float32).astype(np.float64)  # the table's binary32 colour
    np.testing.assert_allclose(rgba[:, :3], np.outer(np.full(4, 1 - (1 - a) ** 1024), rgb), rtol=1e-12)
    for q in range(4):
        cells, first = oracle.mc_traverse(cam, 2, 5, dt, q, dims, cell)
        seg = np.diff(np.r_[first, 1024])
        assert nu[q] == int(np.sum(np.ceil(seg / 16)))
