"""GPU parity, continued: the output-ReLU option, the rendering
configuration the benchmark times, batched graph-captured training, the
trained-model BF16 bound, the device PSNR and graph-replayed training after a
skipped step.  Same bars as test_gpu_parity.py: FP32 outputs <= 1e-5, FP32
gradients <= 1e-4 (normwise, per block), BF16-MFMA outputs <= 2e-2 absolute.
"""
import functools

import numpy as np
import pytest

import oracle
import synth
from models import SEED, edge_coords, gpu_plan, init_params, oracle_model, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ngv = pytest.importorskip("paper_2207_11620_amd")


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ngv.lib()
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _blocks(m):
    out = [(f"table{l}", slice(int(m.level_offset[l]) * m.F, int(m.level_offset[l + 1]) * m.F)) for l in range(m.L)]
    pos = m.n_table
    for i, (o, k) in enumerate(synth.mlp_shapes(m.n_in, m.width, m.n_hidden)):
        out.append((f"W{i}", slice(pos, pos + o * k)))
        pos += o * k
    return out


# -------------------------------------------------------- output ReLU -----

@pytest.mark.parametrize("name,prec", [("tiny", "fp32"), ("cfg1", "fp32"), ("cfg1", "bf16"), ("w32k64", "fp32")])
def test_output_relu_forward(name, prec):
    m = oracle_model(name, out_relu=True)
    p = gpu_plan(name, prec, out_relu=True)
    params = init_params(name, table_scale=0.3)
    xyz = edge_coords(5003, seed=60)
    ref = oracle.forward(m, params.astype(np.float64), xyz)
    assert np.mean(ref == 0) > 0.05 and np.mean(ref > 0) > 0.05
    out = host(ngv.infer(p, dev(params), dev(xyz), sort=False))
    if prec == "fp32":
        assert rel_err(out, ref) <= 1e-5
    else:
        assert np.max(np.abs(out - ref)) <= 2e-2
    assert np.all(out >= 0)


@pytest.mark.parametrize("name", ["tiny", "cfg1"])
def test_output_relu_train_step_gradient(name):
    # Adam's first moment after one step from zero is (1 - beta1) g
    m = oracle_model(name, out_relu=True)
    p = gpu_plan(name, "fp32", out_relu=True)
    params = init_params(name, table_scale=0.3)
    vol = synth.gaussian_blobs(32, SEED)
    B = 4096 + 77
    xyz = oracle.batch_coords(SEED, 3, B)
    y = oracle.sample_volume(vol, xyz)
    st = ngv.TrainState(p, dev(params), B)
    ngv.train_step(st, volume=dev(vol), seed=SEED, step_index=3, loss_scale=128.0)
    g = host(st.m).astype(np.float64) / (1 - np.float32(0.9))
    _, g_ref = oracle.loss_grad(m, params.astype(np.float64), xyz, y)
    for bname, sl in _blocks(m):
        if np.max(np.abs(g_ref[sl])) > 0:
            assert rel_err(g[sl], g_ref[sl]) <= 1e-4, bname


def test_output_relu_autograd_function():
    # the standalone backward masks d_out where the output's input was <= 0
    name = "cfg1"
    m = oracle_model(name, out_relu=True)
    p = gpu_plan(name, "fp32", out_relu=True)
    params = init_params(name, table_scale=0.3)
    B = 3001
    xyz = edge_coords(B, seed=61)
    y = np.random.default_rng(62).random(B).astype(np.float32) * 0.2
    _, g_ref = oracle.loss_grad(m, params.astype(np.float64), xyz, y.astype(np.float64))
    pt = dev(params).requires_grad_(True)
    out = ngv.volume(p, pt, dev(xyz))
    loss = ((out - dev(y)) ** 2).mean()
    loss.backward()
    g = host(pt.grad).astype(np.float64)
    for bname, sl in _blocks(m):
        if np.max(np.abs(g_ref[sl])) > 0:
            assert rel_err(g[sl], g_ref[sl]) <= 1e-4, bname


# --------------------------------------- the benchmark's render config -----

@functools.lru_cache(maxsize=1)
def _render_model():
    # the query model (16 levels, 2^19, 32-64-64-1) fitted for 30 steps by the
    # oracle to a fractal-noise target, so the transfer function sees real values
    name = "cfg1"
    m = oracle_model(name)
    vol = synth.fractal_value_noise(48, SEED)
    th, _, _ = oracle.train(m, init_params(name).astype(np.float64), vol, SEED, 30, 4096, 1e-2, 0.9, 0.99, 1e-15)
    return m, th.astype(np.float32), vol


@pytest.mark.parametrize("skip", [False, True])
def test_render_bench_configuration_matches_oracle(skip):
    # BF16 MLP, FP16 tables, step 2^-10, 256^2 frame, 300 sampled pixels
    m, params, vol = _render_model()
    p = gpu_plan("cfg1", "bf16")
    pt = dev(params)
    f16 = ngv.make_f16_tables(p, pt)
    q = params.astype(np.float64)
    q[:m.n_table] = params[:m.n_table].astype(np.float16).astype(np.float64)  # the gathered FP16 values
    W = H = 256
    cam = synth.orbit_camera(0.6, W, H)
    lut = synth.transfer_function_lut().copy()
    dt = 2.0 ** -10
    mc, mu_o, dims, cell = None, None, (48, 48, 48), 8
    if skip:
        lut[:103, 3] = 0.0  # transparent below v = 0.4
        xyz = oracle.batch_coords(SEED, 0, 1 << 16)
        y = oracle.sample_volume(vol, xyz).astype(np.float32)
        mc = ngv.MacroCells(dims, cell)
        mc.update(dev(xyz), dev(y))
        mc.opacity(dev(lut))
        mu_o = oracle.mc_opacity(oracle.mc_update(dims, cell, xyz, y), lut)
        assert np.any(mu_o == 0)
    rgba, n_geo, n_used, cnt = ngv.render(p, pt, cam, dev(lut), W, H, dt, 9, table_f16=f16, macrocells=mc)
    np.testing.assert_array_equal(host(n_geo).astype(np.uint32), oracle.ray_counts(cam, W, H, 9, dt))
    img, nu = host(rgba).reshape(-1, 4), host(n_used).ravel()
    hit = np.flatnonzero(host(n_geo).ravel() > 0)
    pix = np.random.default_rng(3).choice(hit, 300, replace=False)
    if skip:
        ro, _, nuo = oracle.render_pixels_mc(m, q, cam, lut, W, H, dt, 9, pix, dims, cell, mu_o)
    else:
        ro, _, nuo = oracle.render_pixels(m, q, cam, lut, W, H, dt, 9, pix)
    same = nu[pix] == nuo
    assert np.mean(same) > 0.9
    assert np.all(same | (np.abs(ro[:, 3] - 0.99) < 2e-2))
    assert np.max(np.abs(img[pix][same] - ro[same])) <= 2e-2
    assert host(cnt)[1] == nu.sum()


@pytest.mark.parametrize("prec,s2,pexp", [("fp32", 64.0, 2), ("bf16", 64.0, 2), ("fp32", 16.0, 1), ("fp32", 200.0, 5)])
def test_render_adaptive_matches_oracle(prec, s2, pexp):
    # adaptive marching through macro-cells of known binary32 opacities (the
    # oracle's, copied to the device): the walk is integer work (cell
    # indices, step counts, DDA exits), so the evaluated-sample counts agree
    # exactly except where termination at A = 0.99 is a rounding tie
    m, params, vol = _render_model()
    p = gpu_plan("cfg1", prec)
    pt = dev(params)
    W = H = 192
    cam = synth.orbit_camera(0.9, W, H)
    lut = synth.transfer_function_lut().copy()
    lut[:103, 3] = 0.0
    dt = 2.0 ** -9
    dims, cell = (48, 48, 48), 8
    xyz = oracle.batch_coords(SEED, 0, 1 << 16)
    y = oracle.sample_volume(vol, xyz).astype(np.float32)
    mu_o = oracle.mc_opacity(oracle.mc_update(dims, cell, xyz, y), lut).astype(np.float32)
    assert np.any(mu_o == 0) and np.any((mu_o > 0) & (mu_o < 0.9))
    mc = ngv.MacroCells(dims, cell)
    mc.mu.copy_(dev(mu_o))
    rgba, n_geo, n_used, cnt = ngv.render(p, pt, cam, dev(lut), W, H, dt, 5, macrocells=mc, adaptive=True,
                                          step_max=s2, step_exp=pexp)
    _, _, nu_skip, cnt_skip = ngv.render(p, pt, cam, dev(lut), W, H, dt, 5, macrocells=mc)
    np.testing.assert_array_equal(host(n_geo).astype(np.uint32), oracle.ray_counts(cam, W, H, 5, dt))
    img, nu = host(rgba).reshape(-1, 4), host(n_used).ravel()
    c, cs = host(cnt), host(cnt_skip)
    print(f"evaluated: adaptive {c[0]}, skipping only {cs[0]}")
    assert c[0] < cs[0]
    assert c[1] == nu.sum()
    hit = np.flatnonzero(host(n_geo).ravel() > 0)
    pix = np.random.default_rng(4).choice(hit, 300, replace=False)
    ro, _, nuo = oracle.render_pixels_adaptive(m, params.astype(np.float64), cam, lut, W, H, dt, 5, pix, dims, cell,
                                               mu_o, s2, pexp)
    same = nu[pix] == nuo
    assert np.mean(same) > 0.9
    assert np.all(same | (np.abs(ro[:, 3] - 0.99) < 2e-2))
    tol = 1e-4 if prec == "fp32" else 2e-2
    assert np.max(np.abs(img[pix][same] - ro[same])) <= tol


@functools.lru_cache(maxsize=1)
def _render_model_table2():
    name = "paper"
    m = oracle_model(name)
    vol = synth.fractal_value_noise(48, SEED)
    th, _, _ = oracle.train(m, init_params(name).astype(np.float64), vol, SEED, 30, 4096, 1e-2, 0.9, 0.99, 1e-15)
    return m, th.astype(np.float32), vol


@pytest.mark.parametrize("adaptive", [False, True])
def test_render_macrocells_table2_network(adaptive):
    # skipping and adaptive marching in the renderer's 64-input, four-hidden-
    # layer instantiation (the Table-2 network), FP32, against the oracle
    m, params, vol = _render_model_table2()
    p = gpu_plan("paper", "fp32")
    pt = dev(params)
    W = H = 128
    cam = synth.orbit_camera(0.4, W, H)
    lut = synth.transfer_function_lut().copy()
    lut[:103, 3] = 0.0
    dt = 2.0 ** -9
    dims, cell = (48, 48, 48), 8
    xyz = oracle.batch_coords(SEED, 2, 1 << 16)
    y = oracle.sample_volume(vol, xyz).astype(np.float32)
    mu_o = oracle.mc_opacity(oracle.mc_update(dims, cell, xyz, y), lut).astype(np.float32)
    assert np.any(mu_o == 0)
    mc = ngv.MacroCells(dims, cell)
    mc.mu.copy_(dev(mu_o))
    rgba, n_geo, n_used, cnt = ngv.render(p, pt, cam, dev(lut), W, H, dt, 6, macrocells=mc, adaptive=adaptive)
    np.testing.assert_array_equal(host(n_geo).astype(np.uint32), oracle.ray_counts(cam, W, H, 6, dt))
    img, nu = host(rgba).reshape(-1, 4), host(n_used).ravel()
    hit = np.flatnonzero(host(n_geo).ravel() > 0)
    pix = np.random.default_rng(9).choice(hit, 200, replace=False)
    q = params.astype(np.float64)
    if adaptive:
        ro, _, nuo = oracle.render_pixels_adaptive(m, q, cam, lut, W, H, dt, 6, pix, dims, cell, mu_o, 64.0, 2)
    else:
        ro, _, nuo = oracle.render_pixels_mc(m, q, cam, lut, W, H, dt, 6, pix, dims, cell, mu_o)
    same = nu[pix] == nuo
    assert np.mean(same) > 0.9
    assert np.all(same | (np.abs(ro[:, 3] - 0.99) < 2e-2))
    assert np.max(np.abs(img[pix][same] - ro[same])) <= 1e-4
    assert host(cnt)[1] == nu.sum()


def test_render_adaptive_degenerate_grids():
    # opacity >= 1 everywhere, or s2 = 1: every step is one grid step, so the
    # adaptive walk evaluates exactly the samples of the fixed-step marcher
    # (with the same skipping) and the images agree bit for bit
    m, params, vol = _render_model()
    p = gpu_plan("cfg1", "fp32")
    pt = dev(params)
    W, H = 128, 96
    cam = synth.orbit_camera(0.3, W, H)
    lut = dev(synth.transfer_function_lut())
    dt = 2.0 ** -8
    mc = ngv.MacroCells((48, 48, 48), 8)
    mc.mu.fill_(1.0)
    a, _, na, _ = ngv.render(p, pt, cam, lut, W, H, dt, 3, macrocells=mc, adaptive=True)
    b, _, nb, _ = ngv.render(p, pt, cam, lut, W, H, dt, 3)
    np.testing.assert_array_equal(host(a), host(b))
    np.testing.assert_array_equal(host(na), host(nb))
    g = np.random.default_rng(5).random(mc.mu.numel()).astype(np.float32)
    g[g < 0.3] = 0.0
    mc.mu.copy_(dev(g))
    a, _, na, _ = ngv.render(p, pt, cam, lut, W, H, dt, 3, macrocells=mc, adaptive=True, step_max=1.0)
    b, _, nb, _ = ngv.render(p, pt, cam, lut, W, H, dt, 3, macrocells=mc)
    np.testing.assert_array_equal(host(a), host(b))
    np.testing.assert_array_equal(host(na), host(nb))


def test_render_ex_rejects_bad_options():
    m, params, vol = _render_model()
    p = gpu_plan("cfg1", "fp32")
    pt = dev(params)
    lut = dev(synth.transfer_function_lut())
    cam = synth.orbit_camera(0.3, 32, 32)
    mc = ngv.MacroCells((48, 48, 48), 8)
    with pytest.raises(ValueError):
        ngv.render(p, pt, cam, lut, 32, 32, 2.0 ** -8, 3, adaptive=True)
    for kw in ({"step_max": 0.5}, {"step_exp": 0}, {"step_exp": 9}):
        with pytest.raises(RuntimeError):
            ngv.render(p, pt, cam, lut, 32, 32, 2.0 ** -8, 3, macrocells=mc, adaptive=True, **kw)


# -------------------------------------------- 16 models in one graph -----

def test_multi_model_training_graph_matches_eager():
    # the training steps of 16 models of different levels and table sizes,
    # captured in one graph and replayed, against per-model eager steps
    specs = synth.multi_volume_specs(16)
    plans, params, vols = [], [], []
    for i, sp in enumerate(specs):
        p = ngv.Plan(sp["L"], 2, sp["log2T"], 16, 0.0, 2048, n_neurons=64, n_hidden_layers=2, precision="bf16")
        plans.append(p)
        params.append(dev(synth.init_params(p.n_table_params, p.n_input, 64, 2, 0.05, sp["seed"])))
        v = synth.gaussian_blobs(24, sp["seed"]) if i % 2 == 0 else synth.fractal_value_noise(24, sp["seed"])
        vols.append(dev(v.astype(np.float16)))
    B, steps = 4096, 3
    eager = [ngv.TrainState(p, w, B, f16_tables=True) for p, w in zip(plans, params)]
    for k in range(steps):
        for st, v in zip(eager, vols):
            ngv.train_step(st, volume=v, seed=SEED, step_index=k, loss_scale=128.0)
    cap = [ngv.TrainState(p, w, B, f16_tables=True) for p, w in zip(plans, params)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for st, v in zip(cap, vols):
            ngv.train_step(st, volume=v, seed=SEED, step_index=-1, loss_scale=128.0)  # step 0, eager
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for st, v in zip(cap, vols):
            ngv.train_step(st, volume=v, seed=SEED, step_index=-1, loss_scale=128.0)
    for _ in range(steps - 1):
        g.replay()
        torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(cap, eager)):
        assert host(a.step)[0] == steps and host(a.draws)[0] == steps, i
        d = np.abs(host(a.params) - host(b.params))
        assert np.quantile(d, 0.999) <= 1e-5, i
        assert host(a.loss)[0] == pytest.approx(host(b.loss)[0], rel=1e-3), i
        np.testing.assert_array_equal(host(a.table_f16), host(a.params[:plans[i].n_table_params].half()))


def test_multi_train_step_forked_and_graphed_matches_eager():
    # ngvol_multi_train_step: the 16 models' steps forked over the group's
    # streams, eagerly and captured in one graph (parallel branches), against
    # per-model eager steps
    specs = synth.multi_volume_specs(16)
    plans, params, vols = [], [], []
    for i, sp in enumerate(specs):
        p = ngv.Plan(sp["L"], 2, sp["log2T"], 16, 0.0, 2048, n_neurons=64, n_hidden_layers=2, precision="bf16")
        plans.append(p)
        params.append(dev(synth.init_params(p.n_table_params, p.n_input, 64, 2, 0.05, sp["seed"])))
        v = synth.gaussian_blobs(24, sp["seed"]) if i % 2 == 0 else synth.fractal_value_noise(24, sp["seed"])
        vols.append(dev(v.astype(np.float16)))
    seeds = [SEED + i for i in range(16)]
    B, steps = 4096, 4
    eager = [ngv.TrainState(p, w, B, f16_tables=True) for p, w in zip(plans, params)]
    for k in range(steps):
        for st, v, sd in zip(eager, vols, seeds):
            ngv.train_step(st, volume=v, seed=sd, step_index=k, loss_scale=128.0)
    grp = ngv.Multi(plans)
    forked = [ngv.TrainState(p, w, B, f16_tables=True) for p, w in zip(plans, params)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        grp.train_step(forked, vols, seeds, step_index=-1, loss_scale=128.0)   # step 0, eager
        grp.train_step(forked, vols, seeds, step_index=-1, loss_scale=128.0)   # step 1, eager
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        grp.train_step(forked, vols, seeds, step_index=-1, loss_scale=128.0)
    for _ in range(steps - 2):
        g.replay()
        torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(forked, eager)):
        assert host(a.step)[0] == steps and host(a.draws)[0] == steps, i
        d = np.abs(host(a.params) - host(b.params))
        assert np.quantile(d, 0.999) <= 1e-5, i
        assert host(a.loss)[0] == pytest.approx(host(b.loss)[0], rel=1e-3), i
    # a state given twice is refused before anything runs
    with pytest.raises(RuntimeError):
        grp.train_step([forked[0]] * 16, vols, seeds)


# --------------------------------------------- trained-model BF16 bound -----

def test_bf16_trained_model_within_2e2_absolute():
    # the oracle fits the tiny model (100 steps, the tiny workload); BF16-MFMA
    # inference with FP16 tables on every 64^3 voxel centre stays within 2e-2
    # absolute of the FP64 oracle on the trained model's [0,1] values
    name = "tiny"
    m = oracle_model(name)
    vol = synth.gaussian_blobs(64, SEED)
    th, _, _ = oracle.train(m, init_params(name).astype(np.float64), vol, SEED, 100, 4096, 1e-2, 0.9, 0.99, 1e-15)
    D = 64
    c = (np.arange(D, dtype=np.float32) + 0.5) / D
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    xyz = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.float32)
    ref = oracle.forward(m, th, xyz)
    assert ref.min() > -0.2 and ref.max() < 1.2  # a fitted [0,1] volume
    p = gpu_plan(name, "bf16")
    pt = dev(th.astype(np.float32))
    out = host(ngv.infer(p, pt, dev(xyz), table_f16=ngv.make_f16_tables(p, pt)))
    err = np.max(np.abs(out - ref))
    print(f"BF16 + FP16 tables vs FP64 oracle on the trained tiny model: max abs {err:.3e}")
    assert err <= 2e-2


# ---------------------------------------------------------------- PSNR -----

@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_psnr_matches_oracle(prec):
    name = "tiny"
    m = oracle_model(name)
    vol = synth.gaussian_blobs(40, SEED)
    th, _, _ = oracle.train(m, init_params(name).astype(np.float64), vol, SEED, 40, 4096, 1e-2, 0.9, 0.99, 1e-15)
    mse_o = oracle.mse_grid(m, th, vol)
    p = gpu_plan(name, prec)
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    ps = ngv.psnr(p, dev(th.astype(np.float32)), dev(vol), out=out)
    mse_g = float(host(out)[0])
    assert ps == pytest.approx(-10 * np.log10(mse_g), abs=1e-9)  # the device finish
    if prec == "fp32":
        assert mse_g == pytest.approx(mse_o, rel=1e-3)
        assert ps == pytest.approx(oracle.psnr_from_mse(mse_o), abs=5e-3)
    else:
        assert abs(ps - oracle.psnr_from_mse(mse_o)) <= 0.5
    # an FP16 volume gives the same result as its FP32 values
    v16 = vol.astype(np.float16)
    a = ngv.psnr(p, dev(th.astype(np.float32)), dev(v16))
    b = ngv.psnr(p, dev(th.astype(np.float32)), dev(v16.astype(np.float32)))
    assert a == pytest.approx(b, abs=1e-9)


# ----------------------------------- graph-replayed steps after a skip -----

def test_skipped_step_advances_the_draw_counter():
    # a step whose targets are NaN is skipped; the next step of a
    # graph-replayable run (step_index -1) draws batch 1, not batch 0 again
    p = gpu_plan("tiny", "fp32")
    params = dev(init_params("tiny", table_scale=0.2))
    vol = dev(synth.gaussian_blobs(32, SEED))
    bad = torch.full_like(vol, float("nan"))
    a = ngv.TrainState(p, params, 4096)
    ngv.train_step(a, volume=bad, seed=SEED, step_index=-1, loss_scale=128.0)
    assert host(a.skipped)[0] == 1 and host(a.step)[0] == 0 and host(a.draws)[0] == 1
    assert np.array_equal(host(a.params), host(params)) and np.all(host(a.grad) == 0)
    ngv.train_step(a, volume=vol, seed=SEED, step_index=-1, loss_scale=128.0)
    assert host(a.skipped)[0] == 0 and host(a.step)[0] == 1 and host(a.draws)[0] == 2
    b = ngv.TrainState(p, params, 4096)
    ngv.train_step(b, volume=vol, seed=SEED, step_index=1, loss_scale=128.0)
    assert host(a.loss)[0] == pytest.approx(host(b.loss)[0], rel=1e-12)
    d = np.abs(host(a.params) - host(b.params))
    assert np.quantile(d, 0.999) <= 1e-6
