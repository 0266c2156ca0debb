"""GPU parity of the shadow ray marcher and the path tracer (ngvol_render_ex
modes RM_SHADOW and PT) against the oracle's renderers.

The shading point of a shadow ray is an argmax over floating-point
contributions, and a path's real/null and roulette decisions compare floating
point values with random numbers.  Where the GPU's FP32 or BF16 network and
the FP64 oracle straddle such a threshold, both results are correct readings
of the method but differ.  So the tests compare what is unique: pixels whose
shading point (shadow) or whose real and tentative collision counts (path
tracing) agree must match the oracle within the output bar (FP32 1e-4,
BF16 2e-2); a differing shading point must be a near-maximum of the
contributions; and closed forms (white furnace, empty medium) hold exactly.
"""
import functools

import numpy as np
import pytest

import oracle
import synth
from models import SEED, gpu_plan, init_params, oracle_model

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


@functools.lru_cache(maxsize=3)
def _fitted(name):
    # a model fitted by the oracle to a blob volume: real structure for the
    # transfer function, the shadows and the medium
    m = oracle_model(name)
    vol = synth.gaussian_blobs(48, SEED)
    th, _, _ = oracle.train(m, init_params(name).astype(np.float64), vol, SEED, 40, 4096, 1e-2, 0.9, 0.99, 1e-15)
    return m, th.astype(np.float32)


def _contributions(m, params, cam, lut, W, H, seed, dt, q, n):
    # contributions (1 - A_{k-1}) alpha_k of the first n samples of pixel q,
    # from the oracle's network at the binary32 sample points
    pts = oracle.ray_points(cam, W, H, seed, dt, q, 0, n)
    phi = oracle.forward(m, params.astype(np.float64), pts)
    lut = lut.astype(np.float64)
    v = np.clip(phi, 0, 1)
    u = 255 * v
    i0 = np.minimum(np.floor(u), 254).astype(int)
    f = u - i0
    a = (1 - f) * lut[i0, 3] + f * lut[i0 + 1, 3]
    w, A = np.zeros(n), 0.0
    for k in range(n):
        w[k] = (1 - A) * a[k]
        A += w[k]
    return w


@pytest.mark.parametrize("name,prec,use_mc", [("tiny", "fp32", False), ("tiny", "fp32", True), ("tiny", "bf16", False),
                                              ("cfg1", "bf16", False), ("paper", "fp32", False)])
def test_shadow_matches_oracle(name, prec, use_mc):
    m, params = _fitted(name)
    p = gpu_plan(name, prec)
    pt = dev(params)
    W, H = 96, 72
    cam = synth.orbit_camera(0.8, W, H)
    lut = synth.transfer_function_lut().copy()
    lut[:60, 3] = 0.0
    dt = 2.0 ** -8
    light = (0.4, 0.9, -0.3)
    mc, mu, dims, cell = None, None, (48, 48, 48), 8
    if use_mc:
        xyz = oracle.batch_coords(SEED, 0, 1 << 16)
        y = oracle.forward(m, params.astype(np.float64), xyz).astype(np.float32)
        mu = oracle.mc_opacity(oracle.mc_update(dims, cell, xyz, y), lut)
        assert np.any(mu == 0) and np.any(mu > 0)
        mc = ngv.MacroCells(dims, cell)
        mc.mu.copy_(dev(mu.astype(np.float32)))
    aux = torch.empty((H, W), dtype=torch.int32, device="cuda")
    rgba, n_geo, n_used, cnt = ngv.render(p, pt, cam, dev(lut), W, H, dt, 5, macrocells=mc, mode="rm_shadow",
                                          light=light, aux=aux)
    ks = host(aux).ravel().view(np.uint32)
    img, nu = host(rgba).reshape(-1, 4), host(n_used).ravel()
    np.testing.assert_array_equal(host(n_geo).ravel().astype(np.uint32), oracle.ray_counts(cam, W, H, 5, dt).ravel())
    hit = np.flatnonzero(host(n_geo).ravel() > 0)
    pix = np.random.default_rng(6).choice(hit, 160, replace=False)
    ro, _, nuo, kso = oracle.render_pixels_shadow(m, params.astype(np.float64), cam, lut, W, H, dt, 5, pix, light,
                                                  dims, cell, mu)
    same_k = ks[pix] == kso
    same_n = nu[pix] == nuo
    print(f"shading point agrees on {same_k.mean():.3f}, sample count on {same_n.mean():.3f}")
    assert np.mean(same_k & same_n) > (0.9 if prec == "fp32" else 0.6)
    tol = 1e-4 if prec == "fp32" else 2e-2
    ok = same_k & same_n
    assert np.max(np.abs(img[pix][ok] - ro[ok])) <= tol
    # the alpha channel does not depend on the shading point
    assert np.max(np.abs(img[pix][same_n, 3] - ro[same_n, 3])) <= tol
    # a differing shading point is a near-maximum of the contributions
    if not use_mc:
        for i in np.flatnonzero(~same_k & same_n):
            q = int(pix[i])
            w = _contributions(m, params, cam, lut, W, H, 5, dt, q, int(nu[q]))
            assert ks[q] < w.size and w[ks[q]] >= (1 - (1e-3 if prec == "fp32" else 0.1)) * w.max()
    assert host(cnt)[1] == nu.sum()


def test_shadow_all_transparent_and_no_light_change():
    # nothing visible: no shading point, black pixels; and the RM_SHADOW
    # primary pass equals the plain marcher wherever the shadow is clear
    m, params = _fitted("tiny")
    p = gpu_plan("tiny", "fp32")
    pt = dev(params)
    W, H = 64, 48
    cam = synth.orbit_camera(0.8, W, H)
    lut = np.zeros((256, 4), np.float32)
    aux = torch.empty((H, W), dtype=torch.int32, device="cuda")
    rgba, _, nu, _ = ngv.render(p, pt, cam, dev(lut), W, H, 2.0 ** -8, 5, mode="rm_shadow", light=(0, 1, 0), aux=aux)
    assert np.all(host(rgba) == 0) and np.all(host(aux).view(np.uint32) == 0xFFFFFFFF)
    lut = synth.transfer_function_lut()
    a, _, na, _ = ngv.render(p, pt, cam, dev(lut), W, H, 2.0 ** -8, 5, mode="rm_shadow", light=(0, 1, 0))
    b, _, nb, _ = ngv.render(p, pt, cam, dev(lut), W, H, 2.0 ** -8, 5)
    a, b = host(a), host(b)
    np.testing.assert_array_equal(host(na), host(nb))
    np.testing.assert_array_equal(a[..., 3], b[..., 3])
    T = np.where(b[..., :3] > 0, a[..., :3] / np.where(b[..., :3] > 0, b[..., :3], 1), 1)
    assert np.all(T <= 1 + 1e-6) and np.all(T >= 0)


def _pt_args(**kw):
    a = dict(mode="pt", light=(0.4, 0.9, -0.3), radiance=(8.0, 8.0, 8.0), background=(0.1, 0.2, 0.3), density=40.0,
             spp=4, rr_depth=4, max_depth=64)
    a.update(kw)
    return a


def _pt_lut():
    # the shading colours with an opacity ramp that makes the blobs a dense
    # medium (extinction up to density) and leaves low values empty
    lut = synth.transfer_function_lut().copy()
    v = np.arange(256) / 255.0
    lut[:, 3] = np.clip((v - 0.15) / 0.5, 0.0, 1.0)
    return lut


@pytest.mark.parametrize("name,use_mc", [("tiny", False), ("tiny", True), ("paper", False)])
def test_pt_matches_oracle_fp32(name, use_mc):
    # FP32 network: decisions agree almost everywhere; where a pixel's real
    # and tentative collision counts agree, its radiance matches (the
    # Table-2 network: 64 input features, four hidden layers)
    m, params = _fitted(name)
    p = gpu_plan(name, "fp32")
    pt = dev(params)
    W, H = 48, 40
    cam = synth.orbit_camera(1.3, W, H)
    lut = _pt_lut()
    mc, mu, dims, cell = None, None, (48, 48, 48), 8
    if use_mc:
        xyz = oracle.batch_coords(SEED, 1, 1 << 16)
        y = oracle.forward(m, params.astype(np.float64), xyz).astype(np.float32)
        mu = oracle.mc_opacity(oracle.mc_update(dims, cell, xyz, y), lut).astype(np.float32)
        mc = ngv.MacroCells(dims, cell)
        mc.mu.copy_(dev(mu))
    a = _pt_args()
    rgba, n_real, n_samp, cnt = ngv.render(p, pt, cam, dev(lut), W, H, 1.0, 11, macrocells=mc, **a)
    img, nr, ns = host(rgba).reshape(-1, 4), host(n_real).ravel(), host(n_samp).ravel()
    c = host(cnt)
    assert c[2] == W * H * a["spp"] and c[0] == ns.sum() and c[1] == nr.sum()
    pix = np.random.default_rng(8).choice(W * H, 200, replace=False)
    ro, nro, nso = oracle.render_pixels_pt(m, params.astype(np.float64), cam, lut, W, H, 11, pix, a["density"],
                                           a["light"], a["radiance"], a["background"], spp=a["spp"],
                                           rr_depth=a["rr_depth"], max_depth=a["max_depth"], dims=dims, cell=cell,
                                           mu=mu)
    same = (nr[pix] == nro) & (ns[pix] == nso)
    print(f"paths agree on {same.mean():.3f} of the pixels; samples per pixel {ns[pix].mean():.1f}")
    assert same.mean() > 0.9 and ns[pix].mean() > 8 and nr[pix].mean() > 4
    assert np.max(np.abs(img[pix][same] - ro[same])) <= 1e-4 * max(1.0, np.abs(ro).max())


def test_pt_bf16_image_statistics():
    # BF16 network on the query model: decisions straddle thresholds more
    # often, so the image is compared in the mean over 256 pixels x 16 paths
    m, params = _fitted("cfg1")
    p = gpu_plan("cfg1", "bf16")
    pt = dev(params)
    W = H = 64
    cam = synth.orbit_camera(0.4, W, H)
    lut = _pt_lut()
    a = _pt_args(spp=16)
    rgba, nr, ns, _ = ngv.render(p, pt, cam, dev(lut), W, H, 1.0, 3, **a)
    img = host(rgba).reshape(-1, 4)
    pix = np.random.default_rng(9).choice(W * H, 256, replace=False)
    ro, _, _ = oracle.render_pixels_pt(m, params.astype(np.float64), cam, lut, W, H, 3, pix, a["density"], a["light"],
                                       a["radiance"], a["background"], spp=a["spp"], rr_depth=a["rr_depth"],
                                       max_depth=a["max_depth"])
    g, o = img[pix], ro
    print("mean rgba gpu", g.mean(0), "oracle", o.mean(0), "samples per pixel", host(ns).mean())
    assert o[:, 3].mean() > 0.2   # a good share of camera rays scatter
    se = np.sqrt(g.var(0) / len(pix) + o.var(0) / len(pix))
    assert np.all(np.abs(g.mean(0) - o.mean(0)) <= 4.5 * se + 2e-2)


def test_pt_closed_forms_on_device():
    # all weights 0: Phi = 0 everywhere, the medium takes the table's first
    # row.  Empty medium: every pixel is the background; white furnace
    # (albedo 1, no light): every path leaves with throughput 1
    p = gpu_plan("tiny", "fp32")
    pt = torch.zeros(p.n_params, dtype=torch.float32, device="cuda")
    W, H = 32, 24
    cam = synth.orbit_camera(0.2, W, H)
    lut = np.zeros((256, 4), np.float32)
    lut[:, :3] = 1.0
    rgba, nr, ns, cnt = ngv.render(p, pt, cam, dev(lut), W, H, 1.0, 1, **_pt_args(background=(0.25, 0.5, 0.75)))
    hit = oracle.ray_counts(cam, W, H, 1, 2.0 ** -10).reshape(H, W) > 0
    img = host(rgba)
    np.testing.assert_array_equal(img, np.broadcast_to(np.float32([0.25, 0.5, 0.75, 0.0]), img.shape))
    assert np.all(host(ns) == 0) and hit.any()
    lut[:, 3] = 0.5
    rgba, nr, ns, cnt = ngv.render(p, pt, cam, dev(lut), W, H, 1.0, 1,
                                   **_pt_args(background=(0.7, 0.7, 0.7), radiance=(0, 0, 0), max_depth=1024))
    img = host(rgba)
    np.testing.assert_array_equal(img[..., :3], np.full(img[..., :3].shape, np.float32(0.7)))
    # off the cube no collisions; on it (short chords may be crossed freely) most pixels have some
    assert np.all(host(nr)[~hit] == 0) and np.mean(host(nr)[hit] > 0) > 0.8


def test_render_ex_rejects_bad_lighting_options():
    p = gpu_plan("tiny", "fp32")
    pt = torch.zeros(p.n_params, dtype=torch.float32, device="cuda")
    cam = synth.orbit_camera(0.2, 16, 16)
    lut = dev(synth.transfer_function_lut())
    mc = ngv.MacroCells((48, 48, 48), 8)
    bad = [dict(mode="pt", density=0.0), dict(mode="pt", spp=0), dict(mode="pt", spp=257),
           dict(mode="pt", max_depth=0), dict(mode="pt", rr_depth=-1), dict(mode="pt", light=(0, 0, 0)),
           dict(mode="rm_shadow", light=(0, 0, 0)), dict(mode="pt", light=(float("nan"), 0, 1))]
    for kw in bad:
        with pytest.raises(RuntimeError):
            ngv.render(p, pt, cam, lut, 16, 16, 2.0 ** -8, 1, **kw)
    with pytest.raises(RuntimeError, match="error -4"):
        ngv.render(p, pt, cam, lut, 16, 16, 2.0 ** -8, 1, mode="rm_shadow", macrocells=mc, adaptive=True)
