"""Pins of the oracle's shadow ray marcher and path tracer against what the
mathematics fixes: closed forms of constant media (Beer-Lambert transmittance,
the single-scattering integral), a white furnace, a brute-force argmax of the
samples' contributions, unbiasedness of Russian roulette and of null
collisions under looser majorants, and the per-cell majorant walk.

Statistical pins compare a mean over N independent paths with its expected
value within 4.5 standard errors (a false failure about once in 3e5 runs; the
seeds are fixed, so a pass is reproducible).
"""
import math

import numpy as np
import pytest

import oracle

DT = 2.0 ** -10
CAM_Z = np.array([0.3, 0.6, -1.0, 0, 0, 0, 0, 0, 0, 0, 0, 1], np.float32)  # every pixel: +z through the cube


def _const_phi_model(c):
    # Phi = c everywhere (every table entry 1, hidden weight 1, output weight c)
    m = oracle.Model(1, 1, 10, [5], 1, 1)
    params = np.zeros(m.n_params)
    params[:m.n_table] = 1.0
    params[m.n_table:] = [1.0, c]
    return m, params


def _z_model():
    # Phi(x) = z exactly: one dense level whose vertex values are their z
    # coordinate (trilinear interpolation reproduces affine fields), then
    # relu(1 * e) * 1
    N = 5
    m = oracle.Model(1, 1, 10, [N], 1, 1)
    params = np.zeros(m.n_params)
    v = np.arange(N) / (N - 1)
    vz, _, _ = np.meshgrid(v, v, v, indexing="ij")
    params[:m.n_table] = vz.ravel()
    params[m.n_table:] = [1.0, 1.0]
    return m, params


def _const_lut(rgb, a):
    lut = np.zeros((256, 4), np.float32)
    lut[:] = [*rgb, a]
    return lut


def _tf(lut, v):
    # linear blend of the table at v (FP64)
    lut = lut.astype(np.float64)
    v = np.clip(v, 0.0, 1.0)
    u = 255.0 * v
    i0 = np.minimum(np.floor(u), 254).astype(int)
    f = (u - i0)[..., None]
    return (1 - f) * lut[i0] + f * lut[i0 + 1]


def _within(mean, expect, n, sd=None):
    if sd is None:
        sd = math.sqrt(max(expect * (1 - expect), 1e-12))
    assert abs(mean - expect) <= 4.5 * sd / math.sqrt(n), (mean, expect, n)


# -------------------------------------------------- single-shot shadows -----

@pytest.mark.parametrize("light,chord", [((1, 0, 0), 0.7), ((2, 0, 0), 0.7), ((-1, 0, 0), 0.3), ((0, 1, 0), 0.4)])
def test_shadow_constant_alpha_closed_form(light, chord):
    # constant alpha a: contributions (1-a)^k a fall with k, so the shading
    # point is the first sample; the shadow ray crosses `chord` of constant
    # alpha, T = (1-a)^m for its m samples (the chord's grid steps, less the
    # one at the point itself), and attenuates the whole colour
    m, params = _const_phi_model(0.5)
    a = 0.001
    lut = _const_lut((0.2, 0.4, 0.8), a)
    rgba, ng, nu, ks = oracle.render_pixels_shadow(m, params, CAM_Z, lut, 4, 4, DT, 3, np.arange(16), light)
    af = float(np.float32(a))
    A = 1 - (1 - af) ** 1024
    assert np.all(ng == 1024) and np.all(nu == 1024) and np.all(ks == 0)
    np.testing.assert_allclose(rgba[:, 3], A, rtol=1e-12)
    T = rgba[:, :3] / (np.array([0.2, 0.4, 0.8], np.float32).astype(np.float64) * A)
    steps = chord / DT
    assert np.all(T <= (1 - af) ** (steps - 2) * (1 + 1e-9)) and np.all(T >= (1 - af) ** (steps + 1) * (1 - 1e-9))
    np.testing.assert_allclose(T, T[:, :1].repeat(3, 1), rtol=1e-12)


def test_shadow_saturates_at_one_percent():
    # a dense medium: the shadow ray stops after the sample at which T <= 0.01
    m, params = _const_phi_model(0.5)
    lut = _const_lut((0.5, 0.5, 0.5), 0.05)
    rgba, _, nu, ks = oracle.render_pixels_shadow(m, params, CAM_Z, lut, 2, 2, DT, 4, np.arange(4), (1, 0, 0))
    af = float(np.float32(0.05))
    n_stop = math.ceil(math.log(0.01) / math.log(1 - af))
    A = 1 - (1 - af) ** n_stop
    assert np.all(nu == n_stop) and np.all(ks == 0)
    np.testing.assert_allclose(rgba[:, :3], 0.5 * A * (1 - af) ** n_stop, rtol=1e-12)


def test_shadow_point_is_the_largest_contribution_brute_force():
    # Phi = z along a +z ray with alpha rising in z: the contributions
    # (1 - A_{k-1}) alpha_k rise, then fall; the shading point is their
    # argmax, found here by brute force over the binary32 sample points, and
    # the shadow ray along +x keeps z, so T = (1 - alpha(z*))^m
    m, params = _z_model()
    i = np.arange(256, dtype=np.float64)
    lut = np.stack([i / 255, 1 - i / 255, np.full(256, 0.5), 0.0005 + 0.02 * (i / 255) ** 2], 1).astype(np.float32)
    W = H = 3
    pix = np.arange(W * H)
    rgba, ng, nu, ks = oracle.render_pixels_shadow(m, params, CAM_Z, lut, W, H, DT, 9, pix, (1, 0, 0))
    for q in pix:
        n = int(ng[q])
        pts = oracle.ray_points(CAM_Z, W, H, 9, DT, q, 0, n)
        c4 = _tf(lut, pts[:, 2].astype(np.float64))
        A, w = 0.0, np.zeros(n)
        C = np.zeros(3)
        stop = n
        for k in range(n):
            w[k] = (1 - A) * c4[k, 3]
            C += w[k] * c4[k, :3]
            A += w[k]
            if A >= 0.99:
                stop = k + 1
                break
        k_star = int(np.argmax(w[:stop]))
        assert 50 < k_star < n - 50      # an interior maximum, not the first or last sample
        assert ks[q] == k_star and nu[q] == stop
        a_s = c4[k_star, 3]
        steps = (1 - float(pts[k_star, 0])) / DT
        T = rgba[q, :3] / C
        np.testing.assert_allclose(T, T[0], rtol=1e-10)
        assert (1 - a_s) ** (steps + 1) * (1 - 1e-9) <= T[0] <= (1 - a_s) ** (steps - 2) * (1 + 1e-9)
        np.testing.assert_allclose(rgba[q, 3], A, rtol=1e-12)


def test_shadow_macrocell_skipping():
    # all cells open: the same image as without macro-cells; all closed:
    # nothing is composited and there is no shading point
    m, params = _const_phi_model(0.5)
    lut = _const_lut((0.2, 0.4, 0.8), 0.002)
    dims, cell = (64, 64, 64), 16
    n = int(np.prod(oracle.mc_grid(dims, cell)))
    pix = np.arange(4)
    plain = oracle.render_pixels_shadow(m, params, CAM_Z, lut, 2, 2, DT, 3, pix, (0, 1, 1))
    full = oracle.render_pixels_shadow(m, params, CAM_Z, lut, 2, 2, DT, 3, pix, (0, 1, 1), dims, cell, np.ones(n))
    for x, y in zip(plain, full):
        np.testing.assert_array_equal(x, y)
    none = oracle.render_pixels_shadow(m, params, CAM_Z, lut, 2, 2, DT, 3, pix, (0, 1, 1), dims, cell, np.zeros(n))
    assert np.all(none[0] == 0) and np.all(none[2] == 0) and np.all(none[3] == 0xFFFFFFFF)


# ------------------------------------------------------- path tracing -----

PT_W = PT_H = 8          # 64 pixels, all on the same +z ray through the cube centre line
PT_SPP = 256             # 16384 independent paths per call


def _pt(lut, density, light=(0, 0, -1), radiance=(0, 0, 0), background=(1, 1, 1), phi=0.5, **kw):
    m, params = _const_phi_model(phi)
    cam = np.array([0.5, 0.5, -1.0, 0, 0, 0, 0, 0, 0, 0, 0, 1], np.float32)
    return oracle.render_pixels_pt(m, params, cam, lut, PT_W, PT_H, kw.pop("seed", 17), np.arange(PT_W * PT_H),
                                   density, light, radiance, background, spp=kw.pop("spp", PT_SPP), **kw)


def test_pt_empty_medium_returns_background():
    rgba, nr, ns = _pt(_const_lut((1, 1, 1), 0.0), 5.0, background=(0.25, 0.5, 0.75))
    np.testing.assert_array_equal(rgba, np.broadcast_to([0.25, 0.5, 0.75, 0.0], rgba.shape))
    assert np.all(nr == 0) and np.all(ns == 0)


@pytest.mark.parametrize("use_mc", [False, True])
def test_pt_white_furnace(use_mc):
    # albedo 1, no light, background 0.7: every path leaves with throughput 1
    # (roulette survives with q = 1), so every pixel is exactly 0.7
    lut = _const_lut((1, 1, 1), 0.5)
    kw = {}
    if use_mc:
        dims, cell = (64, 64, 64), 16
        kw = dict(dims=dims, cell=cell, mu=np.full(int(np.prod(oracle.mc_grid(dims, cell))), 0.5, np.float32))
    rgba, nr, ns = _pt(lut, 4.0, background=(0.7, 0.7, 0.7), **kw)
    np.testing.assert_array_equal(rgba[:, :3], np.full((PT_W * PT_H, 3), float(np.float32(0.7))))  # B is binary32
    assert np.all(nr > 0) and np.all(ns >= nr)


def _absorbing(lut_alpha_max=None, **kw):
    # albedo 0, background 1, sigma = density * alpha = 1: a path is 1 iff the
    # camera ray crosses the unit chord without a real collision, probability
    # exp(-sigma); alpha is 1 - that
    lut = _const_lut((0, 0, 0), 0.5)
    if lut_alpha_max is not None:
        lut[200:, 3] = lut_alpha_max    # never looked up (Phi = 0.5): only the majorant grows
    rgba, nr, ns = _pt(lut, 2.0, **kw)
    np.testing.assert_allclose(rgba[:, 3], 1 - rgba[:, 0], rtol=0, atol=1e-15)
    return rgba, nr, ns


def test_pt_beer_lambert_transmittance():
    rgba, nr, ns = _absorbing()
    _within(rgba[:, 0].mean(), math.exp(-1.0), PT_W * PT_H * PT_SPP)
    assert np.all(ns == nr)             # majorant = extinction: every tentative collision is real


def test_pt_null_collisions_are_unbiased():
    # a majorant 4x the extinction: three of four tentative collisions are
    # null, the transmittance estimate is unchanged
    rgba, nr, ns = _absorbing(lut_alpha_max=2.0)
    _within(rgba[:, 0].mean(), math.exp(-1.0), PT_W * PT_H * PT_SPP)
    assert ns.sum() > 3 * nr.sum()


@pytest.mark.parametrize("mu_scale", [1.0, 3.0])
def test_pt_macrocell_majorants(mu_scale):
    # per-cell majorants, tight or loose, walked cell by cell: same estimate
    dims, cell = (64, 64, 64), 16
    mu = np.full(int(np.prod(oracle.mc_grid(dims, cell))), 0.5 * mu_scale, np.float32)
    rgba, nr, ns = _absorbing(dims=dims, cell=cell, mu=mu)
    _within(rgba[:, 0].mean(), math.exp(-1.0), PT_W * PT_H * PT_SPP)


def test_pt_macrocell_empty_half():
    # cells of mu = 0 hold no collisions: the ray meets extinction only over
    # the half z >= 0.5 (cells 2..3 of 4 along z), transmittance exp(-sigma/2)
    dims, cell = (64, 64, 64), 16
    M = oracle.mc_grid(dims, cell)
    mu = np.full(M[::-1], 0.5, np.float32)   # [z][y][x]
    mu[:2] = 0.0
    rgba, nr, ns = _absorbing(dims=dims, cell=cell, mu=mu.ravel())
    _within(rgba[:, 0].mean(), math.exp(-0.5), PT_W * PT_H * PT_SPP)


def test_pt_single_scattering_with_shadow_rays():
    # sigma = density * alpha = 1; albedo 1, light behind the camera (towards
    # -z) of radiance 4 pi (so E/(4 pi) = 1), no background, one scattering:
    # the first collision at
    # depth z (density sigma e^{-sigma z}) sends a shadow ray back over z,
    # which escapes with probability e^{-sigma z}:
    #   E[L] = int_0^1 sigma e^{-2 sigma z} dz = (1 - e^{-2 sigma}) / 2
    lut = _const_lut((1, 1, 1), 0.5)
    rgba, nr, ns = _pt(lut, 2.0, light=(0, 0, -1), radiance=(4 * math.pi,) * 3, background=(0, 0, 0), max_depth=1)
    expect = (1 - math.exp(-2.0)) / 2
    _within(rgba[:, 0].mean(), expect, PT_W * PT_H * PT_SPP)
    np.testing.assert_allclose(rgba[:, 0], rgba[:, 2], rtol=1e-12)
    # the light from the side (+x) crosses x in [0.5, 1]: E[L] =
    # int_0^1 sigma e^{-sigma z} e^{-sigma/2} dz = e^{-sigma/2} (1 - e^{-sigma})
    rgba2, _, _ = _pt(lut, 2.0, light=(1, 0, 0), radiance=(4 * math.pi,) * 3, background=(0, 0, 0), max_depth=1)
    _within(rgba2[:, 0].mean(), math.exp(-0.5) * (1 - math.exp(-1.0)), PT_W * PT_H * PT_SPP)


def test_pt_russian_roulette_is_unbiased():
    # albedo 0.8 with background 1: the same mean with roulette from the
    # first collision on as with (practically) no roulette
    lut = _const_lut((0.8, 0.8, 0.8), 0.5)
    a, _, _ = _pt(lut, 4.0, rr_depth=0, seed=5)
    b, _, _ = _pt(lut, 4.0, rr_depth=1000, seed=6)
    n = PT_W * PT_H * PT_SPP
    sd = math.sqrt(np.var(a[:, 0]) * PT_SPP + np.var(b[:, 0]) * PT_SPP)   # per-path spread, both runs
    assert abs(a[:, 0].mean() - b[:, 0].mean()) <= 4.5 * sd / math.sqrt(n)
    assert 0.3 < b[:, 0].mean() < 0.95
