"""FP64 CPU oracle for the neural-volume hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  The C source
(``ngvol_oracle.c``) shares no code with the HIP library.

Functions mirror the C entry points; arrays are NumPy, parameters FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ngvol_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, u32, u64, dbl, flt = C.c_int64, C.c_int32, C.c_uint32, C.c_uint64, C.c_double, C.c_float
        sig = {
            "orc_rng_u64": (u64, [u64, u32, u64]),
            "orc_rng_u01": (dbl, [u64, u32, u64]),
            "orc_layout": (C.c_int, [P, P, P, P]),
            "orc_resolutions": (C.c_int, [C.c_int, C.c_int, dbl, C.c_int, P]),
            "orc_encode": (C.c_int, [P, P, P, i64, P]),
            "orc_encode_debug": (C.c_int, [P, P, i64, P, P]),
            "orc_mlp_fwd": (C.c_int, [P, P, P, i64, P]),
            "orc_forward": (C.c_int, [P, P, P, i64, P]),
            "orc_sample_volume": (C.c_int, [P, P, P, i64, P]),
            "orc_batch_coords": (C.c_int, [u64, i64, i64, P]),
            "orc_loss_grad": (C.c_int, [P, P, P, P, i64, P, P]),
            "orc_loss_grad_kind": (C.c_int, [P, P, P, P, i64, C.c_int, P, P]),
            "orc_lr_at": (dbl, [dbl, i64, i64, i64, dbl]),
            "orc_adam": (C.c_int, [i64, P, P, P, P, i64, dbl, dbl, dbl, dbl]),
            "orc_adam_reg": (C.c_int, [i64, i64, P, P, P, P, i64, dbl, dbl, dbl, dbl, dbl]),
            "orc_train_opt": (C.c_int, [P, P, P, P, P, P, u64, i64, i64, i64, C.c_int, P, P]),
            "orc_train": (C.c_int, [P, P, P, P, P, P, u64, i64, i64, i64, dbl, dbl, dbl, dbl, P]),
            "orc_mse_grid": (C.c_int, [P, P, P, P, P]),
            "orc_ray_counts": (C.c_int, [P, C.c_int, C.c_int, u32, flt, P]),
            "orc_ray_points": (C.c_int, [P, C.c_int, C.c_int, u32, flt, i64, u32, u32, P]),
            "orc_render_pixels": (C.c_int, [P, P, P, P, C.c_int, C.c_int, flt, u32, P, i64, P, P, P]),
            "orc_num_threads": (C.c_int, []),
            "orc_ooc_slots": (C.c_int, [P, C.c_int, i64, i64, u64, i64, P]),
            "orc_ooc_sample": (C.c_int, [P, P, C.c_int, i64, i64, u64, i64, i64, P, P, P]),
            "orc_set_threads": (None, [C.c_int]),
            "orc_mc_cells": (C.c_int, [P, C.c_int, P, i64, P]),
            "orc_mc_update": (C.c_int, [P, C.c_int, P, P, i64, P, P]),
            "orc_mc_opacity": (C.c_int, [P, P, i64, P, P]),
            "orc_render_pixels_mc": (C.c_int, [P, P, P, P, C.c_int, C.c_int, flt, u32, P, i64, P, C.c_int, P, P, P,
                                               P]),
            "orc_adaptive_steps": (C.c_int, [flt, flt, C.c_int]),
            "orc_mc_traverse": (C.c_int, [P, C.c_int, u32, flt, i64, P, C.c_int, C.c_int, P, P, i64, P]),
            "orc_render_pixels_adaptive": (C.c_int, [P, P, P, P, C.c_int, C.c_int, flt, u32, P, i64, P, C.c_int, P,
                                                     flt, C.c_int, P, P, P]),
            "orc_render_pixels_shadow": (C.c_int, [P, P, P, P, C.c_int, C.c_int, flt, u32, P, i64, P, C.c_int, P, P,
                                                   P, P, P, P]),
            "orc_render_pixels_pt": (C.c_int, [P, P, P, P, C.c_int, C.c_int, u32, P, i64, P, C.c_int, P, P, P, P, P,
                                               P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _chk(rc):
    if rc != 0:
        raise RuntimeError(f"oracle call failed with status {rc}")


class Model:
    """Hash-grid + MLP description: levels L, features F, table 2**log2T,
    vertices per axis N_l (``res``), MLP width, number of hidden layers and
    whether the output neuron is followed by a ReLU."""

    def __init__(self, L, F, log2T, res, width, n_hidden, out_relu=False):
        self.L, self.F, self.log2T, self.width, self.n_hidden = L, F, log2T, width, n_hidden
        self.out_relu = bool(out_relu)
        self.res = [int(r) for r in res]
        assert len(self.res) == L
        self.desc = np.array([L, F, log2T, width, n_hidden, int(self.out_relu)] + self.res, dtype=np.int32)
        size = np.zeros(L, np.int64)
        off = np.zeros(L + 1, np.int64)
        counts = np.zeros(3, np.int64)
        _chk(lib().orc_layout(_p(self.desc), _p(size), _p(off), _p(counts)))
        self.level_size, self.level_offset = size, off
        self.n_table, self.n_mlp, self.n_params = (int(c) for c in counts)
        self.n_in = L * F


def resolutions(L, base, scale=0.0, max_res=0):
    out = np.zeros(L, np.int32)
    _chk(lib().orc_resolutions(L, base, float(scale), int(max_res), _p(out)))
    return [int(v) for v in out]


def rng_u64(seed, stream, index):
    return int(lib().orc_rng_u64(seed, stream, index))


def rng_u01(seed, stream, index):
    return float(lib().orc_rng_u01(seed, stream, index))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def encode(m: Model, params, xyz):
    params, xyz = _f64(params), _f32(xyz)
    n = xyz.shape[0]
    out = np.zeros((n, m.n_in), np.float64)
    _chk(lib().orc_encode(_p(m.desc), _p(params), _p(xyz), n, _p(out)))
    return out


def encode_debug(m: Model, xyz):
    xyz = _f32(xyz)
    n = xyz.shape[0]
    idx = np.zeros((n, m.L, 8), np.uint32)
    w = np.zeros((n, m.L, 8), np.float64)
    _chk(lib().orc_encode_debug(_p(m.desc), _p(xyz), n, _p(idx), _p(w)))
    return idx, w


def mlp_fwd(m: Model, mlp_params, feat):
    mlp_params, feat = _f64(mlp_params), _f64(feat)
    n = feat.shape[0]
    out = np.zeros(n, np.float64)
    _chk(lib().orc_mlp_fwd(_p(m.desc), _p(mlp_params), _p(feat), n, _p(out)))
    return out


def forward(m: Model, params, xyz):
    params, xyz = _f64(params), _f32(xyz)
    n = xyz.shape[0]
    out = np.zeros(n, np.float64)
    _chk(lib().orc_forward(_p(m.desc), _p(params), _p(xyz), n, _p(out)))
    return out


def sample_volume(vol, xyz):
    vol, xyz = _f32(vol), _f32(xyz)
    dims = np.array([vol.shape[2], vol.shape[1], vol.shape[0]], np.int32)
    n = xyz.shape[0]
    y = np.zeros(n, np.float64)
    _chk(lib().orc_sample_volume(_p(vol), _p(dims), _p(xyz), n, _p(y)))
    return y


def batch_coords(seed, step, B):
    xyz = np.zeros((B, 3), np.float32)
    _chk(lib().orc_batch_coords(seed, step, B, _p(xyz)))
    return xyz


LOSS_KIND = {"l2": 0, "l1": 1}


def loss_grad(m: Model, params, xyz, y, loss="l2"):
    """(mean loss, dL/dparams) for loss "l2" (mean square) or "l1" (mean absolute)."""
    params, xyz, y = _f64(params), _f32(xyz), _f64(y)
    n = xyz.shape[0]
    g = np.zeros(m.n_params, np.float64)
    out = np.zeros(1, np.float64)
    _chk(lib().orc_loss_grad_kind(_p(m.desc), _p(params), _p(xyz), _p(y), n, LOSS_KIND[loss], _p(g), _p(out)))
    return float(out[0]), g


def lr_at(lr, k, decay):
    """Learning rate of 0-based step k under decay = (start, interval, base) or None."""
    start, interval, base = decay if decay is not None else (0, 0, 1.0)
    return float(lib().orc_lr_at(lr, k, start, interval, base))


def adam(theta, m_, v_, g, t, lr, b1, b2, eps, l2_reg=0.0, reg_from=None):
    """In-place on FP64 arrays theta, m_, v_; l2_reg * theta joins the gradient
    of indices >= reg_from (the MLP block when called with n_table)."""
    for a in (theta, m_, v_):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    rf = theta.size if reg_from is None else int(reg_from)
    _chk(lib().orc_adam_reg(theta.size, rf, _p(theta), _p(m_), _p(v_), _p(g), t, lr, b1, b2, eps, l2_reg))


def train(m: Model, params, vol, seed, steps, B, lr, b1, b2, eps, step0=0, state=None, loss="l2", l2_reg=0.0,
          decay=None):
    """Returns (params, (m, v), losses); params is a new FP64 array."""
    theta = _f64(params).copy()
    if state is None:
        am, av = np.zeros(m.n_params), np.zeros(m.n_params)
    else:
        am, av = (_f64(s).copy() for s in state)
    vol = _f32(vol)
    dims = np.array([vol.shape[2], vol.shape[1], vol.shape[0]], np.int32)
    losses = np.zeros(steps, np.float64)
    start, interval, base = decay if decay is not None else (0, 0, 1.0)
    opt = np.array([lr, b1, b2, eps, l2_reg, start, interval, base], np.float64)
    _chk(lib().orc_train_opt(_p(m.desc), _p(theta), _p(am), _p(av), _p(vol), _p(dims), seed, step0, steps, B,
                             LOSS_KIND[loss], _p(opt), _p(losses)))
    return theta, (am, av), losses


def mse_grid(m: Model, params, vol):
    params, vol = _f64(params), _f32(vol)
    dims = np.array([vol.shape[2], vol.shape[1], vol.shape[0]], np.int32)
    out = np.zeros(1, np.float64)
    _chk(lib().orc_mse_grid(_p(m.desc), _p(params), _p(vol), _p(dims), _p(out)))
    return float(out[0])


def psnr_from_mse(mse):
    return -10.0 * np.log10(mse)


def ray_counts(cam, W, H, frame_seed, dt):
    cam = _f32(cam)
    n = np.zeros(W * H, np.uint32)
    _chk(lib().orc_ray_counts(_p(cam), W, H, frame_seed, dt, _p(n)))
    return n.reshape(H, W)


def ray_points(cam, W, H, frame_seed, dt, pix, k0, count):
    cam = _f32(cam)
    xyz = np.zeros((count, 3), np.float32)
    _chk(lib().orc_ray_points(_p(cam), W, H, frame_seed, dt, int(pix), k0, count, _p(xyz)))
    return xyz


def render_pixels(m: Model, params, cam, lut, W, H, dt, frame_seed, pix):
    params, cam, lut = _f64(params), _f32(cam), _f32(lut)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.size
    rgba = np.zeros((n, 4), np.float64)
    n_geo = np.zeros(n, np.uint32)
    n_used = np.zeros(n, np.uint32)
    _chk(lib().orc_render_pixels(_p(m.desc), _p(params), _p(cam), _p(lut), W, H, dt, frame_seed, _p(pix), n,
                                 _p(rgba), _p(n_geo), _p(n_used)))
    return rgba, n_geo, n_used


def mc_grid(dims, cell):
    """Cells per axis (x, y, z) of a macro-cell grid over a volume of dims = (Dx, Dy, Dz)."""
    return tuple((int(d) + cell - 1) // cell for d in dims)


def mc_cells(dims, cell, xyz):
    xyz = _f32(xyz)
    out = np.zeros(xyz.shape[0], np.int64)
    _chk(lib().orc_mc_cells(_p(np.asarray(dims, np.int32)), cell, _p(xyz), xyz.shape[0], _p(out)))
    return out


def mc_update(dims, cell, xyz, values, ranges=None):
    """(vmin, vmax) per cell after the samples; ranges continues earlier ones."""
    M = mc_grid(dims, cell)
    n = M[0] * M[1] * M[2]
    if ranges is None:
        vmin, vmax = np.full(n, np.inf), np.full(n, -np.inf)
    else:
        vmin, vmax = (np.array(r, np.float64) for r in ranges)
    xyz, values = _f32(xyz), _f32(values)
    _chk(lib().orc_mc_update(_p(np.asarray(dims, np.int32)), cell, _p(xyz), _p(values), xyz.shape[0], _p(vmin),
                             _p(vmax)))
    return vmin, vmax


def mc_opacity(ranges, lut):
    vmin, vmax = (_f64(r) for r in ranges)
    mu = np.zeros(vmin.size, np.float64)
    _chk(lib().orc_mc_opacity(_p(vmin), _p(vmax), vmin.size, _p(_f32(lut)), _p(mu)))
    return mu


def render_pixels_mc(m: Model, params, cam, lut, W, H, dt, frame_seed, pix, dims, cell, mu):
    params, cam, lut = _f64(params), _f32(cam), _f32(lut)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.size
    rgba = np.zeros((n, 4), np.float64)
    n_geo = np.zeros(n, np.uint32)
    n_used = np.zeros(n, np.uint32)
    mu = None if mu is None else _f64(mu)
    _chk(lib().orc_render_pixels_mc(_p(m.desc), _p(params), _p(cam), _p(lut), W, H, dt, frame_seed, _p(pix), n,
                                    _p(np.asarray(dims, np.int32)), cell, None if mu is None else _p(mu), _p(rgba),
                                    _p(n_geo), _p(n_used)))
    return rgba, n_geo, n_used


def adaptive_steps(mu, s2=64.0, p=2):
    """Grid steps a sample in a cell of maximum opacity mu represents (binary32)."""
    return int(lib().orc_adaptive_steps(mu, s2, int(p)))


def mc_traverse(cam, W, frame_seed, dt, pix, dims, cell, dda=True, cap=1 << 16):
    """(cells, first sample index in each) along a pixel's ray."""
    cam = _f32(cam)
    cells = np.zeros(cap, np.int64)
    first = np.zeros(cap, np.uint32)
    cnt = np.zeros(1, np.int64)
    _chk(lib().orc_mc_traverse(_p(cam), W, frame_seed, dt, int(pix), _p(np.asarray(dims, np.int32)), cell,
                               1 if dda else 0, _p(cells), _p(first), cap, _p(cnt)))
    n = int(cnt[0])
    return cells[:n].copy(), first[:n].copy()


def render_pixels_adaptive(m: Model, params, cam, lut, W, H, dt, frame_seed, pix, dims, cell, mu, s2=64.0, p=2):
    """Adaptive ray marching through macro-cells of maximum opacity mu (binary32)."""
    params, cam, lut = _f64(params), _f32(cam), _f32(lut)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.size
    rgba = np.zeros((n, 4), np.float64)
    n_geo = np.zeros(n, np.uint32)
    n_used = np.zeros(n, np.uint32)
    mu = _f32(mu)
    _chk(lib().orc_render_pixels_adaptive(_p(m.desc), _p(params), _p(cam), _p(lut), W, H, dt, frame_seed, _p(pix), n,
                                          _p(np.asarray(dims, np.int32)), cell, _p(mu), s2, int(p), _p(rgba),
                                          _p(n_geo), _p(n_used)))
    return rgba, n_geo, n_used


def set_threads(n):
    """Thread count of the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(n))


def num_threads():
    return int(lib().orc_num_threads())


def render_pixels_shadow(m: Model, params, cam, lut, W, H, dt, frame_seed, pix, light, dims=(1, 1, 1), cell=1,
                         mu=None):
    """Ray marching with a single-shot shadow from the sample of highest
    contribution towards the light; returns (rgba, n_geo, n_used, kstar)."""
    params, cam, lut = _f64(params), _f32(cam), _f32(lut)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.size
    rgba = np.zeros((n, 4), np.float64)
    n_geo = np.zeros(n, np.uint32)
    n_used = np.zeros(n, np.uint32)
    kstar = np.zeros(n, np.uint32)
    mu = None if mu is None else _f64(mu)
    _chk(lib().orc_render_pixels_shadow(_p(m.desc), _p(params), _p(cam), _p(lut), W, H, dt, frame_seed, _p(pix), n,
                                        _p(np.asarray(dims, np.int32)), cell, None if mu is None else _p(mu), _p(_f32(light)), _p(rgba),
                                        _p(n_geo), _p(n_used), _p(kstar)))
    return rgba, n_geo, n_used, kstar


def render_pixels_pt(m: Model, params, cam, lut, W, H, frame_seed, pix, density, light, radiance, background,
                     spp=1, rr_depth=4, max_depth=1024, dims=(1, 1, 1), cell=1, mu=None):
    """Path tracing with Woodcock tracking and shadow rays (macro-cell
    majorants when mu is given, binary32); returns (rgba, n_real, n_samples)."""
    params, cam, lut = _f64(params), _f32(cam), _f32(lut)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.size
    rgba = np.zeros((n, 4), np.float64)
    n_real = np.zeros(n, np.uint32)
    n_samp = np.zeros(n, np.uint32)
    fo = np.array([density, *light, *radiance, *background], np.float32)
    io = np.array([spp, rr_depth, max_depth], np.int32)
    mu = None if mu is None else _f32(mu)
    _chk(lib().orc_render_pixels_pt(_p(m.desc), _p(params), _p(cam), _p(lut), W, H, frame_seed, _p(pix), n,
                                    _p(np.asarray(dims, np.int32)), cell, None if mu is None else _p(mu), _p(fo), _p(io), _p(rgba),
                                    _p(n_real), _p(n_samp)))
    return rgba, n_real, n_samp


def ooc_slots(dims, block, R, S, seed, step):
    """Block id held by every slot of the out-of-core buffer after step's loads."""
    out = np.zeros(R, np.int64)
    _chk(lib().orc_ooc_slots(_p(np.asarray(dims, np.int32)), block, R, S, seed, step, _p(out)))
    return out


def ooc_sample(vol, block, R, S, seed, step, B):
    """Out-of-core samples of a step: (xyz [B][3] f32, y [B] f64, block id [B])."""
    vol = _f32(vol)
    Dz, Dy, Dx = vol.shape
    xyz = np.zeros((B, 3), np.float32)
    y = np.zeros(B, np.float64)
    blk = np.zeros(B, np.int64)
    _chk(lib().orc_ooc_sample(_p(vol), _p(np.array([Dx, Dy, Dz], np.int32)), block, R, S, seed, step, B, _p(xyz),
                              _p(y), _p(blk)))
    return xyz, y, blk
