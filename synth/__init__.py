"""Seeded synthetic inputs shared by the HIP path's tests, the bench and the oracle.

This module holds none of the method's arithmetic: no encoding, no network, no
ground-truth sampler, no optimiser and no renderer.  It only draws the inputs
both sides consume: initial parameters, query coordinates, ground-truth
volumes, the transfer-function table and camera bases.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: output ``n`` of stream ``(seed, stream)`` is the ``n``-th output of a
SplitMix64 sequence started from state ``seed XOR (stream << 56)``, i.e.
``mix64(s0 + (n + 1) * gamma)``.  A uniform in [0, 1) keeps the top 24 bits,
``(r >> 40) * 2**-24``, so it is exactly representable in binary32.  The paper
only says that training coordinates are drawn uniformly at random in [0,1)^3
(Section 4); the generator choice is ours.

Stream numbers: 1 table init, 2 MLP init, 3 training batch, 4 query
coordinates, 5 pixel jitter, 6 volume generators.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
STREAM_TABLE, STREAM_MLP, STREAM_BATCH, STREAM_QUERY, STREAM_JITTER, STREAM_VOLUME = 1, 2, 3, 4, 5, 6

_U = np.uint64


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> _U(30))) * _U(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> _U(27))) * _U(0x94D049BB133111EB)
    return z ^ (z >> _U(31))


def rng_u64(seed: int, stream: int, index) -> np.ndarray:
    """Counter-based SplitMix64 output for each ``index`` (uint64 array)."""
    if not (0 <= seed < (1 << 56)):
        raise ValueError("seed must be in [0, 2**56)")
    idx = np.asarray(index, dtype=np.uint64)
    s0 = _U(seed) ^ (_U(stream) << _U(56))
    with np.errstate(over="ignore"):
        return _mix64(s0 + (idx + _U(1)) * _U(GAMMA))


def rng_u01(seed: int, stream: int, index) -> np.ndarray:
    """Uniform binary32 values in [0, 1) on the 2**-24 lattice."""
    r = rng_u64(seed, stream, index)
    return ((r >> _U(40)).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def rng_u01_f64(seed: int, stream: int, index) -> np.ndarray:
    r = rng_u64(seed, stream, index)
    return (r >> _U(40)).astype(np.float64) * 2.0 ** -24


# --------------------------------------------------------------------------
# Model inputs
# --------------------------------------------------------------------------

def mlp_shapes(n_in: int, width: int, n_hidden: int) -> list[tuple[int, int]]:
    """(out, in) of each bias-free layer, input layer first, scalar output last."""
    shapes = [(width, n_in)] + [(width, width)] * (n_hidden - 1) + [(1, width)]
    return shapes


def init_params(n_table_params: int, n_in: int, width: int, n_hidden: int,
                table_scale: float, seed: int) -> np.ndarray:
    """FP32 parameter vector: table features, then the MLP matrices.

    Table features are U[-table_scale, table_scale] (stream 1, index = position
    in the table block).  Each MLP matrix is Xavier-uniform with bound
    sqrt(6 / (fan_in + fan_out)) (stream 2, index = position in the MLP block).
    """
    tab = (2.0 * rng_u01_f64(seed, STREAM_TABLE, np.arange(n_table_params)) - 1.0) * table_scale
    parts = [tab]
    pos = 0
    for (o, i) in mlp_shapes(n_in, width, n_hidden):
        bound = math.sqrt(6.0 / (i + o))
        u = rng_u01_f64(seed, STREAM_MLP, np.arange(pos, pos + o * i))
        parts.append((2.0 * u - 1.0) * bound)
        pos += o * i
    return np.concatenate(parts).astype(np.float32)


def query_coords(n: int, seed: int, order: str = "random") -> np.ndarray:
    """[n][3] binary32 coordinates, U[0,1)^3 (stream 4, index = 3*i + axis).

    ``order="morton"`` returns the same points sorted along a 3-D Morton curve
    (10 bits per axis), a stand-in for the spatial coherence of rendering.
    """
    xyz = rng_u01(seed, STREAM_QUERY, np.arange(3 * n)).reshape(n, 3)
    if order == "random":
        return xyz
    if order != "morton":
        raise ValueError(order)
    q = np.minimum((xyz.astype(np.float64) * 1024.0).astype(np.uint64), _U(1023))

    def spread(v):
        v = (v | (v << _U(16))) & _U(0x030000FF)
        v = (v | (v << _U(8))) & _U(0x0300F00F)
        v = (v | (v << _U(4))) & _U(0x030C30C3)
        v = (v | (v << _U(2))) & _U(0x09249249)
        return v

    key = spread(q[:, 0]) | (spread(q[:, 1]) << _U(1)) | (spread(q[:, 2]) << _U(2))
    return np.ascontiguousarray(xyz[np.argsort(key, kind="stable")])


# --------------------------------------------------------------------------
# Ground-truth volumes (x fastest: array index [z][y][x])
# --------------------------------------------------------------------------

def _normalise(v: np.ndarray) -> np.ndarray:
    lo, hi = float(v.min()), float(v.max())
    return ((v - lo) / (hi - lo)).astype(np.float32)


def gaussian_blobs(D: int, seed: int, n_blobs: int = 8) -> np.ndarray:
    """Sum of isotropic Gaussians at voxel centres (i+1/2)/D, min-max normalised.

    Per blob (stream 6, 5 draws): centre U[0,1]^3, sigma U[0.05,0.2],
    amplitude U[0.2,1].
    """
    u = rng_u01_f64(seed, STREAM_VOLUME, np.arange(5 * n_blobs)).reshape(n_blobs, 5)
    x = (np.arange(D, dtype=np.float64) + 0.5) / D
    vol = np.zeros((D, D, D), dtype=np.float64)
    for k in range(n_blobs):
        c = u[k, 0:3]
        sigma = 0.05 + 0.15 * u[k, 3]
        amp = 0.2 + 0.8 * u[k, 4]
        g = [np.exp(-((x - c[a]) ** 2) / (2.0 * sigma * sigma)) for a in range(3)]
        vol += amp * g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
    return _normalise(vol)


def fractal_value_noise(D: int, seed: int, octaves: int = 6, base_freq: int = 4,
                        lacunarity: int = 2, gain: float = 0.5) -> np.ndarray:
    """fbm of smoothstep-blended value noise at voxel centres, min-max normalised.

    Octave o has an (f+1)^3 lattice, f = base_freq * lacunarity**o, with lattice
    values U[0,1) (stream 6, indices after the previous octaves' lattices);
    the blend weight along each axis is s = t^2 (3 - 2t).
    """
    x = (np.arange(D, dtype=np.float64) + 0.5) / D
    vol = np.zeros((D, D, D), dtype=np.float32)
    offset = 0
    amp = 1.0
    for o in range(octaves):
        f = base_freq * lacunarity ** o
        n_lat = (f + 1) ** 3
        lat = rng_u01_f64(seed, STREAM_VOLUME, np.arange(offset, offset + n_lat)).reshape(f + 1, f + 1, f + 1)
        offset += n_lat
        X = x * f
        i0 = np.minimum(np.floor(X).astype(np.int64), f - 1)
        t = X - i0
        s = t * t * (3.0 - 2.0 * t)
        # blend along x (last axis), then y, then z
        a = lat[:, :, i0] * (1.0 - s)[None, None, :] + lat[:, :, i0 + 1] * s[None, None, :]
        b = a[:, i0, :] * (1.0 - s)[None, :, None] + a[:, i0 + 1, :] * s[None, :, None]
        b = b.astype(np.float32)
        s32 = s.astype(np.float32)
        for z in range(D):
            vol[z] += np.float32(amp) * (b[i0[z]] * (1.0 - s32[z]) + b[i0[z] + 1] * s32[z])
        amp *= gain
    return _normalise(vol)


# --------------------------------------------------------------------------
# Rendering inputs
# --------------------------------------------------------------------------

def transfer_function_lut(n: int = 256) -> np.ndarray:
    """[n][4] RGBA binary32: rgb = (v, 1-|2v-1|, 1-v), alpha = 0.05*clamp((v-0.3)/0.7,0,1)^2."""
    v = np.arange(n, dtype=np.float64) / (n - 1)
    a = np.clip((v - 0.3) / 0.7, 0.0, 1.0)
    lut = np.stack([v, 1.0 - np.abs(2.0 * v - 1.0), 1.0 - v, 0.05 * a * a], axis=1)
    return lut.astype(np.float32)


def orbit_camera(angle: float, W: int, H: int, radius: float = 2.0, fov_deg: float = 40.0) -> np.ndarray:
    """Pinhole camera on an orbit around the cube centre, as 12 binary32 values.

    Layout: origin o[3], per-pixel x step U[3], per-pixel y step V[3], and the
    direction W[3] of pixel corner (0,0), so that the (unnormalised) direction
    through pixel centre (px, py) is W + (px+1/2) U + (py+1/2) V.
    Angle 0 puts the eye at (0.5, 0.5, -1.5) looking at (0.5, 0.5, 0.5), up +y.
    """
    c = np.array([0.5, 0.5, 0.5])
    eye = c + radius * np.array([math.sin(angle), 0.0, -math.cos(angle)])
    fwd = (c - eye) / np.linalg.norm(c - eye)
    up = np.array([0.0, 1.0, 0.0])
    right = np.cross(up, fwd)
    right /= np.linalg.norm(right)
    upv = np.cross(fwd, right)
    th = math.tan(math.radians(fov_deg) / 2.0)
    aspect = W / H
    U = right * (2.0 * th * aspect / W)
    V = upv * (2.0 * th / H)
    Wc = fwd - right * th * aspect - upv * th
    return np.concatenate([eye, U, V, Wc]).astype(np.float32)


# --------------------------------------------------------------------------
# The same volumes generated with torch on a device (large targets).
# --------------------------------------------------------------------------

def _torch_normalise_(vol, lo, hi, chunk):
    for z0 in range(0, vol.shape[0], chunk):
        sl = vol[z0:z0 + chunk].float()
        vol[z0:z0 + chunk] = ((sl - lo) / (hi - lo)).to(vol.dtype)
    return vol


def gaussian_blobs_torch(D: int, seed: int, device, dtype=None, n_blobs: int = 8, chunk: int = 64):
    """gaussian_blobs() evaluated with torch (FP32 arithmetic) on `device`."""
    import torch
    dtype = dtype or torch.float16
    u = rng_u01_f64(seed, STREAM_VOLUME, np.arange(5 * n_blobs)).reshape(n_blobs, 5)
    x = (torch.arange(D, device=device, dtype=torch.float32) + 0.5) / D
    vol = torch.empty((D, D, D), dtype=dtype, device=device)
    lo, hi = float("inf"), float("-inf")
    gs = []
    for k in range(n_blobs):
        c = u[k, 0:3]
        sigma = 0.05 + 0.15 * u[k, 3]
        amp = 0.2 + 0.8 * u[k, 4]
        gs.append([torch.exp(-((x - float(c[a])) ** 2) / (2.0 * sigma * sigma)) for a in range(3)] + [amp])
    for z0 in range(0, D, chunk):
        z1 = min(D, z0 + chunk)
        acc = torch.zeros((z1 - z0, D, D), dtype=torch.float32, device=device)
        for gx, gy, gz, amp in gs:
            acc += amp * gz[z0:z1, None, None] * gy[None, :, None] * gx[None, None, :]
        lo, hi = min(lo, float(acc.min())), max(hi, float(acc.max()))
        vol[z0:z1] = acc.to(dtype)
    return _torch_normalise_(vol, lo, hi, chunk)


def fractal_value_noise_torch(D: int, seed: int, device, dtype=None, octaves: int = 6, base_freq: int = 4,
                              lacunarity: int = 2, gain: float = 0.5, chunk: int = 32):
    """fractal_value_noise() evaluated with torch (FP32 arithmetic) on `device`."""
    import torch
    dtype = dtype or torch.float16
    x = (np.arange(D, dtype=np.float64) + 0.5) / D
    octs = []
    offset = 0
    amp = 1.0
    for o in range(octaves):
        f = base_freq * lacunarity ** o
        n_lat = (f + 1) ** 3
        lat = rng_u01_f64(seed, STREAM_VOLUME, np.arange(offset, offset + n_lat)).reshape(f + 1, f + 1, f + 1)
        offset += n_lat
        X = x * f
        i0 = np.minimum(np.floor(X).astype(np.int64), f - 1)
        t = X - i0
        s = t * t * (3.0 - 2.0 * t)
        a = lat[:, :, i0] * (1.0 - s)[None, None, :] + lat[:, :, i0 + 1] * s[None, None, :]
        b = a[:, i0, :] * (1.0 - s)[None, :, None] + a[:, i0 + 1, :] * s[None, :, None]
        octs.append((torch.from_numpy(b.astype(np.float32)).to(device), torch.from_numpy(i0).to(device),
                     torch.from_numpy(s.astype(np.float32)).to(device), amp))
        amp *= gain
    vol = torch.empty((D, D, D), dtype=dtype, device=device)
    lo, hi = float("inf"), float("-inf")
    for z0 in range(0, D, chunk):
        z1 = min(D, z0 + chunk)
        acc = torch.zeros((z1 - z0, D, D), dtype=torch.float32, device=device)
        for b, i0, s, a in octs:
            iz = i0[z0:z1]
            sz = s[z0:z1][:, None, None]
            acc += a * (b[iz] * (1.0 - sz) + b[iz + 1] * sz)
        lo, hi = min(lo, float(acc.min())), max(hi, float(acc.max()))
        vol[z0:z1] = acc.to(dtype)
    return _torch_normalise_(vol, lo, hi, chunk)


def multi_volume_specs(k: int = 16):
    """The batched workload: model i has log2 T = 16 + (i mod 7), L = (8, 12, 16)[i mod 3]
    levels from 16 to 2048 vertices, F = 2, a 64-64 MLP; its target is a
    (128, 256, 512, 1024)[i mod 4]^3 FP16 volume, Gaussian blobs for even i and
    fractal noise for odd i, seed 1000 + i."""
    return [dict(log2T=16 + (i % 7), L=(8, 12, 16)[i % 3], D=(128, 256, 512, 1024)[i % 4],
                 kind="blobs" if i % 2 == 0 else "noise", seed=1000 + i) for i in range(k)]
