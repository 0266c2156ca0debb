"""Pins of the oracle's out-of-core sampling (Section 4.1: a buffer of R
random blocks, S refreshed per step; samples pick a block of the buffer, a
voxel of the block, and jitter the voxel centre by up to half a voxel; the
value is interpolated from the voxel and its neighbours).

What is fixed independently of the oracle's code: the buffer holds R blocks
drawn uniformly, a step replaces at most S of them and the oldest first; a
sample lies within half a voxel of a voxel of a block the buffer holds; the
jitter is uniform over the voxel; on an affine volume the cell-centred
trilinear sampler returns the affine function of the (clamped) coordinate
exactly, so the value is the interpolation at the jittered point.
"""
import math

import numpy as np

import oracle


def _grid(dims, b):
    return [(d + b - 1) // b for d in dims]


def test_buffer_blocks_are_uniform_and_refresh_oldest_first():
    dims, b = (64, 48, 40), 8
    G = _grid(dims, b)
    nb = G[0] * G[1] * G[2]                  # 8 * 6 * 5 = 240 blocks
    R, S = 1 << 14, 1 << 10
    s0 = oracle.ooc_slots(dims, b, R, S, 7, 0)
    assert s0.min() >= 0 and s0.max() < nb
    counts = np.bincount(s0, minlength=nb)
    chi2 = float(((counts - R / nb) ** 2 / (R / nb)).sum())
    assert chi2 < nb + 6 * math.sqrt(2 * nb)  # chi-square, nb - 1 degrees of freedom
    prev = s0
    changed_ever = np.zeros(R, bool)
    for k in range(1, R // S + 1):
        cur = oracle.ooc_slots(dims, b, R, S, 7, k)
        diff = np.flatnonzero(cur != prev)
        # at most S slots change, and they are the S slots refreshed least recently
        oldest = np.arange((k - 1) * S, k * S) % R
        assert diff.size <= S and np.all(np.isin(diff, oldest))
        changed_ever[oldest] = True
        prev = cur
    assert changed_ever.all()                 # after R/S steps every slot was refreshed


def test_samples_lie_in_buffered_blocks_partial_edges():
    dims, b = (37, 20, 29), 8                 # partial blocks on every axis
    vol = np.random.default_rng(1).random(dims[::-1], dtype=np.float32)
    R, S, B = 64, 16, 20000
    G = _grid(dims, b)
    for step in (0, 3):
        xyz, y, blk = oracle.ooc_sample(vol, b, R, S, 11, step, B)
        slots = oracle.ooc_slots(dims, b, R, S, 11, step)
        assert np.all(np.isin(blk, slots))
        bc = np.stack([blk % G[0], (blk // G[0]) % G[1], blk // (G[0] * G[1])], 1)
        vox = np.floor(xyz.astype(np.float64) * np.array(dims)).astype(np.int64)
        lo = bc * b
        hi = np.minimum(lo + b, np.array(dims))
        assert np.all(vox >= lo) and np.all(vox <= hi)       # <= : rounding of x D at the top edge
        assert np.mean(vox < hi) > 0.999
        assert np.all(vox <= np.array(dims)) and np.all(xyz >= 0) and np.all(xyz <= 1)


def test_jitter_is_uniform_over_the_voxel():
    dims, b = (64, 64, 64), 16
    vol = np.zeros((64, 64, 64), np.float32)
    xyz, _, _ = oracle.ooc_sample(vol, b, 32, 8, 3, 1, 1 << 16)
    f = (xyz.astype(np.float64) * 64) % 1.0
    n = f.size
    assert abs(f.mean() - 0.5) < 4.5 * math.sqrt(1 / 12 / n)
    assert abs(f.var() - 1 / 12) < 0.005
    # every voxel of a buffered block is reachable: the voxel offsets in the block cover 0..b-1
    off = np.floor(xyz.astype(np.float64) * 64).astype(int) % b
    assert set(np.unique(off)) == set(range(b))


def test_values_are_the_trilinear_sample_at_the_jittered_point():
    # affine volume v = a . (voxel centre) + c: the cell-centred trilinear
    # sampler returns a . clamp(x, 1/2D, 1 - 1/2D) + c exactly
    dims, b = (40, 24, 32), 8
    a = np.array([0.7, -1.3, 0.45])
    c = 0.2
    ctr = [(np.arange(d) + 0.5) / d for d in dims]
    z, y_, x = np.meshgrid(ctr[2], ctr[1], ctr[0], indexing="ij")
    vol = (a[0] * x + a[1] * y_ + a[2] * z + c).astype(np.float32)
    xyz, y, _ = oracle.ooc_sample(vol, b, 24, 6, 5, 2, 30000)
    p = np.clip(xyz.astype(np.float64), 0.5 / np.array(dims), 1 - 0.5 / np.array(dims))
    expect = p @ a + c
    # the volume's values are binary32 roundings of the affine field
    np.testing.assert_allclose(y, expect, atol=4e-7)
    # and a sample is not the value of its voxel centre
    vc = (np.floor(xyz.astype(np.float64) * dims) + 0.5) / dims
    assert np.mean(np.abs(y - (vc @ a + c)) > 1e-3) > 0.5
