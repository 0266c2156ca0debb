"""Host logic of out-of-core sampling: the bricked file that
ngvol_ooc_brick_file writes holds, per block, the block's voxels and a
one-voxel ghost layer with indices clamped to the volume (no GPU needed)."""
import numpy as np
import pytest

ngv = pytest.importorskip("paper_2207_11620_amd")


def _lib_or_skip():
    try:
        ngv.lib()
    except Exception as e:  # library not built here
        pytest.skip(f"library not loadable: {e}")


@pytest.mark.parametrize("dtype,block", [("f32", 8), ("f16", 6)])
def test_bricked_records_hold_block_and_clamped_ghost(tmp_path, dtype, block):
    _lib_or_skip()
    dims = (21, 13, 17)                       # partial blocks on every axis
    npdt = np.float32 if dtype == "f32" else np.float16
    vol = np.random.default_rng(3).random(dims[::-1]).astype(npdt)
    raw, out = tmp_path / "v.raw", tmp_path / "v.brk"
    vol.tofile(raw)
    ngv.ooc_brick_file(raw, dims, dtype, block, out)
    data = out.read_bytes()
    assert data[:8] == b"NGVBRICK"
    G = [(d + block - 1) // block for d in dims]
    e = block + 2
    esz = np.dtype(npdt).itemsize
    rec = (e ** 3 * esz + 4095) // 4096 * 4096
    assert len(data) == 4096 + G[0] * G[1] * G[2] * rec
    for bz in range(G[2]):
        for by in range(G[1]):
            for bx in range(G[0]):
                bid = bx + G[0] * (by + G[1] * bz)
                r = np.frombuffer(data, npdt, e ** 3, 4096 + bid * rec).reshape(e, e, e)
                idx = [np.clip(np.arange(-1, block + 1) + o * block, 0, d - 1) for o, d in zip((bx, by, bz), dims)]
                expect = vol[np.ix_(idx[2], idx[1], idx[0])]
                np.testing.assert_array_equal(r, expect)


def test_brick_file_rejects_bad_inputs(tmp_path):
    _lib_or_skip()
    raw, out = tmp_path / "v.raw", tmp_path / "v.brk"
    np.zeros((4, 4, 4), np.float32).tofile(raw)
    with pytest.raises(RuntimeError):
        ngv.ooc_brick_file(raw, (4, 4, 5), "f32", 4, out)     # raw file too short
    with pytest.raises(RuntimeError):
        ngv.ooc_brick_file(raw, (4, 4, 4), "f32", 1, out)     # block too small
    with pytest.raises(RuntimeError):
        ngv.ooc_brick_file(tmp_path / "missing.raw", (4, 4, 4), "f32", 4, out)
