"""GPU parity of out-of-core sampling (ngvol_ooc_*) against the oracle's
schedule and sampler: slot contents and sample coordinates bit-exact, targets
<= 1e-6, over the warm-up and several refreshes, including a refresh issued
while the previous samples are still to be consumed."""
import numpy as np
import pytest

import oracle
import synth

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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("dtype,block,dims", [("f32", 8, (37, 20, 29)), ("f16", 6, (48, 48, 48)),
                                              ("f32", 23, (64, 64, 64))])
def test_ooc_samples_match_oracle(tmp_path, dtype, block, dims):
    npdt = np.float32 if dtype == "f32" else np.float16
    vol = synth.gaussian_blobs(max(dims), 5)[:dims[2], :dims[1], :dims[0]].astype(npdt)
    raw, brk = tmp_path / "v.raw", tmp_path / "v.brk"
    np.ascontiguousarray(vol).tofile(raw)
    ngv.ooc_brick_file(raw, dims, dtype, block, brk)
    R, S, seed, B = 48, 12, 21, 6000
    ooc = ngv.OutOfCore(brk, R, S, seed, threads=4)
    v32 = vol.astype(np.float32)
    for step in range(4):
        ooc.refresh(step)
        xyz, y = ooc.sample(step, B)
        np.testing.assert_array_equal(ooc.slots(), oracle.ooc_slots(dims, block, R, S, seed, step).astype(np.int32))
        ox, oy, _ = oracle.ooc_sample(v32, block, R, S, seed, step, B)
        np.testing.assert_array_equal(host(xyz), ox)
        assert np.max(np.abs(host(y) - oy)) <= 1e-6
    ooc.close()


def test_ooc_refresh_overlaps_consumption(tmp_path):
    # order of a training loop: sample(k), refresh(k+1), [train on k], sample(k+1):
    # the samples of k are unaffected by the refresh that follows them
    dims, block = (64, 64, 64), 8
    vol = synth.fractal_value_noise(64, 3).astype(np.float32)
    raw, brk = tmp_path / "v.raw", tmp_path / "v.brk"
    vol.tofile(raw)
    ngv.ooc_brick_file(raw, dims, "f32", block, brk)
    R, S, B = 64, 32, 1 << 16
    ooc = ngv.OutOfCore(brk, R, S, 9, threads=8)
    ooc.refresh(0)
    for k in range(3):
        xyz, y = ooc.sample(k, B)
        ooc.refresh(k + 1)
        burn = torch.randn(4096, 4096, device="cuda") @ torch.randn(4096, 4096, device="cuda")  # the "step"
        ox, oy, _ = oracle.ooc_sample(vol, block, R, S, 9, k, B)
        np.testing.assert_array_equal(host(xyz), ox)
        assert np.max(np.abs(host(y) - oy)) <= 1e-6
        del burn
    ooc.close()


def test_ooc_train_step_with_buffered_samples(tmp_path):
    # the explicit-batch training step consumes out-of-core samples; with a
    # buffer covering the volume the model fits it about as well as with the
    # in-core sampler
    from models import gpu_plan, init_params
    dims, block = (48, 48, 48), 8
    vol = synth.gaussian_blobs(48, 2).astype(np.float32)
    raw, brk = tmp_path / "v.raw", tmp_path / "v.brk"
    vol.tofile(raw)
    ngv.ooc_brick_file(raw, dims, "f32", block, brk)
    ooc = ngv.OutOfCore(brk, 512, 64, 4, threads=4)
    p = gpu_plan("tiny", "fp32")
    p0 = torch.from_numpy(init_params("tiny")).cuda()
    vd = torch.from_numpy(vol).cuda()
    st = ngv.TrainState(p, p0, 4096)
    ref = ngv.TrainState(p, p0, 4096)
    ooc.refresh(0)
    for k in range(100):
        xyz, y = ooc.sample(k, 4096)
        ooc.refresh(k + 1)
        ngv.train_step(st, xyz=xyz, target=y, loss_scale=128.0)
        ngv.train_step(ref, volume=vd, seed=4, step_index=k, loss_scale=128.0)
    a = ngv.psnr(p, st.params, vd)
    b = ngv.psnr(p, ref.params, vd)
    print(f"PSNR after 100 steps: out-of-core {a:.2f} dB, in-core {b:.2f} dB")
    assert a > b - 3.0
    ooc.close()


def test_ooc_rejects_misuse(tmp_path):
    raw, brk = tmp_path / "v.raw", tmp_path / "v.brk"
    np.zeros((16, 16, 16), np.float32).tofile(raw)
    ngv.ooc_brick_file(raw, (16, 16, 16), "f32", 8, brk)
    with pytest.raises(RuntimeError):
        ngv.OutOfCore(raw, 4, 2, 1)                 # not a bricked file
    with pytest.raises(RuntimeError):
        ngv.OutOfCore(brk, 4, 5, 1)                 # S > R
    ooc = ngv.OutOfCore(brk, 4, 2, 1)
    with pytest.raises(RuntimeError):
        ooc.sample(0, 16)                           # before the warm-up
    ooc.refresh(0)
    with pytest.raises(RuntimeError):
        ooc.refresh(2)                              # out of order
    ooc.refresh(1)
    xyz, y = ooc.sample(1, 16)
    assert np.all(host(y) == 0)
    ooc.close()
