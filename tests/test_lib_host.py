"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and its plan/layout logic agrees with the oracle.  No
kernel is launched here."""
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ngv = pytest.importorskip("paper_2207_11620_amd")


def _lib_or_skip():
    if not os.path.exists(ngv.LIB_PATH):
        pytest.skip("libngvol.so not built")
    return ngv.lib()


def header_functions():
    src = open(os.path.join(ROOT, "include", "ngvol.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ngvol_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = _lib_or_skip()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(ngv.EXPORTED)


def test_nm_lists_symbols():
    _lib_or_skip()
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", ngv.LIB_PATH], capture_output=True, text=True).stdout
    for n in header_functions():
        assert re.search(rf"\bT {n}\b", out), n


CFG0 = dict(n_levels=8, n_features=2, log2_hashmap_size=14, base_resolution=4, per_level_scale=1.5, n_neurons=32,
            n_hidden_layers=2)
CFG1 = dict(n_levels=16, n_features=2, log2_hashmap_size=19, base_resolution=16, max_resolution=2048, n_neurons=64,
            n_hidden_layers=2)


@pytest.mark.parametrize("cfg,base,scale,maxr", [(CFG0, 4, 1.5, 0), (CFG1, 16, 0.0, 2048)])
def test_layout_matches_oracle(cfg, base, scale, maxr):
    _lib_or_skip()
    for prec in ("fp32", "bf16"):
        p = ngv.Plan(**cfg, precision=prec)
        res = oracle.resolutions(cfg["n_levels"], base, scale, maxr)
        assert p.resolution == res
        m = oracle.Model(cfg["n_levels"], 2, cfg["log2_hashmap_size"], res, cfg["n_neurons"], cfg["n_hidden_layers"])
        assert p.level_entries == list(m.level_size)
        assert p.level_offset == list(m.level_offset)
        assert (p.n_table_params, p.n_mlp_params, p.n_params) == (m.n_table, m.n_mlp, m.n_params)
        assert p.layer_offset[0] == m.n_table


def test_paper_configs_layout():
    _lib_or_skip()
    # Table-2 fixed network: L8 F8 T2^19 base 4, 64 wide, 4 hidden (parameter count pinned in the oracle tests)
    p = ngv.Plan(8, 8, 19, 4, 2.0, n_neurons=64, n_hidden_layers=4)
    res = oracle.resolutions(8, 4, 2.0)
    m = oracle.Model(8, 8, 19, res, 64, 4)
    assert p.n_params == m.n_params


def test_explicit_resolutions():
    _lib_or_skip()
    p = ngv.Plan(3, 2, 10, resolutions=[3, 7, 40], n_neurons=32, n_hidden_layers=1)
    assert p.resolution == [3, 7, 40]
    assert p.dense == [True, True, False]
    assert p.level_entries == [27, 343, 1024]


@pytest.mark.parametrize("kw,code", [
    (dict(n_levels=0), ngv.EINVAL),
    (dict(n_levels=33), ngv.EINVAL),
    (dict(n_features=3), ngv.EUNSUPPORTED),
    (dict(n_neurons=48), ngv.EUNSUPPORTED),
    (dict(n_levels=16, n_features=8), ngv.EUNSUPPORTED),
    (dict(log2_hashmap_size=40), ngv.EINVAL),
    (dict(n_hidden_layers=0), ngv.EINVAL),
    (dict(base_resolution=1), ngv.EINVAL),
    (dict(precision=7), ngv.EINVAL),
])
def test_plan_rejects(kw, code):
    _lib_or_skip()
    cfg = dict(CFG0)
    prec = kw.pop("precision", "fp32")
    cfg.update(kw)
    if prec == 7:
        with pytest.raises(KeyError):
            ngv.Plan(**cfg, precision=prec)
        return
    with pytest.raises(ngv.NgvolError) as ei:
        ngv.Plan(**cfg, precision=prec)
    assert ei.value.code == code


def test_null_arguments_rejected_without_launch():
    import ctypes as C
    L = _lib_or_skip()
    p = ngv.Plan(**CFG0)
    w = ngv.Weights(None, None)
    assert L.ngvol_infer(p.handle, C.byref(w), None, 10, None, None, 0, None) == ngv.EINVAL
    assert L.ngvol_infer(None, C.byref(w), None, 10, None, None, 0, None) == ngv.EINVAL
    assert b"NULL" in L.ngvol_last_error()
    # misaligned pointers are rejected before any launch
    w2 = ngv.Weights(C.c_void_p(16), None)
    assert L.ngvol_infer(p.handle, C.byref(w2), C.c_void_p(18), 10, C.c_void_p(32), None, 0, None) == ngv.EINVAL
    # n = 0 is a no-op even with null data pointers (after the weights check)
    assert L.ngvol_infer(p.handle, C.byref(w2), None, 0, None, None, 0, None) == ngv.OK
    # a workspace smaller than needed is refused
    nb = C.c_size_t()
    assert L.ngvol_infer_workspace_bytes(p.handle, 1 << 20, C.byref(nb)) == ngv.OK and nb.value > (1 << 20) * 16
    assert L.ngvol_infer(p.handle, C.byref(w2), C.c_void_p(32), 1 << 20, C.c_void_p(64), C.c_void_p(128), 64,
                         None) == ngv.ENOMEM
    assert L.ngvol_infer_workspace_bytes(p.handle, 1000, C.byref(nb)) == ngv.OK and nb.value == 0
    sz = C.c_size_t()
    assert L.ngvol_train_workspace_bytes(p.handle, 4096, C.byref(sz)) == ngv.OK
    assert sz.value > 4096 * 32 * 4


def _fake_state(p):
    """A training state whose device pointers are never dereferenced on the
    host (every call below is refused before any launch)."""
    import ctypes as C
    addr = lambda k: C.c_void_p(4096 * (k + 1))
    st = ngv.TrainStateC(addr(0), None, addr(1), addr(2), addr(3), addr(4), addr(5), addr(6), addr(7), 1 << 40)
    return st


def test_train_limits_checked_on_the_host():
    import ctypes as C
    L = _lib_or_skip()
    p = ngv.Plan(**CFG1)  # 16 levels: 128 table-gradient records per sample
    sz = C.c_size_t()
    # B * 8 * L = 2^32 records would overflow the scatter's 32-bit positions
    assert L.ngvol_train_workspace_bytes(p.handle, 1 << 25, C.byref(sz)) == ngv.EINVAL
    assert b"2^32" in L.ngvol_last_error()
    assert L.ngvol_train_workspace_bytes(p.handle, (1 << 25) - 1, C.byref(sz)) == ngv.OK
    st = _fake_state(p)
    batch = ngv.Batch(1 << 25, None, None, C.c_void_p(1 << 20), (C.c_int32 * 3)(64, 64, 64), 0, 1, 0, None)
    adam = ngv.Adam(1e-2, 0.9, 0.99, 1e-15, 0.0, 0, 0, 1.0)
    assert L.ngvol_train_step(p.handle, C.byref(st), C.byref(batch), C.byref(adam), 128.0, None) == ngv.EINVAL
    # a table whose gradient-bucket histogram exceeds the LDS: 2^28 entries of
    # 2 features = 65536 buckets of 2^12 entries
    big = ngv.Plan(1, 2, 28, resolutions=[1024], n_neurons=32, n_hidden_layers=1)
    assert L.ngvol_train_workspace_bytes(big.handle, 4096, C.byref(sz)) == ngv.EUNSUPPORTED
    batch.batch_size = 4096
    assert L.ngvol_train_step(big.handle, C.byref(st), C.byref(batch), C.byref(adam), 128.0, None) == ngv.EUNSUPPORTED
    ok = ngv.Plan(1, 2, 27, resolutions=[1024], n_neurons=32, n_hidden_layers=1)  # 32768 buckets: fits
    assert L.ngvol_train_workspace_bytes(ok.handle, 4096, C.byref(sz)) == ngv.OK


def test_output_activation_option():
    _lib_or_skip()
    p = ngv.Plan(**CFG0, output_activation="relu")
    assert p.output_activation == "relu"
    with pytest.raises(ngv.NgvolError) as ei:
        import ctypes as C
        cfg = ngv.Config(8, 2, 14, 4, 1.5, 0, None, 32, 2, 0, 0, 5)
        h = C.c_void_p()
        ngv._check(ngv.lib().ngvol_plan_create(C.byref(cfg), C.byref(h)))
    assert ei.value.code == ngv.EINVAL
