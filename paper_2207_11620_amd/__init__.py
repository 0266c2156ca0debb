"""ngvol: neural-volume query and training on MI355X (gfx950).

Thin Python binding of the C-ABI in ``include/ngvol.h`` (``libngvol.so``,
built by ``python -m paper_2207_11620_amd.build``).  Every function marshals
torch tensors into device pointers and the current HIP stream and calls the
library; all arithmetic runs in the library's HIP kernels.  PyTorch supplies
device memory and streams only.  There is no fallback: if the library is not
built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libngvol.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4
FP32, BF16, FP16 = 0, 1, 2
DT_F32, DT_F16, DT_BF16 = 0, 1, 2
LOSS_L2, LOSS_L1 = 0, 1
MAX_LEVELS, MAX_LAYERS = 32, 9


class NgvolError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ngvol error {code}: {msg}")
        self.code = code


# --------------------------------------------------------------------------
# C structs (mirror include/ngvol.h)
# --------------------------------------------------------------------------
class Config(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_features", C.c_int32), ("log2_hashmap_size", C.c_int32),
                ("base_resolution", C.c_int32), ("per_level_scale", C.c_double), ("max_resolution", C.c_int32),
                ("resolutions", C.POINTER(C.c_int32)), ("n_neurons", C.c_int32), ("n_hidden_layers", C.c_int32),
                ("precision", C.c_int32), ("loss", C.c_int32), ("output_activation", C.c_int32)]


class Layout(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_features", C.c_int32), ("n_input", C.c_int32),
                ("n_neurons", C.c_int32), ("n_hidden_layers", C.c_int32), ("precision", C.c_int32),
                ("resolution", C.c_int32 * MAX_LEVELS), ("dense", C.c_int32 * MAX_LEVELS),
                ("level_entries", C.c_int64 * MAX_LEVELS), ("level_offset", C.c_int64 * (MAX_LEVELS + 1)),
                ("n_table_params", C.c_int64), ("n_mlp_params", C.c_int64), ("n_params", C.c_int64),
                ("layer_offset", C.c_int64 * MAX_LAYERS)]


class Weights(C.Structure):
    _fields_ = [("params", C.c_void_p), ("table_f16", C.c_void_p)]


class TrainStateC(C.Structure):
    _fields_ = [("params", C.c_void_p), ("table_f16", C.c_void_p), ("grad", C.c_void_p), ("adam_m", C.c_void_p),
                ("adam_v", C.c_void_p), ("step", C.c_void_p), ("skipped", C.c_void_p), ("loss", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t), ("draws", C.c_void_p)]


class MacroCellsC(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("cell", C.c_int32), ("range", C.c_void_p), ("mu", C.c_void_p)]


class Batch(C.Structure):
    _fields_ = [("batch_size", C.c_int64), ("xyz", C.c_void_p), ("target", C.c_void_p), ("volume", C.c_void_p),
                ("dims", C.c_int32 * 3), ("volume_dtype", C.c_int32), ("seed", C.c_uint64),
                ("step_index", C.c_int64), ("macrocells", C.c_void_p)]


class Adam(C.Structure):
    _fields_ = [("learning_rate", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("epsilon", C.c_double), ("l2_reg", C.c_double), ("decay_start", C.c_int64),
                ("decay_interval", C.c_int64), ("decay_base", C.c_double)]


class Camera(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("du", C.c_float * 3), ("dv", C.c_float * 3), ("dir00", C.c_float * 3)]


class RenderOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("adaptive", C.c_int32), ("step_max", C.c_float), ("step_exp", C.c_int32),
                ("light_dir", C.c_float * 3), ("light_radiance", C.c_float * 3), ("background", C.c_float * 3),
                ("density", C.c_float), ("spp", C.c_int32), ("rr_depth", C.c_int32), ("max_depth", C.c_int32),
                ("d_aux", C.c_void_p)]


RENDER_MODES = {"rm": 0, "rm_shadow": 1, "pt": 2}


class OocInfo(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("dtype", C.c_int32), ("block", C.c_int32), ("grid", C.c_int32 * 3),
                ("n_blocks", C.c_int64), ("record_bytes", C.c_int64), ("R", C.c_int64), ("S", C.c_int64)]


_P = C.c_void_p
_SIGS = {
    "ngvol_last_error": (C.c_char_p, []),
    "ngvol_version": (C.c_char_p, []),
    "ngvol_set_debug": (C.c_int, [C.c_int32]),
    "ngvol_plan_create": (C.c_int, [C.POINTER(Config), C.POINTER(_P)]),
    "ngvol_plan_destroy": (C.c_int, [_P]),
    "ngvol_get_layout": (C.c_int, [_P, C.POINTER(Layout)]),
    "ngvol_encode": (C.c_int, [_P, C.POINTER(Weights), _P, C.c_int64, _P, _P]),
    "ngvol_encode_debug": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P]),
    "ngvol_mlp_fwd": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P, _P]),
    "ngvol_infer_workspace_bytes": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_size_t)]),
    "ngvol_infer": (C.c_int, [_P, C.POINTER(Weights), _P, C.c_int64, _P, _P, C.c_size_t, _P]),
    "ngvol_sort_queries": (C.c_int, [_P, _P, C.c_int64, _P, C.c_size_t, _P]),
    "ngvol_infer_sorted": (C.c_int, [_P, C.POINTER(Weights), _P, C.c_int64, _P, _P]),
    "ngvol_mlp_bwd_workspace_bytes": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_size_t)]),
    "ngvol_mlp_bwd": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, _P, _P, C.c_size_t, _P]),
    "ngvol_mlp_bwd_noalloc_scratch_bytes": (C.c_size_t, []),
    "ngvol_mlp_bwd_noalloc": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, _P, _P]),
    "ngvol_encode_bwd": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P]),
    "ngvol_sample_batch": (C.c_int, [_P, C.POINTER(Batch), _P, _P, _P]),
    "ngvol_train_workspace_bytes": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_size_t)]),
    "ngvol_train_step": (C.c_int, [_P, C.POINTER(TrainStateC), C.POINTER(Batch), C.POINTER(Adam), C.c_float, _P]),
    "ngvol_adam_step": (C.c_int, [_P, C.POINTER(TrainStateC), C.POINTER(Adam), C.c_float, _P]),
    "ngvol_make_f16_tables": (C.c_int, [_P, _P, _P, _P]),
    "ngvol_sq_error_grid": (C.c_int, [_P, C.POINTER(Weights), _P, C.POINTER(C.c_int32), C.c_int32, _P, _P]),
    "ngvol_psnr": (C.c_int, [_P, C.POINTER(Weights), _P, C.POINTER(C.c_int32), C.c_int32, _P, _P, _P]),
    "ngvol_render_workspace_bytes": (C.c_size_t, []),
    "ngvol_render": (C.c_int, [_P, C.POINTER(Weights), C.POINTER(Camera), _P, C.c_int32, C.c_int32, C.c_float,
                               C.c_uint32, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "ngvol_render_ex": (C.c_int, [_P, C.POINTER(Weights), C.POINTER(Camera), _P, C.c_int32, C.c_int32, C.c_float,
                                  C.c_uint32, _P, C.POINTER(RenderOpts), _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "ngvol_mc_reset": (C.c_int, [_P, _P]),
    "ngvol_ooc_brick_file": (C.c_int, [C.c_char_p, _P, C.c_int32, C.c_int32, C.c_char_p]),
    "ngvol_ooc_open": (C.c_int, [C.c_char_p, C.c_int64, C.c_int64, C.c_uint64, C.c_int32, C.POINTER(_P)]),
    "ngvol_ooc_close": (C.c_int, [_P]),
    "ngvol_ooc_get_info": (C.c_int, [_P, C.POINTER(OocInfo)]),
    "ngvol_ooc_device_bytes": (C.c_size_t, [_P]),
    "ngvol_ooc_refresh": (C.c_int, [_P, C.c_int64, _P, _P]),
    "ngvol_ooc_sample": (C.c_int, [_P, C.c_int64, C.c_int64, _P, _P, _P, _P]),
    "ngvol_ooc_slots": (C.c_int, [_P, _P]),
    "ngvol_mc_update": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "ngvol_mc_opacity": (C.c_int, [_P, _P, _P]),
    "ngvol_multi_table_bytes": (C.c_size_t, [C.c_int32]),
    "ngvol_multi_create": (C.c_int, [C.POINTER(_P), C.c_int32, _P, C.c_size_t, _P, C.POINTER(_P)]),
    "ngvol_multi_destroy": (C.c_int, [_P]),
    "ngvol_multi_infer": (C.c_int, [_P, C.POINTER(Weights), C.POINTER(_P), C.POINTER(C.c_int64), C.POINTER(_P), _P]),
    "ngvol_multi_autotune": (C.c_int, [_P, C.POINTER(Weights), C.POINTER(_P), C.POINTER(C.c_int64), C.POINTER(_P),
                                       _P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ngvol_multi_train_step": (C.c_int, [_P, C.POINTER(TrainStateC), C.POINTER(Batch), C.POINTER(Adam), C.c_float,
                                         _P]),
}
EXPORTED = tuple(_SIGS)

_lib = None


def lib():
    """Load libngvol.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2207_11620_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise NgvolError(rc, lib().ngvol_last_error().decode())


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("ngvol needs device tensors")
    if not t.is_contiguous():
        raise ValueError("ngvol needs contiguous tensors")
    return C.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------
# Plan
# --------------------------------------------------------------------------
class Plan:
    """Resolved model: hash grid (L levels, F features, 2^log2T entries) + MLP."""

    def __init__(self, n_levels, n_features, log2_hashmap_size, base_resolution=16, per_level_scale=2.0,
                 max_resolution=0, resolutions=None, n_neurons=64, n_hidden_layers=2, precision="fp32", loss="l2",
                 output_activation="none"):
        prec = {"fp32": FP32, "bf16": BF16, "fp16": FP16, FP32: FP32, BF16: BF16, FP16: FP16}[precision]
        self.loss = loss
        loss_kind = {"l2": LOSS_L2, "l1": LOSS_L1}[loss]
        self._res = None
        if resolutions is not None:
            self._res = (C.c_int32 * len(resolutions))(*[int(r) for r in resolutions])
        cfg = Config(n_levels, n_features, log2_hashmap_size, base_resolution, float(per_level_scale),
                     int(max_resolution), C.cast(self._res, C.POINTER(C.c_int32)) if self._res else None,
                     n_neurons, n_hidden_layers, prec, loss_kind, {"none": 0, "relu": 1}[output_activation])
        self.output_activation = output_activation
        h = C.c_void_p()
        _check(lib().ngvol_plan_create(C.byref(cfg), C.byref(h)))
        self.handle = h
        lay = Layout()
        _check(lib().ngvol_get_layout(h, C.byref(lay)))
        L = lay.n_levels
        self.n_levels, self.n_features, self.n_input = L, lay.n_features, lay.n_input
        self.n_neurons, self.n_hidden_layers, self.precision = lay.n_neurons, lay.n_hidden_layers, lay.precision
        self.resolution = list(lay.resolution[:L])
        self.dense = [bool(d) for d in lay.dense[:L]]
        self.level_entries = list(lay.level_entries[:L])
        self.level_offset = list(lay.level_offset[:L + 1])
        self.n_table_params, self.n_mlp_params, self.n_params = lay.n_table_params, lay.n_mlp_params, lay.n_params
        self.layer_offset = list(lay.layer_offset[:lay.n_hidden_layers + 1])

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.ngvol_plan_destroy(h)
            self.handle = None


def _weights(params, table_f16=None):
    return Weights(_ptr(params), _ptr(table_f16))


def encode(plan, params, xyz, table_f16=None):
    torch = _torch()
    n = xyz.shape[0]
    feat = torch.empty((n, plan.n_input), dtype=torch.float32, device=xyz.device)
    w = _weights(params, table_f16)
    _check(lib().ngvol_encode(plan.handle, C.byref(w), _ptr(xyz), n, _ptr(feat), _stream()))
    return feat


def encode_debug(plan, xyz):
    torch = _torch()
    n = xyz.shape[0]
    idx = torch.empty((n, plan.n_levels, 8), dtype=torch.int32, device=xyz.device)
    w = torch.empty((n, plan.n_levels, 8), dtype=torch.float32, device=xyz.device)
    _check(lib().ngvol_encode_debug(plan.handle, _ptr(xyz), n, _ptr(idx), _ptr(w), _stream()))
    return idx, w


def mlp_fwd(plan, params, feat, out=None):
    torch = _torch()
    n = feat.shape[0]
    dt = {torch.float32: DT_F32, torch.bfloat16: DT_BF16, torch.float16: DT_F16}[feat.dtype]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=feat.device)
    _check(lib().ngvol_mlp_fwd(plan.handle, _ptr(params), _ptr(feat), dt, n, _ptr(out), _stream()))
    return out


def infer_workspace_bytes(plan, n):
    nb = C.c_size_t()
    _check(lib().ngvol_infer_workspace_bytes(plan.handle, n, C.byref(nb)))
    return nb.value


def infer(plan, params, xyz, table_f16=None, out=None, sort=True, workspace=None):
    """Phi(xyz).  sort=True groups the queries by spatial cell on the device
    first (same values, better cache locality); sort=False keeps the order."""
    torch = _torch()
    n = xyz.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=xyz.device)
    w = _weights(params, table_f16)
    nb = infer_workspace_bytes(plan, n) if sort else 0
    if nb and (workspace is None or workspace.numel() < nb):
        workspace = torch.empty(nb, dtype=torch.uint8, device=xyz.device)
    ws = workspace if nb else None
    _check(lib().ngvol_infer(plan.handle, C.byref(w), _ptr(xyz), n, _ptr(out), _ptr(ws), nb, _stream()))
    return out


def sort_queries(plan, xyz, workspace=None):
    """Group xyz by spatial cell into a workspace for infer_sorted."""
    torch = _torch()
    n = xyz.shape[0]
    nb = infer_workspace_bytes(plan, n)
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(max(nb, 256), dtype=torch.uint8, device=xyz.device)
    _check(lib().ngvol_sort_queries(plan.handle, _ptr(xyz), n, _ptr(workspace), workspace.numel(), _stream()))
    return workspace


def infer_sorted(plan, params, workspace, n, table_f16=None, out=None):
    torch = _torch()
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=workspace.device)
    w = _weights(params, table_f16)
    _check(lib().ngvol_infer_sorted(plan.handle, C.byref(w), _ptr(workspace), n, _ptr(out), _stream()))
    return out


def mlp_bwd(plan, params, feat, dout, grad, want_dfeat=True):
    """Adds dL/dW into grad's MLP block; returns dL/dfeat (or None)."""
    torch = _torch()
    n = feat.shape[0]
    nb = C.c_size_t()
    _check(lib().ngvol_mlp_bwd_workspace_bytes(plan.handle, n, C.byref(nb)))
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=feat.device)
    dfeat = torch.empty((n, plan.n_input), dtype=torch.float32, device=feat.device) if want_dfeat else None
    _check(lib().ngvol_mlp_bwd(plan.handle, _ptr(params), _ptr(feat), n, _ptr(dout), _ptr(dfeat), _ptr(grad),
                               _ptr(ws), nb.value, _stream()))
    return dfeat


def mlp_bwd_noalloc(plan, params, feat, dout, grad, dfeat=None):
    """ngvol_mlp_bwd_noalloc: adds dL/dW into grad's MLP block and, if a
    [n][n_input] FP32 dfeat tensor is given, writes dL/dfeat into it.  The
    library call allocates nothing (its scratch is a static device array)."""
    n = feat.shape[0]
    _check(lib().ngvol_mlp_bwd_noalloc(plan.handle, _ptr(params), _ptr(feat), n, _ptr(dout), _ptr(dfeat),
                                       _ptr(grad), _stream()))
    return dfeat


def encode_bwd(plan, xyz, dfeat, grad):
    _check(lib().ngvol_encode_bwd(plan.handle, _ptr(xyz), xyz.shape[0], _ptr(dfeat), _ptr(grad), _stream()))


_volume_fn_cls = None


def _volume_fn():
    """torch.autograd.Function over the library's forward and backward kernels."""
    global _volume_fn_cls
    if _volume_fn_cls is None:
        torch = _torch()

        class _VolumeFn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, params, xyz, plan, table_f16):
                feat = encode(plan, params, xyz, table_f16)
                y = mlp_fwd(plan, params, feat)
                ctx.plan = plan
                ctx.save_for_backward(params, xyz, feat)
                return y

            @staticmethod
            def backward(ctx, dy):
                params, xyz, feat = ctx.saved_tensors
                grad = torch.zeros_like(params)
                # MLP backward recomputes the activations from the features;
                # it adds dL/dW and returns dL/dfeature for the table scatter
                dfeat = mlp_bwd(ctx.plan, params, feat, dy.contiguous().to(torch.float32), grad)
                encode_bwd(ctx.plan, xyz, dfeat, grad)
                return grad, None, None, None

        _volume_fn_cls = _VolumeFn
    return _volume_fn_cls


def volume(plan, params, xyz, table_f16=None):
    """Phi(xyz) as a differentiable torch op.  Gradients flow to `params` (the
    level tables and the MLP) through the library's backward kernels; the
    coordinates get none.  With `table_f16` the forward reads the FP16 table
    shadow (the gradient is that of the shadowed model)."""
    return _volume_fn().apply(params, xyz, plan, table_f16)


def _volume_batch(volume, B, seed, step):
    torch = _torch()
    dt = {torch.float32: DT_F32, torch.float16: DT_F16}[volume.dtype]
    Dz, Dy, Dx = volume.shape
    return Batch(B, None, None, _ptr(volume), (C.c_int32 * 3)(Dx, Dy, Dz), dt, seed, step, None)


def sample_batch(plan, volume, B, seed, step):
    torch = _torch()
    xyz = torch.empty((B, 3), dtype=torch.float32, device=volume.device)
    y = torch.empty(B, dtype=torch.float32, device=volume.device)
    b = _volume_batch(volume, B, seed, step)
    _check(lib().ngvol_sample_batch(plan.handle, C.byref(b), _ptr(xyz), _ptr(y), _stream()))
    return xyz, y


def make_f16_tables(plan, params, out=None):
    torch = _torch()
    if out is None:
        out = torch.empty(plan.n_table_params, dtype=torch.float16, device=params.device)
    _check(lib().ngvol_make_f16_tables(plan.handle, _ptr(params), _ptr(out), _stream()))
    return out


class TrainState:
    """Device buffers of a training run (FP32 master, optional FP16 table shadow)."""

    def __init__(self, plan, params, batch_size, f16_tables=False):
        torch = _torch()
        dev = params.device
        self.plan = plan
        self.params = params.detach().clone().contiguous()
        self.table_f16 = make_f16_tables(plan, self.params) if f16_tables else None
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = torch.zeros(1, dtype=torch.int64, device=dev)
        self.draws = torch.zeros(1, dtype=torch.int64, device=dev)
        self.skipped = torch.zeros(1, dtype=torch.int32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        nb = C.c_size_t()
        _check(lib().ngvol_train_workspace_bytes(plan.handle, batch_size, C.byref(nb)))
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        self.batch_size = batch_size
        self._c = TrainStateC(_ptr(self.params), _ptr(self.table_f16), _ptr(self.grad), _ptr(self.m), _ptr(self.v),
                              _ptr(self.step), _ptr(self.skipped), _ptr(self.loss), _ptr(self.workspace), nb.value,
                              _ptr(self.draws))

    def weights(self):
        return self.params, self.table_f16


def _adam(lr, betas, eps, l2_reg, decay):
    start, interval, base = decay if decay is not None else (0, 0, 1.0)
    return Adam(lr, betas[0], betas[1], eps, l2_reg, int(start), int(interval), float(base))


def train_step(state, volume=None, seed=0, step_index=0, xyz=None, target=None, lr=1e-2, betas=(0.9, 0.99),
               eps=1e-15, loss_scale=1.0, l2_reg=0.0, decay=None, macrocells=None):
    """One training step.  step_index=-1 draws the batch indexed by the state's
    device draw counter (steps taken, applied or skipped: the form to capture
    in a graph).  decay =
    (start, interval, base) gives the exponentially decaying learning rate;
    l2_reg regularises the MLP weights; macrocells (a MacroCells) takes the
    batch's samples into its value ranges."""
    B = state.batch_size
    if xyz is not None:
        b = Batch(B, _ptr(xyz), _ptr(target), None, (C.c_int32 * 3)(0, 0, 0), 0, 0, 0, None)
    else:
        b = _volume_batch(volume, B, seed, step_index)
    if macrocells is not None:
        b.macrocells = C.cast(C.pointer(macrocells._c), C.c_void_p)
    a = _adam(lr, betas, eps, l2_reg, decay)
    _check(lib().ngvol_train_step(state.plan.handle, C.byref(state._c), C.byref(b), C.byref(a),
                                  float(loss_scale), _stream()))


def adam_step(state, lr=1e-2, betas=(0.9, 0.99), eps=1e-15, loss_scale=1.0, l2_reg=0.0, decay=None):
    a = _adam(lr, betas, eps, l2_reg, decay)
    _check(lib().ngvol_adam_step(state.plan.handle, C.byref(state._c), C.byref(a), float(loss_scale), _stream()))


def sq_error_grid(plan, params, volume, table_f16=None, out=None):
    """Device FP64 sum of squared errors over all voxel centres."""
    torch = _torch()
    if out is None:
        out = torch.zeros(1, dtype=torch.float64, device=volume.device)
    dt = {torch.float32: DT_F32, torch.float16: DT_F16}[volume.dtype]
    Dz, Dy, Dx = volume.shape
    dims = (C.c_int32 * 3)(Dx, Dy, Dz)
    w = _weights(params, table_f16)
    _check(lib().ngvol_sq_error_grid(plan.handle, C.byref(w), _ptr(volume), dims, dt, _ptr(out), _stream()))
    return out


def psnr(plan, params, volume, table_f16=None, out=None):
    """ngvol_psnr: (MSE, PSNR) over all voxel centres, reduced in FP64 on the
    device; out (two float64 device values) receives them."""
    torch = _torch()
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=volume.device)
    dt = {torch.float32: DT_F32, torch.float16: DT_F16}[volume.dtype]
    Dz, Dy, Dx = volume.shape
    dims = (C.c_int32 * 3)(Dx, Dy, Dz)
    w = _weights(params, table_f16)
    _check(lib().ngvol_psnr(plan.handle, C.byref(w), _ptr(volume), dims, dt, _ptr(out), _ptr(out[1:]), _stream()))
    mse, p = out.tolist()
    return p


def render(plan, params, cam, lut, width, height, dt, frame_seed, table_f16=None, want_counts=True,
           rgba=None, workspace=None, counters=None, macrocells=None, adaptive=False, step_max=64.0, step_exp=2,
           mode="rm", light=(0.0, 0.0, 1.0), radiance=(1.0, 1.0, 1.0), background=(0.0, 0.0, 0.0), density=1.0,
           spp=1, rr_depth=4, max_depth=1024, aux=None):
    """Returns (rgba [H][W][4], n_geo [H][W] or None, n_used or None, counters [4] int64).
    macrocells (a MacroCells with opacities set): skip samples in empty cells;
    with adaptive=True also march with steps of up to step_max grid steps,
    shortened by the cells' opacities with exponent step_exp.  mode "rm_shadow"
    adds a single-shot shadow towards `light`; mode "pt" path-traces the
    volume (density, light, radiance, background, spp, rr_depth, max_depth;
    macro-cells give per-cell majorants).  aux: optional int32 [H][W] output
    (rm_shadow: index of the shading sample).  Options go through
    ngvol_render_ex."""
    torch = _torch()
    dev = params.device
    if rgba is None:
        rgba = torch.empty((height, width, 4), dtype=torch.float32, device=dev)
    n_geo = torch.empty((height, width), dtype=torch.int32, device=dev) if want_counts else None
    n_used = torch.empty((height, width), dtype=torch.int32, device=dev) if want_counts else None
    if workspace is None:
        workspace = torch.empty(int(lib().ngvol_render_workspace_bytes()), dtype=torch.uint8, device=dev)
    if counters is None:
        counters = torch.zeros(4, dtype=torch.int64, device=dev)
    c = [float(v) for v in cam]
    camc = Camera((C.c_float * 3)(*c[0:3]), (C.c_float * 3)(*c[3:6]), (C.c_float * 3)(*c[6:9]),
                  (C.c_float * 3)(*c[9:12]))
    w = _weights(params, table_f16)
    mcp = C.byref(macrocells._c) if macrocells is not None else None
    if adaptive or mode != "rm" or aux is not None:
        if adaptive and macrocells is None:
            raise ValueError("adaptive marching needs macrocells")
        if mode == "rm_shadow" and aux is None:
            aux = torch.empty((height, width), dtype=torch.int32, device=dev)
        f3 = C.c_float * 3
        opts = RenderOpts(RENDER_MODES[mode], 1 if adaptive else 0, float(step_max), int(step_exp),
                          f3(*[float(v) for v in light]), f3(*[float(v) for v in radiance]),
                          f3(*[float(v) for v in background]), float(density), int(spp), int(rr_depth),
                          int(max_depth), _ptr(aux))
        _check(lib().ngvol_render_ex(plan.handle, C.byref(w), C.byref(camc), _ptr(lut), width, height, float(dt),
                                     frame_seed, mcp, C.byref(opts), _ptr(rgba), _ptr(n_geo), _ptr(n_used),
                                     _ptr(counters), _ptr(workspace), workspace.numel(), _stream()))
    else:
        _check(lib().ngvol_render(plan.handle, C.byref(w), C.byref(camc), _ptr(lut), width, height, float(dt),
                                  frame_seed, mcp, _ptr(rgba), _ptr(n_geo), _ptr(n_used), _ptr(counters),
                                  _ptr(workspace), workspace.numel(), _stream()))
    return rgba, n_geo, n_used, counters


class MacroCells:
    """Macro-cell grid (cells of `cell` voxels per axis) over a volume of
    dims = (Dx, Dy, Dz) voxels, with device value ranges and opacities."""

    def __init__(self, dims, cell=64, device="cuda"):
        torch = _torch()
        self.dims = tuple(int(d) for d in dims)
        self.cell = int(cell)
        self.grid = tuple((d + self.cell - 1) // self.cell for d in self.dims)
        n = self.grid[0] * self.grid[1] * self.grid[2]
        self.range = torch.empty(2 * n, dtype=torch.int32, device=device)
        self.mu = torch.zeros(n, dtype=torch.float32, device=device)
        self._c = MacroCellsC((C.c_int32 * 3)(*self.dims), self.cell, _ptr(self.range), _ptr(self.mu))
        self.reset()

    def reset(self):
        _check(lib().ngvol_mc_reset(C.byref(self._c), _stream()))

    def update(self, xyz, values):
        _check(lib().ngvol_mc_update(C.byref(self._c), _ptr(xyz), _ptr(values), xyz.shape[0], _stream()))

    def opacity(self, lut):
        _check(lib().ngvol_mc_opacity(C.byref(self._c), _ptr(lut), _stream()))

    def ranges(self):
        """(vmin, vmax) per cell as float64 numpy arrays (+inf, -inf when empty)."""
        import numpy as np
        _torch().cuda.synchronize()
        k = self.range.cpu().numpy().view(np.uint32).reshape(-1, 2)
        def val(key):
            bits = np.where(key & 0x80000000, key & 0x7FFFFFFF, ~key).astype(np.uint32)
            return bits.view(np.float32).astype(np.float64)
        lo, hi = val(k[:, 0]), val(k[:, 1])
        empty = k[:, 0] > k[:, 1]
        lo[empty], hi[empty] = np.inf, -np.inf
        return lo, hi


def version():
    return lib().ngvol_version().decode()


def set_debug(on=True):
    """Synchronise and check for device errors after every library call."""
    _check(lib().ngvol_set_debug(1 if on else 0))


class Multi:
    """A group of independent models (same MLP shape, F = 2) queried in one launch."""

    def __init__(self, plans):
        torch = _torch()
        k = len(plans)
        self.plans = list(plans)
        self.table = torch.empty(max(int(lib().ngvol_multi_table_bytes(k)), 256), dtype=torch.uint8, device="cuda")
        arr = (_P * k)(*[p.handle for p in plans])
        h = C.c_void_p()
        _check(lib().ngvol_multi_create(arr, k, _ptr(self.table), self.table.numel(), _stream(), C.byref(h)))
        self.handle = h
        self.k = k

    def _args(self, weights, xyz, outs):
        k = self.k
        W = (Weights * k)(*[_weights(p, f) for (p, f) in weights])
        X = (_P * k)(*[_ptr(x) for x in xyz])
        N = (C.c_int64 * k)(*[x.shape[0] for x in xyz])
        O = (_P * k)(*[_ptr(o) for o in outs])
        return W, X, N, O

    def infer(self, weights, xyz, outs=None):
        """weights: list of (params, table_f16 or None); xyz: list of [n_i][3] tensors."""
        torch = _torch()
        if outs is None:
            outs = [torch.empty(x.shape[0], dtype=torch.float32, device=x.device) for x in xyz]
        W, X, N, O = self._args(weights, xyz, outs)
        _check(lib().ngvol_multi_infer(self.handle, W, X, N, O, _stream()))
        return outs

    def autotune(self, weights, xyz, outs):
        W, X, N, O = self._args(weights, xyz, outs)
        b, c = C.c_int32(), C.c_int32()
        _check(lib().ngvol_multi_autotune(self.handle, W, X, N, O, _stream(), C.byref(b), C.byref(c)))
        return b.value, c.value

    def train_step(self, states, volumes, seeds, step_index=-1, lr=1e-2, betas=(0.9, 0.99), eps=1e-15,
                   loss_scale=1.0, l2_reg=0.0, decay=None):
        """ngvol_multi_train_step: one training step of every model (states[i]
        on generated batches of volumes[i] with seeds[i]); step_index -1 draws
        each model's batch by its device draw counter (graph-replayable)."""
        k = self.k
        S = (TrainStateC * k)(*[st._c for st in states])
        Bt = (Batch * k)(*[_volume_batch(v, st.batch_size, sd, step_index) for st, v, sd in zip(states, volumes, seeds)])
        a = _adam(lr, betas, eps, l2_reg, decay)
        _check(lib().ngvol_multi_train_step(self.handle, S, Bt, C.byref(a), float(loss_scale), _stream()))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.ngvol_multi_destroy(h)
            self.handle = None


def ooc_brick_file(raw_path, dims, dtype, block, bricked_path):
    """ngvol_ooc_brick_file: bricked copy (block^3 voxels per record plus a
    ghost layer) of a raw [Dz][Dy][Dx] volume; dtype "f32" or "f16"."""
    dt = {"f32": DT_F32, "f16": DT_F16}[dtype]
    d = (C.c_int32 * 3)(*[int(v) for v in dims])
    _check(lib().ngvol_ooc_brick_file(os.fsencode(raw_path), d, dt, int(block), os.fsencode(bricked_path)))


class OutOfCore:
    """Out-of-core sampler over a bricked volume file: R device-resident block
    slots (S refreshed per step), samples drawn on the device."""

    def __init__(self, bricked_path, R, S, seed, threads=8, device="cuda"):
        torch = _torch()
        h = C.c_void_p()
        _check(lib().ngvol_ooc_open(os.fsencode(bricked_path), int(R), int(S), int(seed), int(threads),
                                    C.byref(h)))
        self._h = h
        self.info = OocInfo()
        _check(lib().ngvol_ooc_get_info(h, C.byref(self.info)))
        self.buf = torch.empty(int(lib().ngvol_ooc_device_bytes(h)), dtype=torch.uint8, device=device)

    def refresh(self, step):
        _check(lib().ngvol_ooc_refresh(self._h, int(step), _ptr(self.buf), _stream()))

    def sample(self, step, B, xyz=None, target=None):
        torch = _torch()
        if xyz is None:
            xyz = torch.empty((B, 3), dtype=torch.float32, device=self.buf.device)
        if target is None:
            target = torch.empty(B, dtype=torch.float32, device=self.buf.device)
        _check(lib().ngvol_ooc_sample(self._h, int(step), int(B), _ptr(self.buf), _ptr(xyz), _ptr(target),
                                      _stream()))
        return xyz, target

    def slots(self):
        import numpy as np
        out = np.zeros(self.info.R, np.int32)
        _check(lib().ngvol_ooc_slots(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value is not None:
            lib().ngvol_ooc_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
