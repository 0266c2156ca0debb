"""The allocation-free MLP backward (ngvol_mlp_bwd_noalloc) against the
workspace form (ngvol_mlp_bwd) on the same inputs, through the C-ABI.

Two calls in a row per model, the second with fewer samples: the scratch
array keeps the first call's partial sums, and the second call must not see
them.  Both entry points run the same kernels; their dW sums may differ in
order (LDS atomics, and a smaller grid where the scratch caps it), so the bar
is the FP32 gradient bar, 1e-4 normwise per block.  The Table-2 network
(16,448 MLP weights) fits 127 partial-sum rows in the 8 MiB scratch, fewer
than the workspace form's 256 workgroups at 2^18 samples: that case checks
the capped grid.
"""
import numpy as np
import pytest

from models import gpu_plan, init_params, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ngv = pytest.importorskip("paper_2207_11620_amd")


def _blocks(p):
    offs = list(p.layer_offset) + [p.n_params]
    return [(offs[i], offs[i + 1]) for i in range(len(p.layer_offset))]


@pytest.mark.parametrize("name,prec,sizes", [("tiny", "fp32", (5003, 1001)), ("cfg1", "bf16", (70001, 4099)),
                                             ("paper", "bf16", (1 << 18, 777))])
def test_noalloc_matches_workspace_form(name, prec, sizes):
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    p = gpu_plan(name, prec)
    params = torch.from_numpy(init_params(name, table_scale=0.3)).cuda()
    assert ngv.lib().ngvol_mlp_bwd_noalloc_scratch_bytes() == 8 << 20
    gen = torch.Generator(device="cuda").manual_seed(7)
    for call, n in enumerate(sizes):
        print(f"noalloc {name} {prec} call {call} n={n}", flush=True)
        feat = (torch.rand((n, p.n_input), generator=gen, device="cuda") - 0.5) * 0.2
        dout = torch.randn(n, generator=gen, device="cuda") * 1e-3
        g_ref = torch.zeros(p.n_params, device="cuda")
        g_new = torch.zeros(p.n_params, device="cuda")
        df_ref = ngv.mlp_bwd(p, params, feat, dout, g_ref)
        df_new = torch.full((n, p.n_input), float("nan"), device="cuda")
        ngv.mlp_bwd_noalloc(p, params, feat, dout, g_new, df_new)
        torch.cuda.synchronize()
        gr, gn = g_ref.cpu().numpy(), g_new.cpu().numpy()
        assert np.all(gn[: p.n_table_params] == 0.0)  # the table part is untouched
        for lo, hi in _blocks(p):
            assert rel_err(gn[lo:hi], gr[lo:hi]) <= 1e-4, (name, call, lo)
        assert rel_err(df_new.cpu().numpy(), df_ref.cpu().numpy()) <= 1e-4
