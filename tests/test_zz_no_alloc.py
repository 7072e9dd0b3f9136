"""GPU check of sg_conv3d_bwd_data_noalloc, the input gradient that takes
its mirrored weights from the library's fixed device array instead of a
workspace: same output as sg_conv3d_bwd_data, on two calls in a row (the
second smaller, so stale contents of the array would show), and within the
oracle's bound."""
import numpy as np
import pytest

from oracle import conv as oc

pytestmark = pytest.mark.gpu

EPS32 = float(np.finfo(np.float32).eps)


def _bf16(torch, a):
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda").to(torch.bfloat16)
    return t, t.float().cpu().numpy().astype(np.float64)


def _ulp_bf16(v):
    e = np.floor(np.log2(np.maximum(np.abs(v), 2.0 ** -126)))
    return 2.0 ** (e - 7)


def test_bwd_data_noalloc_matches_workspace_variant():
    import torch
    assert torch.cuda.is_available()
    from paper_2012_06144_amd import sg

    # the first call fills most of the 4 MiB array (256 x 256 x 27 x 2 B =
    # 3.5 MiB); the second mirrors a smaller weight set into its start
    for case in [(1, 4, 6, 20, 256, 256), (2, 3, 5, 7, 32, 48)]:
        n, d, h, w, ci, co = case
        print(f"no-alloc input gradient, case {case}", flush=True)
        rng = np.random.default_rng(7 * sum(case))
        dyt, dy = _bf16(torch, rng.standard_normal((n, d, h, w, co)))
        wt, wv = _bf16(torch, rng.standard_normal((27, co, ci)) / np.sqrt(27 * co))
        wm = torch.empty((27, ci, co), device="cuda", dtype=torch.bfloat16)
        ref_dx = torch.empty((n, d, h, w, ci), device="cuda", dtype=torch.bfloat16)
        dx = torch.full((n, d, h, w, ci), float("nan"), device="cuda", dtype=torch.bfloat16)
        sg.sg_conv3d_bwd_data(dyt, wt, ref_dx, wm)
        sg.sg_conv3d_bwd_data_noalloc(dyt, wt, dx)
        torch.cuda.synchronize()
        # same kernels on the same operands: identical bits
        assert torch.equal(dx.view(torch.int16), ref_dx.view(torch.int16))
        ref = oc.conv3d_bwd_data(dy, wv)
        mag = oc.conv3d_bwd_data(np.abs(dy), np.abs(wv))
        bound = 27 * co * EPS32 * mag + 0.5 * _ulp_bf16(ref) + 1e-30
        got = dx.float().cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


def test_bwd_data_noalloc_rejects_weights_beyond_the_array():
    import torch
    assert torch.cuda.is_available()
    from paper_2012_06144_amd import sg

    # 27 x 256 x 320 x 2 B = 4.2 MiB > 4 MiB: refused on the host, nothing launched
    dy = torch.zeros((1, 2, 2, 2, 320), device="cuda", dtype=torch.bfloat16)
    wt = torch.zeros((27, 320, 256), device="cuda", dtype=torch.bfloat16)
    dx = torch.zeros((1, 2, 2, 2, 256), device="cuda", dtype=torch.bfloat16)
    with pytest.raises(sg.SgError, match="fixed scratch"):
        sg.sg_conv3d_bwd_data_noalloc(dy, wt, dx)
