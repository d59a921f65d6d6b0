"""The allocation-free entry point (lbm_lee_compare_fields_static, file-scope device scratch)
against lbm_lee_compare_fields with a caller-owned workspace, through the C ABI."""
import numpy as np
import pytest

from tests._gpu import gpu_ok, say

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ok(), reason="needs a GPU")]


def test_compare_fields_static_matches_workspace_entry():
    """Two calls in a row, the second on smaller boxes: the results equal the workspace entry
    point's bit for bit (same kernels, same fixed reduction order), and the second call's result
    does not depend on what the first left in the shared scratch."""
    import torch
    from paper_1601_08103_amd import lbm
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(7)
    ws = torch.empty(lbm.lbm_lee_scratch_bytes(lbm.make_desc("D3Q7", "f32", (4, 4, 4))), dtype=torch.uint8,
                     device=dev)
    cases = [((40, 33, 70), (61, 50, 90), (7, 11, 3)),   # several blocks' worth of cells
             ((3, 5, 9), (4, 6, 17), (8, 0, 1))]         # then a smaller one
    for n_a, n_b, org in cases:
        say("compare_fields_static", n_a, n_b, org)
        a = torch.from_numpy(rng.standard_normal(n_a)).to(dev)
        b = torch.from_numpy(rng.standard_normal(n_b)).to(dev)
        dims_a = tuple(reversed(n_a))
        dims_b = tuple(reversed(n_b))
        got = lbm.lbm_lee_compare_fields_static(a.data_ptr(), dims_a, b.data_ptr(), dims_b, org, stream)
        want = lbm.lbm_lee_compare_fields(a.data_ptr(), dims_a, b.data_ptr(), dims_b, org, ws.data_ptr(),
                                          ws.numel(), stream)
        assert got == want
        # and the definition, in FP64 on the host
        bs = b.cpu().numpy()[org[2]:org[2] + n_a[0], org[1]:org[1] + n_a[1], org[0]:org[0] + n_a[2]]
        d = a.cpu().numpy() - bs
        assert abs(got[0] - np.sum(d * d)) <= 1e-12 * np.sum(d * d)
        assert abs(got[1] - np.sum(bs * bs)) <= 1e-12 * np.sum(bs * bs)
        assert got[2] == np.abs(d).max()
    with pytest.raises(lbm.LbmError):
        lbm.lbm_lee_compare_fields_static(a.data_ptr(), (10, 5, 3), b.data_ptr(), (9, 6, 4), (0, 0, 0), stream)
