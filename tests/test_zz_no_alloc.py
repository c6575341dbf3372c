"""The allocation-free region sum (chebtd_region_sum_noalloc) against the
context's chebtd_region_sum, through the C ABI: two calls in a row, the second
on a smaller input, bit for bit (the same kernels), plus the size limit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_region_sum_noalloc_matches_context_entry_point():
    import torch
    import paper_0907_3022_amd as P
    from paper_0907_3022_amd import _lib as L

    assert torch.cuda.is_available()
    P.load_library()
    outs = []
    # a ragged ribbon, then a smaller chain: the fixed scratch keeps the
    # first call's partials, the second must not read them
    for (w, l, seed) in ((96, 4099, 1), (1, 777, 2)):
        n = w * l
        eps = torch.from_numpy(W.anderson_disorder(w, l, 0.5, seed)).cuda()
        psi = torch.from_numpy(W.random_state(n, 40 + seed)).cuda()
        mask = torch.from_numpy((W.random_weights(n, 50 + seed) < 0.5).astype(np.uint8)).cuda()
        ctx = P.Context()
        ctx.honeycomb(w, l, eps)
        ref = ctx.region_sum(psi, mask)
        out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        print(f"[gpu] region_sum_noalloc n={n}", flush=True)
        P.region_sum_noalloc(psi, mask, out)
        torch.cuda.synchronize()
        assert out.item() == ref.item()  # bit for bit
        host = psi.cpu().numpy()
        exact = float(np.sum(np.abs(host[mask.cpu().numpy() == 1]) ** 2))
        assert out.item() == pytest.approx(exact, rel=1e-13)
        outs.append(out.item())
        ctx.close()
    assert outs[0] != outs[1]
    # beyond the fixed scratch: refused with CHEBTD_E_ARG before any launch
    import ctypes as C
    big = L.CHEBTD_NOALLOC_MAX_SITES if hasattr(L, "CHEBTD_NOALLOC_MAX_SITES") else 16777216
    dummy = torch.zeros(2, dtype=torch.float64, device="cuda")
    rc = L.lib().chebtd_region_sum_noalloc(C.c_void_p(dummy.data_ptr()), C.c_void_p(dummy.data_ptr()),
                                           big + 1, C.c_void_p(dummy.data_ptr()), None)
    assert rc == L.E_ARG
    assert "outside" in L.last_error(None)
