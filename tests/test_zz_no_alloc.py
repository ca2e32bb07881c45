"""fwi_misfit_noalloc (partial sums in the library's static device array,
no allocation) against fwi_misfit (partial sums in the caller's workspace),
through the C ABI: two calls in a row, the second on a smaller input (so it
runs after a call that filled the whole array).  Results must be bitwise
equal (same kernels, same reduction order)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_misfit_noalloc_matches_workspace_call():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_01184_amd import _lib as L
    from paper_1804_01184_amd import api
    from paper_1804_01184_amd import workloads as W

    dev = torch.device("cuda")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # 6 x 300 x 2500 samples use all 2048 partial sums; 2 x 7 x 13 use one
    for S, nrec, nt in ((6, 300, 2500), (2, 7, 13)):
        w = W.gauss_problem(61, S, nrec, nt, npml=10, seed=S)
        plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz)
        rng = np.random.default_rng(nt)
        d = torch.tensor(rng.standard_normal((S, nrec, nt)), dtype=torch.float32, device=dev)
        q = torch.tensor(rng.standard_normal((S, nrec, nt)), dtype=torch.float32, device=dev)
        J_ws, r_ws = plan.misfit(d, q)
        J = torch.full((1,), np.nan, dtype=torch.float32, device=dev)
        r = torch.full_like(d, np.nan)
        L.check(L.lib().fwi_misfit_noalloc(plan._h, ptr(d), ptr(q), ptr(r), ptr(J), stream))
        torch.cuda.synchronize()
        assert J.item() == J_ws.item()
        assert torch.equal(r, r_ws)
        ref = 0.5 * float(((d.double() - q.double()) ** 2).sum())
        assert abs(J.item() - ref) <= 1e-5 * ref
        # without a residual array
        J2 = torch.full((1,), np.nan, dtype=torch.float32, device=dev)
        L.check(L.lib().fwi_misfit_noalloc(plan._h, ptr(d), ptr(q), None, ptr(J2), stream))
        torch.cuda.synchronize()
        assert J2.item() == J_ws.item()
