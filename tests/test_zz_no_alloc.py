"""The allocation-free entry point dg_column_stats_noalloc (its scratch a static device array of the
library) against dg_column_stats (caller workspace), through the C ABI: the same bits, on two
calls in a row, the second with fewer rows and columns (the array keeps the first call's partials;
each call must overwrite what it reads)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dgm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_09079_amd import dg
    dg.lib()
    return dg


def noalloc(dgm, x):
    rows, cols = x.shape
    out = [torch.empty(cols, dtype=torch.float64, device="cuda") for _ in range(4)]
    s = torch.cuda.current_stream()
    st = dgm.lib().dg_column_stats_noalloc(ctypes.c_void_p(x.data_ptr()), rows, cols,
                                           *[ctypes.c_void_p(o.data_ptr()) for o in out],
                                           ctypes.c_void_p(s.cuda_stream))
    assert st == dgm.DG_OK, dgm.lib().dg_error_string(None)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


@pytest.mark.parametrize("shapes", [((5000, 140), (700, 20)), ((3000, 160), (5, 7))])
def test_noalloc_matches_workspace_entry_point(dgm, shapes):
    g = torch.Generator(device="cpu").manual_seed(4)
    for rows, cols in shapes:
        x = (torch.randn(rows, cols, generator=g) * 3.0 + torch.arange(cols) * 0.5).to("cuda", torch.float32)
        want = [t.cpu().numpy() for t in dgm.column_stats(x)]
        got = noalloc(dgm, x)
        for name, a, b in zip(("mean", "std", "rms", "maxabs"), got, want):
            assert np.array_equal(a, b), (rows, cols, name, np.abs(a - b).max())
        # and the statistics themselves, against numpy in FP64
        xh = x.cpu().double().numpy()
        np.testing.assert_allclose(got[0], xh.mean(axis=0), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(got[1], xh.std(axis=0), rtol=1e-10)
        np.testing.assert_allclose(got[3], np.abs(xh).max(axis=0), rtol=0, atol=0)


def test_noalloc_rejects_too_many_columns(dgm):
    x = torch.zeros(10, 161, device="cuda", dtype=torch.float32)
    out = [torch.empty(161, dtype=torch.float64, device="cuda") for _ in range(4)]
    st = dgm.lib().dg_column_stats_noalloc(ctypes.c_void_p(x.data_ptr()), 10, 161,
                                           *[ctypes.c_void_p(o.data_ptr()) for o in out], None)
    assert st == dgm.DG_ERR_ARG
