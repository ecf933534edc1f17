"""The allocation-free entry point mag_film_moment_noalloc against the moment
of mag_observe (the entry point it is a variant of), through the C ABI: two
calls in a row, the second on a smaller grid, and the size limit."""
import ctypes

import numpy as np
import pytest

from tests._cases import film_case, make_gpu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1801_04869_amd import _lib, api  # noqa: E402


def _noalloc(g, L, m):
    lib = _lib.lib()
    ny, nx = g.shape
    return lib.mag_film_moment_noalloc(ctypes.c_void_p(g.data_ptr()), nx, ny, L[0], L[1],
                                       ctypes.c_void_p(m.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_moment_matches_observe_on_two_calls():
    m = torch.full((3,), np.nan, dtype=torch.float64, device="cuda")
    for nx, ny, kind in ((512, 256, "ring"), (128, 64, "rect")):
        case = film_case(nx, ny, L=(2.0, 1.5), kind=kind, jc_s=0.1)
        ctx = make_gpu(case, api.FP64)
        g = torch.from_numpy(case["state"]).cuda()
        _, _, m_ref = ctx.observe(g, 0.2, want_hz=False, want_j=False)
        assert _noalloc(g, case["L"], m) == api.OK
        torch.cuda.synchronize()
        got = m.cpu().numpy()
        scale = float(np.abs(case["state"]).sum()) * (4.0 / nx) * (3.0 / ny)
        print("noalloc", nx, ny, got, m_ref, flush=True)
        assert got[0] == 0.0 and got[1] == 0.0
        assert abs(got[2] - m_ref[2]) <= 1e-13 * scale
        ctx.close()


def test_noalloc_moment_rejects_oversized_grids_and_null():
    m = torch.zeros(3, dtype=torch.float64, device="cuda")
    g = torch.zeros(8, dtype=torch.float64, device="cuda")
    lib = _lib.lib()
    big = 8192 * 2048 + 1
    # the size check comes before any use of g (nothing is enqueued)
    assert lib.mag_film_moment_noalloc(ctypes.c_void_p(g.data_ptr()), big, 1, 1.0, 1.0,
                                       ctypes.c_void_p(m.data_ptr()), None) == api.E_ARG
    assert lib.mag_film_moment_noalloc(None, 4, 2, 1.0, 1.0, ctypes.c_void_p(m.data_ptr()), None) == api.E_ARG
    assert lib.mag_film_moment_noalloc(ctypes.c_void_p(g.data_ptr()), 4, 2, 1.0, 1.0, None, None) == api.E_ARG
    # a small grid is accepted
    assert _noalloc(g[:8].reshape(2, 4), (1.0, 1.0), m) == api.OK
    torch.cuda.synchronize()
    assert m.cpu().numpy()[2] == 0.0
