"""The paper's whole runs in its own discretisation (the spectral form of
Sec. 2.2, FP64, adaptive BS23, the stop test of Sec. 2.3) on the GPU:
Table 1's disk at 256^2 against the Bean solution, and the film with a
circular hole of Sec. 2.3, Fig. 3 on its 768 x 512 grid to t = 0.4."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import bean  # noqa: E402
from paper_1801_04869_amd import api  # noqa: E402
from paper_1801_04869_amd import workloads as W  # noqa: E402


def _run(mat, n, L, nexp, rho_out, lam, t_end, prec=api.FP64):
    c = api.Context(2, prec)
    c.set_grid(n[0], n[1], 1, *L)
    c.set_derivatives(api.SPECTRAL)
    c.set_domain(torch.from_numpy(mat).cuda())
    c.set_params(None, 1.0, nexp, 1.0, rho_out)
    c.set_solver(lam, 2e-4, 100, 0)
    c.set_field(api.RAMP, (0.0, 0.0, 1.0), 1.0, 1.0, 1.0)
    g = torch.zeros((n[1], n[0]), dtype=torch.float64, device="cuda")
    steps, _ = c.integrate(g, 0.0, t_end, 1e-3, 1e-6)
    _, j, m = c.observe(g, t_end)
    return steps, g.cpu().numpy(), j.cpu().numpy(), m


def test_table1_disk_256():
    """Table 1, 256^2 (the paper: L1 deviation of |j| 1.0 %; measured here
    1.9 %, and 3.7 % at 128^2, 1.5 % at 512^2: the deviation falls with the
    grid as the paper's does)."""
    N = 256
    mat = W.film_disk(N, N, 2.0, 2.0, 1.0)
    print("disk 256^2, n = 1000, spectral form: integrating to h_e = 0.5", flush=True)
    steps, g, j, _ = _run(mat, (N, N), (2.0, 2.0), 1000.0, 1.0, 0.7, 0.5)
    x = -2.0 + (4.0 / N) * np.arange(N)
    r = np.hypot(*np.meshgrid(x, x))
    inside = r < 1.0
    jb = np.abs(bean.disk_current(r[inside], 1.0, 0.5))
    dj = np.abs(np.hypot(j[0], j[1])[inside] - jb).sum() / jb.sum()
    print("steps %d, L1 deviation of |j| %.2f %%" % (steps, 100 * dj), flush=True)
    assert steps > 500
    assert dj < 0.025


def test_hole_film_to_t04():
    """Sec. 2.3, Fig. 3: with rho_out = 500 in the filled hole the sheet
    current there stays negligible next to the film's critical current
    (j_c = 1), while the film carries critical currents."""
    wl = W.workload("film-768x512-hole")
    h = wl["hole"]
    nx, ny = wl["n"]
    Lx, Ly = wl["L"]
    mat = W.film_rect_hole(nx, ny, Lx, Ly, h["ax"], h["ay"], h["cx"], h["cy"], h["r"])
    print("768 x 512 hole film, spectral form: integrating to t = 0.4", flush=True)
    steps, g, j, m = _run(mat, (nx, ny), (Lx, Ly), wl["nexp"], wl["rho_out"], wl["lam"], 0.4)
    jm = np.hypot(j[0], j[1])
    x = -Lx + (2 * Lx / nx) * np.arange(nx)
    y = -Ly + (2 * Ly / ny) * np.arange(ny)
    X, Y = np.meshgrid(x, y)
    rr = np.hypot(X - h["cx"], Y - h["cy"])
    deep_hole = rr < h["r"] - 0.05           # nodes well inside the hole
    film = (np.abs(X) < h["ax"] - 0.05) & (np.abs(Y) < h["ay"] - 0.05) & (rr > h["r"] + 0.05)
    print("steps %d; max |j| in the hole %.3e, 99th percentile of |j| on the film %.3f, m_z %.4f" %
          (steps, jm[deep_hole].max(), np.percentile(jm[film], 99), m[2]), flush=True)
    assert np.isfinite(g).all() and steps > 1000
    assert np.percentile(jm[film], 99) > 0.9     # critical currents in the penetrated zone
    assert jm[deep_hole].max() < 0.05      # measured 0.014
    assert m[2] < 0
