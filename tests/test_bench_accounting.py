"""Host-side accounting of bench.py (CPU only): the free-space node count that
the algorithmic bytes use, the bytes themselves, and the reading of the
recorded HBM traffic.  The GPU figures bench.py prints rest on these."""
import numpy as np

import bench
from paper_1801_04869_amd import workloads as W


def test_free_nodes_matches_brute_force():
    """A node is inside when the four cells around it are film (periodic)."""
    rng = np.random.default_rng(3)
    mat = (rng.random((12, 16)) < 0.6).astype(np.uint8)
    ny, nx = mat.shape
    inside = 0
    for q in range(ny):
        for p in range(nx):
            cells = [mat[q % ny, p % nx], mat[q % ny, (p - 1) % nx], mat[(q - 1) % ny, p % nx],
                     mat[(q - 1) % ny, (p - 1) % nx]]
            inside += all(c != 0 for c in cells)
    assert bench.free_nodes(mat) == mat.size - inside


def test_algorithmic_bytes_of_the_benchmark_passes():
    """At 2048^2 (mixed, 4 iterations) the per-launch bytes follow from the
    arrays each pass reads and writes once."""
    n, kx, ny = 2048 * 2048, 1025, 2048
    mat = W.film_ring(2048, 2048, 2.0, 2.0, 0.5, 1.0)
    n_out = bench.free_nodes(mat)
    assert 0 < n_out < n
    spec = 8 * kx * ny   # FP32 complex half spectrum
    K = 4
    assert bench.alg_bytes("film_cols", n, kx, ny, "mixed", K, n_out) == round(7 * 2 * spec / 8)
    assert bench.alg_bytes("film_rows_inv_g", n, kx, ny, "mixed", K, n_out) == round(2 * spec + 4 * n + 8 * n / K)
    assert bench.alg_bytes("film_rows_inv_upd", n, kx, ny, "mixed", K, n_out) == 2 * spec + 8 * n + 4 * n_out
    # FP64 doubles every complex and iterate entry
    assert bench.alg_bytes("film_cols", n, kx, ny, "fp64", K, n_out) == \
        2 * bench.alg_bytes("film_cols", n, kx, ny, "mixed", K, n_out)
    assert bench.alg_bytes("unknown_kernel", n, kx, ny, "mixed", K, n_out) is None


def test_recorded_traffic_is_read_only_for_matching_sources(tmp_path, monkeypatch):
    """A traffic line is used only while its source hash matches."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = bench.sources_hash()
    (prof / "x_film2048_mixed.md").write_text(
        "text\n    traffic film_cols mixed bytes_per_launch=123 sources_sha256_16=%s\n"
        "    traffic film_stencil mixed bytes_per_launch=7 sources_sha256_16=0000000000000000\n" % h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_hash", lambda: h)
    assert bench.recorded_traffic("film_cols", "mixed") == 123
    assert bench.recorded_traffic("film_stencil", "mixed") is None
    assert bench.recorded_traffic("film_rows_inv_g", "mixed") is None
