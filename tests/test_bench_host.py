"""Host-side logic of bench.py (no GPU): the refusal of more than one GPU, the
step byte model behind the roofline fractions, and the guard that drops the
committed HBM-traffic figure once the kernel sources change."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2409_11382_amd import problem as P  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_step_byte_model_of_the_benchmarked_schedule():
    """MG(3,4) with three cycles: each of the 2K sweeps reads and writes the 8
    populations and reads the 2 force components (plus the 2 reference
    components in shifted storage); the residual, restriction and prolongation
    add 14 values per fine cell per cycle; the coarse levels a third of the
    fine sweeps with their right-hand side; then the force, flow, extraction
    and re-basing passes (the displacement's at the step start, the pressure's
    in the flow step, the displacement reference between cycles).  3204 B per
    cell and step in FP32 shifted storage, 5768 B in FP64."""
    p = P.loaded_strip(n=512, alpha=1.0, ne_fixed=3)
    assert bench.step_bytes_per_cell(p, fp64=False, shifted=True) == pytest.approx(3204.0)
    assert bench.step_bytes_per_cell(p, fp64=True, shifted=False) == pytest.approx(5768.0)
    # one more cycle adds one cycle's sweeps and one more re-based reference
    q = p.replace(ne_fixed=4)
    d32 = bench.step_bytes_per_cell(q, False, True) - bench.step_bytes_per_cell(p, False, True)
    assert d32 == pytest.approx(4 * (2 * 4 * 20 + 14 + (2 * 4 * 24 + 20) / 3.0) + 4 * 2)


def test_traffic_figure_needs_matching_kernel_sources(monkeypatch):
    """The committed counter summary is used only while its recorded source
    hash matches the kernels being timed."""
    if not os.path.exists(bench.PMC_SUMMARY):
        pytest.skip("no committed counter summary")
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.measured_traffic() is None


def test_cpu_model_is_text_or_none():
    m = bench.cpu_model()
    assert m is None or (isinstance(m, str) and m)


def test_terzaghi_series_matches_the_analytic_module():
    """bench.py's own statement of the Terzaghi closed form (it may not import
    the oracle outside its CPU-baseline leg) against oracle/analytic.py."""
    import numpy as np
    from oracle import analytic as A

    lam, mu, c0, alpha, kappa, load = 1.0, 1.0, 0.1, 1.0, 1.0, 1.0
    c = A.terzaghi_constants(lam, mu, c0, alpha, kappa, load)
    y = (np.arange(128) + 0.5) / 128
    for t in (1e-5, 3e-3, 0.2):
        pa, Sa = bench.terzaghi_series(t, y, lam, mu, c0, alpha, kappa, load)
        assert np.abs(pa - A.terzaghi_p(t, y, c["p0"], c["cf"])).max() < 1e-12
        assert abs(Sa - A.terzaghi_S(t, c["S0"], c["Sinf"], c["cf"])) < 1e-12
