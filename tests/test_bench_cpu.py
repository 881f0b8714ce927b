"""Host logic of bench.py (no GPU): when a committed rocprofv3 counter
summary may be reported as the kernel's HBM traffic, and the --gpus guard."""
from __future__ import annotations

import os
import subprocess
import sys

import bench


def _tree(root, kernel_src="// kernel v1\n"):
    csrc = root / "paper_1102_1343_amd" / "csrc"
    csrc.mkdir(parents=True, exist_ok=True)
    (csrc / "fire_kernels.hip").write_text(kernel_src)
    (csrc / "fire_internal.h").write_text("// header\n")
    (root / "profiles").mkdir(exist_ok=True)


def _summary(root, name, hbm, tile, digest):
    (root / "profiles" / name).write_text(
        f"# counters\nhbm_bytes_per_launch: {hbm:.6e}\ntile: {tile}\n"
        f"kernel_source_sha256_16: {digest}\n")


def test_traffic_needs_current_source_and_same_tile(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _tree(tmp_path)
    h = bench.kernel_source_hash()
    _summary(tmp_path, "k_step_patchy8192_f32_pmc.txt", 2.2e9, "120x20", h)
    assert bench.pmc_traffic("patchy8192", "f32", (120, 20)) == 2.2e9
    assert bench.pmc_traffic("patchy8192", "f32", (120, 40)) is None    # other tile
    assert bench.pmc_traffic("patchy8192", "f64", (120, 20)) is None    # no summary
    # the kernel source changed since the counters were taken
    _tree(tmp_path, "// kernel v2\n")
    assert bench.kernel_source_hash() != h
    assert bench.pmc_traffic("patchy8192", "f32", (120, 20)) is None


def test_per_tile_summary_takes_precedence(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _tree(tmp_path)
    h = bench.kernel_source_hash()
    _summary(tmp_path, "k_ens_step_ensemble256_f32_120x20_pmc.txt", 3.25e9, "120x20", h)
    _summary(tmp_path, "k_ens_step_ensemble256_f32_120x40_pmc.txt", 3.47e9, "120x40", h)
    get = lambda t: bench.pmc_traffic("ensemble256", "f32", t, kernel="k_ens_step")
    assert get((120, 20)) == 3.25e9
    assert get((120, 40)) == 3.47e9
    assert get((60, 20)) is None
    # a per-tile file whose recorded tile disagrees with its name is refused
    _summary(tmp_path, "k_ens_step_ensemble256_f32_60x20_pmc.txt", 1.0e9, "120x20", h)
    assert get((60, 20)) is None


def test_untiled_summary_for_the_coupling_input(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _tree(tmp_path)
    csrc = tmp_path / "paper_1102_1343_amd" / "csrc"
    (csrc / "fire_wind.hip").write_text("// wind\n")
    files = ("fire_wind.hip", "fire_internal.h")
    h = bench.kernel_source_hash(files)
    _summary(tmp_path, "k_wind_wind8192_f32_pmc.txt", 6.4e8, "none", h)
    assert bench.pmc_traffic("wind8192", "f32", None, kernel="k_wind", files=files) == 6.4e8
    # the step kernel's hash is not the coupling input's
    assert bench.pmc_traffic("wind8192", "f32", None, kernel="k_wind") is None


def test_committed_summaries_name_their_commands():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    prof = os.path.join(root, "profiles")
    names = sorted(os.listdir(prof))
    assert any(n.startswith("k_step_patchy8192") for n in names)
    for n in names:
        txt = open(os.path.join(prof, n)).read()
        assert "rocprofv3" in txt and "bench.py" in txt, n
        if n.endswith("_pmc.txt"):
            assert "kernel_source_sha256_16:" in txt and "hbm_bytes_per_launch:" in txt, n


def test_more_than_one_gpu_is_refused():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_cpu_baseline_reports_one_thread_and_the_host():
    """The oracle's host rate comes with its one-thread rate and the host's
    processor, on a small patchy window (a few seconds of CPU)."""
    import oracle
    from paper_1102_1343_amd import synth

    prob = synth.patchy_fire(256, steps=4)
    before = oracle.threads()
    r = bench.cpu_baseline(prob, "f64", 0.2)
    assert oracle.threads() == before
    assert r["kind"] == "oracle" and r["cores"] == before
    st = r["single_thread"]
    assert st["cores"] == 1 and st["value"] > 0 and st["threads_speedup_same_steps"] > 0
    assert r["host"]["cpus_available"] >= 1 and isinstance(r["host"]["model"], str)
