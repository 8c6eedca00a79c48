"""Host-side checks of the benchmark's contract: one GPU only, and the
counter summaries that feed the roofline's traffic and MFMA fields were
taken on the kernel sources in this tree (otherwise the benchmark reports
them as null, and the summaries must be re-taken with the commands they
list)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

WORKLOADS = ("cfg1", "cfg2", "batch64", "serve", "bands", "density_matrix", "modes", "integration")


@pytest.mark.parametrize("workload", WORKLOADS)
def test_more_than_one_gpu_is_refused(workload):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--workload", workload,
                        "--no-cpu-baseline"], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2, (r.returncode, r.stderr[-400:])
    assert "one GPU only" in r.stderr
    assert not r.stdout.strip()                 # no JSON line for a run that did not happen


def test_counter_summaries_match_the_kernel_sources():
    sha = bench.kernel_source_sha1()
    for path in (bench.TRAFFIC_FILE, bench.TRAFFIC_FILE_DM, bench.MFMA_FILE):
        txt = open(path).read()
        assert f"kernel_source_sha1: {sha}" in txt, f"{os.path.basename(path)} was taken on other kernel sources"
    t = bench.measured_traffic()
    tdm = bench.measured_traffic(bench.TRAFFIC_FILE_DM)
    mf = bench.measured_mfma()
    assert t is not None and tdm is not None and mf is not None
    # algorithmic bytes per launch (N = 200, m = 64, 2048 energies): X_i and
    # z_i written and read once, 4 N m^2 16 B per energy; the measured HBM
    # bytes can only exceed that, and the summaries explain a factor near 3
    alg = 2048 * 4 * 200 * 64 ** 2 * 16
    assert 1.0 <= t / alg <= 4.0
    alg_dm = alg + 2048 * 2 * (2 * 200 - 1) * 64 ** 2 * 16
    assert 1.0 <= tdm / alg_dm <= 4.0
    # executed FP64 MFMA flops per sweep launch: at least the algorithmic
    # count N (152/3) m^3 per energy, and a utilisation in (0, 100] percent
    assert mf["mfma_flops_executed_per_launch"] >= 2048 * 200 * (152.0 / 3.0) * 64 ** 3
    assert 0.0 < mf["mfma_util_pct"] <= 100.0


def test_flop_count_of_the_whole_solve():
    # (N + n_dec) (152/3) m^3: the slabs of the sweep plus the decimation
    # doublings, each priced like one slab
    assert bench.flops_per_energy(200, 64, 0.0) == pytest.approx(200 * (152.0 / 3.0) * 64 ** 3)
    assert bench.flops_per_energy(200, 64, 22.0) == pytest.approx(222 * (152.0 / 3.0) * 64 ** 3)
