"""Host-side parts of bench.py that need no GPU: the multi-GPU refusal, the
step bound of the coalescence timing case and the kernel-source hash that
guards the committed HBM traffic figures."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_coalescence_timing_is_bounded():
    with pytest.raises(ValueError):
        bench.coalescence_bench(149, 2)


def test_paper_coalescence_throughput_is_derived_from_its_table():
    # 120^3 cells x 8 steps / wall time
    for lat, s in bench.PAPER_COALESCENCE_S.items():
        assert abs(120 ** 3 * 8 / s / 1e6 - {15: 0.7238, 19: 0.7089, 27: 0.7018}[lat]) < 1e-3


def test_traffic_entries_are_guarded_by_the_kernel_hash():
    h = bench.csrc_hash()
    assert len(h) == 16
    # an entry is used only while its hash matches the kernel sources
    assert bench.measured_traffic("no_such_kernel", "fp32") is None


def test_committed_traffic_belongs_to_the_current_kernels():
    """profiles/traffic.json holds rocprofv3 FETCH_SIZE + WRITE_SIZE bytes for
    every kernel of the 3-D step in both precisions, measured on the kernel
    sources as they are now, and each figure lies near that kernel's
    algorithmic bytes at 256^3 (each field read once and written once)."""
    import json

    data = json.load(open(bench.TRAFFIC_FILE))
    fields = {"flow_stage1": 9, "flow_stage2": 13, "flow_stage3": 16,
              "ch_rk4_stage1": 6, "ch_rk4_stage2": 8, "ch_rk4_stage3": 8, "ch_rk4_stage4": 7}
    for prec, esize in (("fp32", 4), ("fp64", 8)):
        for k, nf in fields.items():
            ent = data[f"{k}:{prec}"]
            assert ent["csrc_hash"] == bench.csrc_hash(), k
            got = bench.measured_traffic(k, prec)
            assert got == ent["bytes_per_launch"] == ent["fetch_bytes"] + ent["write_bytes"]
            ratio = got / (nf * 256 ** 3 * esize)
            assert 0.95 < ratio < 1.5, (k, prec, ratio)
