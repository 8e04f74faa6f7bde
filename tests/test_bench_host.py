"""Host logic of the benchmark's roofline line (CPU): the profiling keys map
to the kernel names the profiler prints, and the committed HBM-traffic
summaries are used only for their own kernel and while the kernel's source
still hashes to the digest they record."""
import re

import pytest

import bench
from paper_1605_01522_amd import nfield


@pytest.mark.parametrize("prof,name", [
    (dict(lanes=16, rows=4, mode="sgs", fp32=False), "k_sgs_color<16, 4, 1, double>"),
    (dict(lanes=16, rows=3, mode="sgs_bsr", fp32=False), "k_sgs_color_bsr<3, 16, double>"),
    (dict(lanes=16, rows=2, mode="sgs_bsr", fp32=True), "k_sgs_color_bsr<2, 16, float>"),
    (dict(lanes=16, rows=3, mode="resid", fp32=False), "k_spmv_bsr<3, 16, 1, double>"),
    (dict(lanes=64, rows=0, mode="store", fp32=False), "k_spmv<64, 0, double>"),
    (dict(lanes=64, rows=4, mode="sgs_node", fp32=False), "k_sgs_node<64, 4, 1, double>"),
])
def test_kernel_names(prof, name):
    assert nfield.kernel_name(prof) == name


@pytest.mark.parametrize("workload", sorted(bench.TRAFFIC_PROFILES))
def test_traffic_summary_is_tied_to_kernel_and_source(workload, monkeypatch):
    path, _ = bench.TRAFFIC_PROFILES[workload]
    text = open(path).read()
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("kernel: ", "source_sha256_16: ", "traffic_bytes_per_launch: ")))
    assert set(fields) == {"kernel", "source_sha256_16", "traffic_bytes_per_launch"}
    assert re.fullmatch(r"[0-9a-f]{16}", fields["source_sha256_16"])
    kernel, digest = fields["kernel"], fields["source_sha256_16"]
    # every segment the digest covers is present in the source
    assert re.fullmatch(r"[0-9a-f]{16}", bench.kernel_source_digest(workload))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda w: digest)
    assert bench.measured_traffic(workload, kernel) == float(fields["traffic_bytes_per_launch"])
    assert bench.measured_traffic(workload, kernel + " ") is None        # another kernel
    assert bench.measured_traffic("tsi2d", kernel) is None              # no summary for it
    monkeypatch.setattr(bench, "kernel_source_digest", lambda w: "0" * 16)
    assert bench.measured_traffic(workload, kernel) is None             # the source changed since
