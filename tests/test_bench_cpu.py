"""Host-side checks of bench.py's reporting: the kernel names it gives each
pipeline shape, and the committed HBM-traffic summaries it reads (they parse,
carry a figure for every shape, and are tied to the kernel sources by hash)."""
import os

import pytest

import bench
import paper_2010_16114_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_names_cover_every_shape():
    for v in range(P.MFMA_VARIANTS):
        xk, _ = bench.mfma_kernel_names(v, 0)
        assert xk.startswith("mfma_xtr_split_kernel" if v < 8 else "mfma_xtr_lds_kernel")
        assert ("xtr_tail_kernel" in xk) == (v >= 15)
    for v in range(P.ETA_VARIANTS):
        _, ek = bench.mfma_kernel_names(0, v)
        assert ek.startswith("mfma_eta_kernel" if v < 2 else "mfma_eta_split_kernel")
        assert ("eta_fixup_kernel" in ek) == (v >= 8)


@pytest.mark.parametrize("summary,keys", [
    ("mfma_xtr_kernel_geno_fp8_400000x500000_b64_traffic.md",
     [("launch", f"shape{v}") for v in range(P.MFMA_VARIANTS)]
     + [("column", f"eta_shape{v}") for v in range(P.ETA_VARIANTS)]),
    ("mfma_eta_kernel_dense_geno_fp8_400000x500000_b64_traffic.md",
     [("launch", f"shape{v}") for v in range(P.ETA_VARIANTS)]),
])
def test_traffic_summaries(summary, keys):
    path = os.path.join(ROOT, "profiles", summary)
    text = open(path).read()
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
    stored = [line.split(":", 1)[1].strip() for line in text.splitlines() if line.startswith("- source_sha256:")]
    assert len(stored) == 1 and len(stored[0]) == 64
    current = bench.kernel_source_hash(bench.MFMA_SOURCES)
    for per, shape in keys:
        v = bench.stored_traffic(summary, bench.MFMA_SOURCES, shape, per=per)
        if stored[0] == current:
            assert v is not None and v > 0, (per, shape)
        else:  # the kernels changed since the counters were taken: no figure is reported
            assert v is None
    assert bench.stored_traffic(summary, bench.MFMA_SOURCES, "shape99") is None
    assert bench.stored_traffic("no_such_summary.md", bench.MFMA_SOURCES, "shape0") is None


def test_column_sum_traffic_summary():
    summary = "gemvt_sums_kernel_gauss_fp32_20000x50000_traffic.md"
    text = open(os.path.join(ROOT, "profiles", summary)).read()
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
    for src in bench.GEMVT_SOURCES:  # every file the kernel is built from is named under the hash
        assert src in text
    stored = [line.split(":", 1)[1].strip() for line in text.splitlines() if line.startswith("- source_sha256:")]
    assert len(stored) == 1
    v = bench.stored_traffic(summary, bench.GEMVT_SOURCES)
    if stored[0] == bench.kernel_source_hash(bench.GEMVT_SOURCES):
        # within 1% of X once (20,000 x 50,000 FP32) plus the vectors
        assert v is not None and abs(v / 4.0005e9 - 1) < 0.01
    else:
        assert v is None
