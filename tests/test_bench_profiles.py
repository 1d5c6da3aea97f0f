"""The profiled figures bench.py reports (ops per site update, measured HBM
bytes) belong to the kernels as built from specific sources. bench.py keys
each recorded profile by a hash of those sources and reports the figure only
while the tree still hashes to it; otherwise the figure is null. These tests
check that rule, and that the profile summaries the figures come from are in
profiles/."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _batched_result():
    return {"value": 2000.0, "ms": 1000.0, "sweeps": 100, "attempts": 2.0e12}


def test_batched_roofline_only_for_profiled_sources(monkeypatch):
    for stepped, key in ((False, "PROFILED_BATCH_SOURCES"), (True, "PROFILED_MULTI_FUSED_SOURCES")):
        files = bench.MULTI_FUSED_FILES if stepped else bench.BATCH_FILES
        monkeypatch.setattr(bench, key, bench.kernel_sources_hash(files))
        assert bench.batched_roofline(_batched_result(), stepped) is not None
        monkeypatch.setattr(bench, key, "0" * 16)
        assert bench.batched_roofline(_batched_result(), stepped) is None


def test_headline_profile_only_for_profiled_sources(monkeypatch):
    kname = sorted(bench.PROFILED)[0]
    monkeypatch.setattr(bench, "PROFILED_SOURCES", bench.kernel_sources_hash())
    assert bench.headline_profile(kname) is not None
    monkeypatch.setattr(bench, "PROFILED_SOURCES", "0" * 16)
    assert bench.headline_profile(kname) is None


def test_profile_summaries_exist():
    for name in ("k_fused_rows_ising2d_32768.md", "k_fused_ising2d_32768.md", "k_fused_ising2d_4096.md",
                 "k_creutz_fused_creutz_32768.md", "k_batch_bits_batched_1024.md", "k_multi_fused_batched_1024.md",
                 "k_multi_fused_served_stream.md", "k_vec_micro.md", "k_perc_relax_percolation_32768.md",
                 "k_bands_ising2d_4096.md"):
        assert os.path.isfile(os.path.join(ROOT, "profiles", name)), name


def test_recorded_profiles_belong_to_the_committed_kernels():
    # every figure bench.py prices was taken on the kernels as they are now:
    # a kernel source change without a new profile fails here
    assert bench.kernel_sources_hash() == bench.PROFILED_SOURCES
    assert bench.kernel_sources_hash(bench.CREUTZ_FILES) == bench.PROFILED_CREUTZ_SOURCES
    assert bench.kernel_sources_hash(bench.BATCH_FILES) == bench.PROFILED_BATCH_SOURCES
    assert bench.kernel_sources_hash(bench.MULTI_FUSED_FILES) == bench.PROFILED_MULTI_FUSED_SOURCES
