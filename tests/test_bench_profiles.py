"""The profiled figures bench.py reports (ops per site update, measured HBM
bytes) belong to the kernels as built from specific sources: each recorded
source hash must match the sources in the tree, or the bench line would
silently fall back to unprofiled roofs. A kernel change therefore needs a
new profile (profiles/) or, when the profiled kernel still compiles to the
same instructions, the recorded hash moved forward."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_headline_profile_matches_sources():
    assert bench.kernel_sources_hash() == bench.PROFILED_SOURCES


def test_creutz_profile_matches_sources():
    assert bench.kernel_sources_hash(bench.CREUTZ_FILES) == bench.PROFILED_CREUTZ_SOURCES


def test_batched_profiles_match_sources():
    assert bench.kernel_sources_hash(bench.BATCH_FILES) == bench.PROFILED_BATCH_SOURCES
    assert bench.kernel_sources_hash(bench.MULTI_FUSED_FILES) == bench.PROFILED_MULTI_FUSED_SOURCES


def test_profile_summaries_exist():
    for name in ("k_fused_ising2d_32768.md", "k_creutz_fused_creutz_32768.md", "k_batch_bits_batched_1024.md",
                 "k_multi_fused_batched_1024.md"):
        assert os.path.isfile(os.path.join(ROOT, "profiles", name)), name
