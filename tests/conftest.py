import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "first_run_tuning: keeps the library's tuning on a plan's first run")


@pytest.fixture(autouse=True)
def _rule_variants_unless_tuning_is_tested(request, monkeypatch):
    """Runs take the rule's kernel variant unless a test is about first-run
    tuning: a tuned variant chosen by timing could differ between two runs that
    a test compares bit for bit (a grouped launch against its single launches,
    a dynamic call against its static plan). Explicit autotuner calls still
    tune; the process-wide table starts empty in every GPU test."""
    if request.node.get_closest_marker("first_run_tuning") is None and "SPMM_AUTOTUNE" not in os.environ:
        monkeypatch.setenv("SPMM_AUTOTUNE", "0")
    if request.node.get_closest_marker("gpu") is not None:  # no tuned variant carries over from another test
        from paper_2303_16999_amd import spmm
        spmm.autotune_clear()
