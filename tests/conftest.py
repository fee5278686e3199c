"""Shared pytest configuration.

``gpu`` marks tests that need an MI355X (the HIP library and a visible
device); everything else runs on the CPU.
"""

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU oracle work of more than a few seconds")


def pytest_collection_modifyitems(config, items):
    """GPU tests are skipped where no HIP device is visible (the CPU container)."""
    if not any("gpu" in item.keywords for item in items):
        return
    try:
        import torch

        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no HIP device visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def pytest_runtest_logstart(nodeid, location):
    """Name each test on stderr before it runs, so a run that dies mid-test says which."""
    sys.stderr.write(f"\n[start] {nodeid}\n")
    sys.stderr.flush()
