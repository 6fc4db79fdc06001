"""Shared test setup: the `gpu` marker, import paths and the oracle build."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build(force=False)
    yield


def pytest_sessionfinish(session, exitstatus):
    """With RAMPPI_PARITY_SUMMARY=<path>, write the report of every full-step
    comparison with the oracle that ran in this session as a markdown table."""
    path = os.environ.get("RAMPPI_PARITY_SUMMARY")
    helpers = sys.modules.get("parity_helpers")
    if path and helpers is not None and (helpers.REPORTS or helpers.GRAD_REPORTS):
        helpers.write_reports(path)
