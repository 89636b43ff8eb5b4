import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Print the session's parity totals (exact l, cost ties, order ties,
    flagged end-to-end cases) so that they appear in the tail of the log."""
    try:
        from tests.vp_parity import TOTALS
    except Exception:   # pragma: no cover - the helper failed to import
        return
    if not TOTALS:
        return
    terminalreporter.write_sep("-", "parity totals")
    for kind in sorted(TOTALS):
        items = " ".join(f"{k}={v:.2e}" if isinstance(v, float) else f"{k}={v}" for k, v in TOTALS[kind].items())
        terminalreporter.write_line(f"parity[{kind}] {items}")
