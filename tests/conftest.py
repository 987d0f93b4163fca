import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_terminal_summary(terminalreporter):
    """Report every gradient parity check of the session: elements checked and
    plain-rule (1e-3 relative, 1e-6 absolute) violations per test and parameter.
    With GS_GRAD_REPORT set, the records are also written there as JSON."""
    mod = sys.modules.get("tests.gpu_util")
    recs = getattr(mod, "RECORDS", None) if mod is not None else None
    if not recs:
        return
    tr = terminalreporter
    tr.write_sep("-", "gradient parity (plain rule |g-ref| <= 1e-3|ref| + 1e-6)")
    tot = sum(r["checked"] for r in recs)
    bad = sum(r["plain_violations"] for r in recs)
    for r in recs:
        tr.write_line(f"{r['test']:<80.80} {r['param']:<15} {r['checked']:>9} "
                      f"{r['plain_violations']:>5}  worst {r['worst_plain']:.3f}")
    tr.write_line(f"total: {tot} elements checked, {bad} plain-rule violations")
    path = os.environ.get("GS_GRAD_REPORT")
    if path:
        import json
        with open(path, "w") as f:
            json.dump(recs, f, indent=1)
