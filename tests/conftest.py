import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU-side runs")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import loops
    loops.build(force=False)
    return loops


def pytest_terminal_summary(terminalreporter):
    """Prints the parity errors that the GPU checks recorded: per field (the
    asserted bar) and each component's own relative L2 error against the
    fp64 oracle."""
    try:
        import gpu_util
    except ImportError:
        return
    if not gpu_util.REPORT:
        return
    tr = terminalreporter
    tr.section("parity errors per component (relative L2 vs the fp64 oracle)")
    for r in gpu_util.REPORT:
        comp = " ".join(f"{k if isinstance(k, str) else '/'.join(map(str, k))}={v:.2e}" for k, v in r["comp"].items())
        over = [k for k, v in r["comp"].items() if v >= gpu_util.TOL[r["prec"]]]
        flag = ("  above the bar on its own: " + ",".join(str(k) for k in over)) if over else ""
        now = r.get("field_now")
        rel = (f" (to the run's peak norm; to the current norm E={now['E']:.2e} H={now['H']:.2e})"
               if now else "")
        tr.write_line(f"{r['check']} [{r['prec']}] E={r['field']['E']:.2e} H={r['field']['H']:.2e}{rel} | {comp}{flag}")
