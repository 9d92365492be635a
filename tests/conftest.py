import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


_capman = None


def pytest_configure(config):
    global _capman
    _capman = config.pluginmanager.getplugin("capturemanager")
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long CPU run (oracle physics pins)")


def progress(msg: str) -> None:
    """Write msg to stderr at once, past pytest's output capture, so that a
    long test (full-horizon oracle references take minutes) shows progress
    while it runs."""
    if _capman is None:
        print(msg, file=sys.stderr, flush=True)
        return
    with _capman.global_and_fixture_disabled():
        sys.stderr.write(msg + "\n")
        sys.stderr.flush()
