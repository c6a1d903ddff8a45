import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle run")


def _paper_values():
    import json

    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.json")) as fh:
        return {k: v["value"] for k, v in json.load(fh).items() if isinstance(v, dict)}


# Numbers the paper reports (tests/golden/paper_values.json, each cited there).
PAPER = _paper_values()
