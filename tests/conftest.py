import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    if not (ROOT / "oracle" / "liboracle.so").exists():
        oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def synth_lib():
    import synth
    if not (ROOT / "synth" / "libsynth.so").exists():
        synth.build(force=False)
    return synth
