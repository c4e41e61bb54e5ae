"""Pin the oracle's Philox4x32-10 against rocRAND's independent implementation.

rocRAND's philox4x32_10 engine (open-source header, evaluated on the host)
is a second implementation of Salmon et al. (SC 2011); agreement on random
and edge-case counters/keys pins the oracle's rounds, multipliers and key
schedule.
"""
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

HELPER_SRC = Path(__file__).parent / "helpers" / "philox_rocrand.cpp"
HELPER_BIN = Path(__file__).parent / "helpers" / "philox_rocrand.bin"


def _helper():
    if HELPER_BIN.exists() and HELPER_BIN.stat().st_mtime >= HELPER_SRC.stat().st_mtime:
        return HELPER_BIN
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(hipcc).exists():
        pytest.skip("hipcc not available to build the rocRAND reference")
    subprocess.run([hipcc, "-O1", str(HELPER_SRC), "-o", str(HELPER_BIN)], check=True)
    return HELPER_BIN


def test_philox_matches_rocrand(oracle_lib):
    rng = np.random.default_rng(1234)
    cases = [
        ([0, 0, 0, 0], [0, 0]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF, 0xFFFFFFFF]),
        ([1, 0, 0, 0], [0, 0]),
        ([0, 0, 0, 1], [1, 0]),
        ([7, 0, 123, 2], [0xDEADBEEF, 0x12345678]),
    ]
    for _ in range(200):
        cases.append((rng.integers(0, 2**32, 4, dtype=np.uint64).tolist(),
                      rng.integers(0, 2**32, 2, dtype=np.uint64).tolist()))
    text = "".join(" ".join(str(int(x)) for x in c + k) + "\n" for c, k in cases)
    out = subprocess.run([str(_helper())], input=text, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for (c, k), r in zip(cases, ref):
        got = oracle_lib.philox(c, k).tolist()
        assert got == r, (c, k, got, r)


def test_derived_keys_distinct(oracle_lib):
    keys = {oracle_lib.derived_key(0, i) for i in range(1, 200)}
    assert len(keys) == 199
    assert oracle_lib.derived_key(5, 1) != oracle_lib.derived_key(6, 1)
