"""Pins for the oracle's Philox4x32-10 (oracle/philox.py).

The generator is fixed by its published definition (Salmon et al., SC'11);
the pin is rocRAND's independent implementation, compiled and run on the
host, on random and edge-case counters and keys.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32_10, key_from_seed

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host pin")
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    src = os.path.join(HERE, "pins", "rocrand_philox_kat.cpp")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include",
                    src, "-o", exe], check=True, capture_output=True)

    def run(rows):
        text = "".join(" ".join(f"{int(v):x}" for v in row) + "\n" for row in rows)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(x, 16) for x in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64)
    return run


def test_philox_matches_rocrand(rocrand_kat):
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 2**32, size=(400, 6), dtype=np.uint64)
    rows[:, 1] &= np.uint64(2**30 - 1)  # rocRAND's offset argument covers c1 < 2^30
    edge = np.array([
        [0, 0, 0, 0, 0, 0],
        [0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF],
        [1, 0, 0, 0, 0, 0],
        [0, 1, 0, 0, 0, 0],
        [0, 0, 1, 0, 0, 0],
        [0, 0, 0, 1, 0, 0],
        [0, 0, 0, 0, 1, 0],
        [0, 0, 0, 0, 0, 1],
        [12345, 678, 0, 0, 1503, 0],
    ], dtype=np.uint64)
    rows = np.vstack([edge, rows])
    want = rocrand_kat(rows)
    got = np.stack(philox4x32_10(rows[:, 0], rows[:, 1], rows[:, 2], rows[:, 3],
                                 rows[:, 4], rows[:, 5]), axis=1).astype(np.uint64)
    assert np.array_equal(got, want)


def test_key_from_seed_split():
    assert key_from_seed(0x0123456789ABCDEF) == (0x89ABCDEF, 0x01234567)
    assert key_from_seed(5) == (5, 0)


def test_philox_avalanche_and_balance():
    # flipping one counter bit flips about half of the 128 output bits
    n = 2000
    rng = np.random.default_rng(3)
    c = rng.integers(0, 2**32, size=(4, n), dtype=np.uint64)
    base = np.stack(philox4x32_10(*c, 99, 7))
    c2 = c.copy()
    c2[0] ^= np.uint64(1)
    flip = np.stack(philox4x32_10(*c2, 99, 7))
    diff = np.bitwise_xor(base, flip)
    bits = sum(int(np.unpackbits(diff[i].view(np.uint8)).sum()) for i in range(4))
    frac = bits / (128.0 * n)
    assert 0.48 < frac < 0.52
    ones = sum(int(np.unpackbits(base[i].view(np.uint8)).sum()) for i in range(4))
    assert abs(ones / (128.0 * n) - 0.5) < 0.01
