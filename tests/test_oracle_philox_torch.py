"""Pin of the oracle's Philox4x32-10 words against a third, independent implementation:
PyTorch's header-only CPU engine (ATen/core/PhiloxRNGEngine.h), compiled on the host.

The oracle's generator (Salmon et al., SC'11) is written from the published definition;
a swapped output word, a misplaced key bump or a wrong multiplier would change the words
and fail here, while passing every statistical test of test_oracle_rng.py."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("PyTorch's Philox header is not installed")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_torch_check")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", inc,
                           os.path.join(HERE, "philox_torch_check.cpp"), "-o", exe])

    def run(rows):
        text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64).astype(np.uint32)
    return run


def _cases():
    rng = np.random.default_rng(20230704)
    rows = [
        (0, 0, 0, 0, 0, 0),
        (0xFFFFFFFF,) * 6,
        (1, 2, 3, 4, 5, 6),
        # the stream layouts the method uses: push (id, step, PUSH), cell streams
        # (cell, block, step, KMC), creation (cell, slot, step, CREATE)
        (12345, 1 << 29, 199, 1 << 24, 1, 0),
        (5 + 64 * (6 + 64 * 7), 3, 17, 3 << 24, 1, 0),
        (70000, 63, 4000, 4 << 24, 1, 255),
    ]
    rows += [tuple(int(v) for v in rng.integers(0, 2**32, size=6, dtype=np.uint64)) for _ in range(200)]
    return rows


def test_philox_words_match_torch_engine(orc, torch_philox):
    rows = _cases()
    ref = torch_philox(rows)
    assert ref.shape == (len(rows), 4)
    for r, want in zip(rows, ref):
        got = orc.philox(np.array(r[:4], dtype=np.uint32), np.array(r[4:], dtype=np.uint32))
        assert np.array_equal(got, want), (r, got, want)


def test_philox_words_change_with_every_input(orc, torch_philox):
    # each counter and key word reaches the output (guards a comparison that would
    # pass if both sides ignored an input word)
    base = (11, 22, 33, 44, 55, 66)
    rows = [base]
    for i in range(6):
        r = list(base)
        r[i] ^= 1
        rows.append(tuple(r))
    ref = torch_philox(rows)
    for i in range(1, 7):
        assert not np.array_equal(ref[0], ref[i])
        got = orc.philox(np.array(rows[i][:4], dtype=np.uint32), np.array(rows[i][4:], dtype=np.uint32))
        assert np.array_equal(got, ref[i])
