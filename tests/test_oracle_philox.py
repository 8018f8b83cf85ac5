"""Pin the oracle's Philox4x32-10 against two independent implementations
and the published known-answer vectors.

The oracle writes Philox from its published definition (Salmon et al.,
SC'11). Here it must agree, word for word, with PyTorch's ATen
``philox_engine`` and with rocRAND's ``philox4x32_10_engine``, both compiled
from their source headers, on a million random (counter, key) pairs plus
edge counters, and it must give the generator's published known-answer
vectors. A wrong multiplier, a swapped output word, a missing key bump
or a wrong round count fails this.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xcheck", "philox_xcheck.cpp")


def _torch_include():
    import torch
    return os.path.join(os.path.dirname(torch.__file__), "include")


def _build(tmp_path, which):
    exe = str(tmp_path / f"xcheck_{which}")
    if which == "torch":
        cmd = ["g++", "-O2", "-std=c++17", "-DUSE_TORCH", "-I", _torch_include(), SRC, "-o", exe]
    else:
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        if not os.path.exists(hipcc):
            pytest.skip("hipcc not available for the rocRAND header")
        cmd = [hipcc, "-O2", "-std=c++17", "-DUSE_ROCRAND", SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def _cases(n, seed, max_ctr1=None):
    rng = np.random.default_rng(seed)
    ctr = rng.integers(0, 1 << 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 1 << 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    if max_ctr1 is not None:
        ctr[:, 1] %= max_ctr1
    # edge counters and keys
    edge = np.array([[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0, 0, 1, 0],
                     [0, 2, 7, 0], [5, 0, 0xFFFFFFFF, 0]], dtype=np.uint32)
    if max_ctr1 is not None:
        edge[:, 1] %= max_ctr1
    ekey = np.array([[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [1, 0], [0, 1], [0x9E3779B9, 0], [3, 5]],
                    dtype=np.uint32)
    return np.concatenate([edge, ctr]), np.concatenate([ekey, key])


def _run(tmp_path, exe, ctr, key):
    rec = np.concatenate([ctr, key], axis=1).astype(np.uint32)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    rec.tofile(fin)
    subprocess.run([exe, str(fin), str(fout)], check=True)
    return np.fromfile(fout, dtype=np.uint32).reshape(-1, 4)


def test_philox_matches_aten_engine(tmp_path):
    exe = _build(tmp_path, "torch")
    ctr, key = _cases(1_000_000, seed=11)
    ref = _run(tmp_path, exe, ctr, key)
    got = oracle.philox4x32_10(ctr, key)
    assert np.array_equal(got, ref)


def test_philox_matches_rocrand_engine(tmp_path):
    exe = _build(tmp_path, "rocrand")
    # rocRAND takes its offset in 32-bit outputs (4 per block): keep the
    # 64-bit offset * 4 from overflowing.
    ctr, key = _cases(1_000_000, seed=12, max_ctr1=1 << 29)
    ref = _run(tmp_path, exe, ctr, key)
    got = oracle.philox4x32_10(ctr, key)
    assert np.array_equal(got, ref)


def test_philox_is_a_bijection_on_a_sample():
    # Philox with a fixed key is a permutation of 128-bit blocks: distinct
    # counters give distinct outputs.
    n = 1 << 16
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 2] = np.arange(n, dtype=np.uint32)
    key = np.tile(np.array([[123, 456]], dtype=np.uint32), (n, 1))
    out = oracle.philox4x32_10(ctr, key)
    packed = out.view(np.dtype([("a", np.uint32), ("b", np.uint32), ("c", np.uint32),
                                ("d", np.uint32)])).ravel()
    assert np.unique(packed).shape[0] == n


def test_philox_output_words_are_uniform():
    # Each output bit of sequential counters is a fair coin (chi-square on
    # the byte histogram of a million words).
    n = 1 << 18
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 2] = np.arange(n, dtype=np.uint32)
    key = np.zeros((n, 2), dtype=np.uint32)
    out = oracle.philox4x32_10(ctr, key).ravel()
    hist = np.bincount((out & 0xFF).astype(np.int64), minlength=256)
    expected = out.shape[0] / 256
    chi2 = ((hist - expected) ** 2 / expected).sum()
    assert chi2 < 350.0  # 255 dof: p(chi2 > 350) < 1e-4
    bits = np.unpackbits(out.view(np.uint8)).reshape(-1, 32).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.005)


def test_philox_known_answer_vectors():
    """The published known-answer vectors of Philox4x32-10 (Salmon et al.,
    SC'11), stored under ``tests/golden/``: all-zero, all-ones and the
    digits-of-pi counter and key."""
    path = os.path.join(HERE, "golden", "philox4x32_10_kat.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    v = np.array([[int(w, 16) for w in r] for r in rows], dtype=np.uint64).astype(np.uint32)
    out = oracle.philox4x32_10(np.ascontiguousarray(v[:, 0:4]), np.ascontiguousarray(v[:, 4:6]))
    np.testing.assert_array_equal(out, v[:, 6:10])
