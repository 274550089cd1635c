"""Random words of the binary16 stores, checked on the host.

Each node rounds its 19 new binary16 values stochastically with 13 random
bits apiece, taken from ten 32-bit words (plane 2j: the top 13 bits of word
j; plane 2j + 1: those of word j shifted left by 16).  The words come from
the node's hashed seed s (s = 0 replaced by 0x9E3779B9): four xorshift32
steps (Marsaglia 2003, shifts 13, 17, 5) give W1..W4, and the words are

    W1, W3, W4, W1^W2, W1^W3, W1^W4, W3^W4, W1^W2^W4, W1^W3^W4, W2.

Checked here:
* the library's host form (lks::F16Words, built from
  paper_2112_13930_amd/csrc/lks_sr.hpp by tests/native/f16words.cpp) gives
  the words of this statement, bit for bit;
* every pair of the 19 fields is jointly uniform over the seed: as maps over
  GF(2) of the 32 seed bits their stacked 26 x 32 matrix has full rank, so
  the rounding errors of a node's values are pairwise independent;
* the rank check has teeth: two plausible variants (pairs of the four words
  only; a seed with its low bit forced to one) fail it.
"""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = os.environ.get("LKS_HOST_CLANG", "/opt/rocm/llvm/bin/clang++")


def _xorshift32(s):
    s = s ^ ((s << np.uint32(13)) & np.uint32(0xFFFFFFFF))
    s = s ^ (s >> np.uint32(17))
    s = s ^ ((s << np.uint32(5)) & np.uint32(0xFFFFFFFF))
    return s


def words_statement(seeds):
    """The 19 words (as passed to the rounding) per seed, from the definition."""
    s = np.asarray(seeds, dtype=np.uint32).copy()
    s[s == 0] = np.uint32(0x9E3779B9)
    w1 = _xorshift32(s)
    w2 = _xorshift32(w1)
    w3 = _xorshift32(w2)
    w4 = _xorshift32(w3)
    ten = [w1, w3, w4, w1 ^ w2, w1 ^ w3, w1 ^ w4, w3 ^ w4, w1 ^ w2 ^ w4, w1 ^ w3 ^ w4, w2]
    out = []
    for q in range(19):
        w = ten[q // 2]
        out.append(w if q % 2 == 0 else (w << np.uint32(16)) & np.uint32(0xFFFFFFFF))
    return np.stack(out, axis=1)


@pytest.mark.skipif(not (os.path.exists(CLANG) or shutil.which(CLANG)), reason="no clang++ for the host build")
def test_host_words_match_statement(tmp_path):
    exe = str(tmp_path / "f16words")
    subprocess.run([CLANG, "-std=c++17", "-O2", "-I", os.path.join(ROOT, "paper_2112_13930_amd", "csrc"),
                    "-o", exe, os.path.join(ROOT, "tests", "native", "f16words.cpp")], check=True)
    for first, count in ((0, 4096), (0xFFFFF000, 4096), (0x9E3779B0, 32)):
        r = subprocess.run([exe, str(first), str(count)], capture_output=True, text=True, timeout=60, check=True)
        got = np.array([[int(t, 16) for t in line.split()] for line in r.stdout.splitlines()], dtype=np.uint64)
        seeds = (np.arange(count, dtype=np.uint64) + first) & 0xFFFFFFFF
        want = words_statement(seeds.astype(np.uint32)).astype(np.uint64)
        assert got.shape == (count, 19)
        np.testing.assert_array_equal(got, want)


# ---- pairwise joint uniformity over GF(2) ----

def _shift_matrix(k, left):
    m = np.zeros((32, 32), dtype=np.uint8)  # bit i of the result (row) from bit j (column)
    for j in range(32):
        i = j + k if left else j - k
        if 0 <= i < 32:
            m[i, j] = 1
    return m


def _xorshift_matrix():
    eye = np.eye(32, dtype=np.uint8)
    a = (eye + _shift_matrix(13, True)) % 2
    b = (eye + _shift_matrix(17, False)) % 2
    c = (eye + _shift_matrix(5, True)) % 2
    return (c @ b @ a) % 2


def _rank2(m):
    m = m.copy() % 2
    r = 0
    for c in range(m.shape[1]):
        rows = np.nonzero(m[r:, c])[0]
        if rows.size == 0:
            continue
        p = r + rows[0]
        m[[r, p]] = m[[p, r]]
        hit = np.nonzero(m[:, c])[0]
        for i in hit:
            if i != r:
                m[i] ^= m[r]
        r += 1
        if r == m.shape[0]:
            break
    return r


def _field_maps(ten, seed_cols=slice(0, 32)):
    """13 x n maps of the 19 fields (rows: the field's bits, high to low)."""
    maps = []
    for q in range(19):
        w = ten[q // 2]
        rows = w[19:32] if q % 2 == 0 else w[3:16]  # bits 31..19 or, shifted by 16, bits 15..3
        maps.append(rows[:, seed_cols])
    return maps


def _deficient_pairs(maps):
    return [(a, b) for a, b in itertools.combinations(range(len(maps)), 2)
            if _rank2(np.vstack([maps[a], maps[b]])) < 26]


def _base_words():
    m = _xorshift_matrix()
    w = [m]
    for _ in range(3):
        w.append((m @ w[-1]) % 2)
    return w


def test_fields_pairwise_jointly_uniform():
    w1, w2, w3, w4 = _base_words()
    x = lambda *ms: sum(ms) % 2
    ten = [w1, w3, w4, x(w1, w2), x(w1, w3), x(w1, w4), x(w3, w4), x(w1, w2, w4), x(w1, w3, w4), w2]
    maps = _field_maps(ten)
    assert all(_rank2(f) == 13 for f in maps)
    assert _deficient_pairs(maps) == []


def test_rank_check_catches_weaker_schemes():
    w1, w2, w3, w4 = _base_words()
    x = lambda *ms: sum(ms) % 2
    # the four words and their six pairs only
    pairs = [w1, w2, w3, w4, x(w1, w2), x(w1, w3), x(w1, w4), x(w2, w3), x(w2, w4), x(w3, w4)]
    assert _deficient_pairs(_field_maps(pairs))
    # the chosen words from a seed whose low bit is forced to one (31 free bits)
    ten = [w1, w3, w4, x(w1, w2), x(w1, w3), x(w1, w4), x(w3, w4), x(w1, w2, w4), x(w1, w3, w4), w2]
    assert _deficient_pairs(_field_maps(ten, seed_cols=slice(1, 32)))


def test_fields_empirically_uniform():
    rng = np.random.default_rng(7)
    seeds = rng.integers(0, 2**32, size=1 << 16, dtype=np.uint64).astype(np.uint32)
    fields = words_statement(seeds) >> np.uint32(19)  # the 13 bits the rounding takes
    # each field's top 4 bits: 16 bins of 4096 expected; a pair's joint top
    # 3 bits: 64 bins of 1024 expected (binomial sd about 62 and 31)
    for q in range(19):
        h = np.bincount(fields[:, q] >> np.uint32(9), minlength=16)
        assert np.all(np.abs(h - 4096) < 400), (q, h)
    for a, b in itertools.combinations(range(19), 2):
        h = np.bincount((fields[:, a] >> np.uint32(10)) * 8 + (fields[:, b] >> np.uint32(10)), minlength=64)
        assert np.all(np.abs(h - 1024) < 200), (a, b)
