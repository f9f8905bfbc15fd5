"""Pins for the oracle's random numbers (Philox4x32-10) and bin indices.

Philox4x32-10 is fixed by its published definition (Salmon, Moraes, Dror,
Shaw, SC'11).  The oracle's rounds are compared with an independent
open-source implementation, PyTorch's header-only ATen/core/PhiloxRNGEngine.h,
compiled as a test-only reference (the torch_philox fixture of conftest.py).
"""
import numpy as np
import pytest

import oracle as O

def test_philox_matches_independent_implementation(torch_philox):
    rng = np.random.default_rng(7)
    triples = []
    for _ in range(300):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        ev = int(rng.integers(0, 2**63))
        it = int(rng.integers(0, 2**32))
        blk = int(rng.integers(0, 2**32))
        triples.append((seed, ev, it | (blk << 32)))
    triples += [(0, 0, 0), (2**64 - 1, 2**64 - 1, 2**64 - 1), (0, 99_999, 4 | (1 << 32))]
    ref = torch_philox(triples)
    for (seed, ev, sub), r in zip(triples, ref):
        ctr = [ev & 0xFFFFFFFF, ev >> 32, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert O.philox4x32_10(ctr, key) == r


def test_event_stream_layout(torch_philox):
    """Event e, iteration j, block b uses counter (e_lo, e_hi, j, b) and key = seed;
    the word pairs (r0, r1), (r2, r3) give k = ((hi << 32) | lo) >> 11."""
    cases = [(0, 0, 0), (0, 1, 3), (4, 123456789012, 9), (2**40 + 3, 7, 1)]
    for seed, ev, it in cases:
        for D in (4, 7, 10):
            k = O.event_k53(seed, it, ev, D)
            blocks = [(seed, ev, it | (b << 32)) for b in range((D + 1) // 2)]
            words = torch_philox(blocks)
            expect = []
            for w in words:
                expect.append(((w[0] << 32) | w[1]) >> 11)
                expect.append(((w[2] << 32) | w[3]) >> 11)
            assert [int(v) for v in k] == expect[:D]


def test_uniform_and_bin_are_exact_integer_identities():
    rng = np.random.default_rng(3)
    ks = [0, 1, 2**53 - 1, 2**52] + [int(v) for v in rng.integers(0, 2**53, 2000)]
    for nb in (2, 7, 50, 64, 1000, 1024):
        for k in ks:
            b, delta = O.bin_from_k53(k, nb)
            # floor(y * nb) with y = k / 2^53, in exact integer arithmetic
            assert b == (k * nb) // 2**53
            assert 0 <= b < nb
            assert delta == float((k * nb) % 2**53) / 2**53
            assert 0.0 <= delta < 1.0


def test_uniforms_are_uniform():
    ks = np.array([O.event_k53(0, 0, e, 4) for e in range(4000)], dtype=np.float64)
    y = ks * 2.0**-53
    assert y.min() >= 0.0 and y.max() < 1.0
    # mean 1/2 with standard error 1/sqrt(12 n); 5 sigma
    assert abs(y.mean() - 0.5) < 5 * (1 / np.sqrt(12 * y.size))
    assert abs(np.corrcoef(y[:, 0], y[:, 1])[0, 1]) < 5 / np.sqrt(len(y))
