"""The FP64 oracle against the pins of the paper (CPU only)."""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle.sfft_oracle as O
import pins
from paper_2011_05698_amd.signals import SignalSpec, make_signal


def _signal(N, K, seed):
    x, sup, vals = make_signal(SignalSpec(N, K, seed))
    return x, sup, vals


def test_p1_permutation():
    pins.check_p1_permutation(O)


def test_p2_subsampling():
    pins.check_p2_subsampling(O)


def test_p3_lemma1_single_tone():
    pins.check_p3_lemma1_single_tone(O)


def test_p4_window():
    pins.check_p4_window(O)


def test_p5_subtraction():
    pins.check_p5_subtraction(O)


def test_p6_bucket_fft():
    pins.check_p6_bucket_fft(O)


def test_p7_location_exhaustive():
    pins.check_p7_location(O)


@pytest.mark.parametrize("l,q", [(2, Fraction(1, 2)), (2, Fraction(1, 4)), (2, Fraction(1, 8)),
                                 (4, Fraction(1, 2)), (4, Fraction(1, 8)), (16, Fraction(1, 2)),
                                 (16, Fraction(1, 4)), (16, Fraction(1, 8)), (8, Fraction(3, 2))])
def test_p7_location_mapped_pairs(l, q):
    pins.check_p7_location(O, lq=((l, q),), us=range(0, 4096, 7))


def test_p8_estimate():
    pins.check_p8_estimate(O)
    pins.check_p8b_median_rule(O)


CASES = [
    # N, K, B, w, M, l, q, delta, signal seed, plan seed
    (2 ** 14, 50, 512, 7169, 8, 16, Fraction(1), 1e-8, 101, 102),
    (2 ** 14, 50, 512, 7169, 8, 4, Fraction(1, 4), 1e-8, 101, 102),
    (2 ** 12, 10, 128, 1537, 6, 16, Fraction(1), 1e-8, 7, 8),
    (2 ** 16, 200, 512, 8193, 10, 16, Fraction(1), 1e-6, 9, 10),
]


def test_p9_end_to_end():
    pins.check_p9_end_to_end(O, CASES, _signal)


def test_p9_bruteforce_dft_support():
    """At small N a brute-force DFT followed by top-K gives the planted
    support, and the oracle returns the same support."""
    N, K = 2048, 12
    x, sup, vals = _signal(N, K, 31)
    xhat = pins.brute_dft(x)
    order = sorted(range(N), key=lambda f: (-abs(xhat[f]), f))[:K]
    assert sorted(order) == sorted(sup.tolist())
    P = O.make_plan(N, K, 128, (128 * 11) | 1, 6, 16, 1, 1e-8, seed=32)
    idx, val, _ = O.sfft(x, P)
    assert idx.tolist() == sorted(order)
    assert np.max(np.abs(val - xhat[idx])) < 1e-6


def test_p11_detect():
    pins.check_p11_detect(O)


def test_p10_samples():
    pins.check_p10_samples(O)


def test_schedule_rules():
    pins.check_schedule(O)


def test_splitmix64_vector():
    pins.check_splitmix64(O)


def test_degenerate_inputs():
    """Zero signal gives no coefficient; a single tone gives exactly it."""
    N, B = 4096, 64
    P = O.make_plan(N, 1, B, (B * 12) | 1, 4, 16, 1, 1e-8, seed=4)
    idx, val, _ = O.sfft(np.zeros(N, dtype=complex), P)
    assert idx.size == 0 and val.size == 0
    x = (0.3 - 0.4j) * np.exp(2j * np.pi * 1234 * np.arange(N) / N)
    idx, val, _ = O.sfft(x, P)
    assert idx.tolist() == [1234] and abs(val[0] - (0.3 - 0.4j)) < 1e-9


def test_top_k_ties_and_order():
    """Output rule (Sec. 2.1 goal): K largest by magnitude, ties to the
    smaller index, exact zeros dropped, returned sorted by index."""
    N, K = 4096, 3
    x = np.zeros(N, dtype=complex)
    n = np.arange(N)
    for f, v in [(100, 1.0), (50, 1.0), (3000, 1.0), (7, 0.5)]:
        x += v * np.exp(2j * np.pi * f * n / N)
    P = O.make_plan(N, K, 64, (64 * 12) | 1, 6, 16, 1, 1e-8, seed=12)
    idx, val, _ = O.sfft(x, P)
    assert idx.tolist() == [50, 100, 3000]


def test_p12_direct_location_exhaustive():
    pins.check_p12_direct_location(O)


def test_p12_direct_end_to_end():
    cases = [(2 ** 14, 50, 512, 7169, 8, 16, Fraction(1), 1e-8, 121, 122),
             (2 ** 16, 300, 2048, 32769, 10, 16, Fraction(1), 1e-6, 123, 124)]
    pins.check_p9_end_to_end(O, cases, _signal, location="direct")


def test_p13_vote():
    pins.check_p13_vote(O, _signal)


def test_p14_verify_bound_and_home_range():
    pins.check_p14_verify(O)


def test_p15_home_bucket_only():
    pins.check_p15_home_bucket(O)


def test_p16_detection_floor():
    pins.check_p16_eta_floor(O)
