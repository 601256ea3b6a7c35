"""Planted mistakes in the oracle are caught by its pins (CPU only).

Each case loads a fresh copy of the oracle's source with one plausible
mistake written in (a dropped term, a flipped sign, a wrong index, a
transposed operand), then runs the pins named for it and requires that at
least one of them fails.  The real oracle is never modified.
"""

import importlib
import itertools
import os
import sys
import types
from fractions import Fraction

import pytest

import pins
from paper_2011_05698_amd.signals import SignalSpec, make_signal

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sfft_oracle.py")
_COUNTER = itertools.count()


def mutated_oracle(old: str, new: str) -> types.ModuleType:
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not unique: {old!r}"
    name = f"sfft_oracle_mutant_{next(_COUNTER)}"
    mod = types.ModuleType(name)
    mod.__file__ = SRC
    sys.modules[name] = mod          # dataclasses resolve annotations through sys.modules
    exec(compile(text.replace(old, new), SRC + " (mutant)", "exec"), mod.__dict__)
    return mod


def _sig(N, K, seed):
    return make_signal(SignalSpec(N, K, seed))


E2E = [(2 ** 14, 50, 512, 7169, 8, 16, Fraction(1), 1e-8, 101, 102),
       (2 ** 12, 10, 128, 1537, 6, 4, Fraction(1, 4), 1e-8, 7, 8)]

CHECKS = {
    "p1": pins.check_p1_permutation,
    "p2": pins.check_p2_subsampling,
    "p3": pins.check_p3_lemma1_single_tone,
    "p4": pins.check_p4_window,
    "p5": pins.check_p5_subtraction,
    "p6": pins.check_p6_bucket_fft,
    "p7": lambda O: pins.check_p7_location(O, us=range(0, 4096, 3)),
    "p8": pins.check_p8_estimate,
    "p9": lambda O: pins.check_p9_end_to_end(O, E2E, _sig),
    "sched": pins.check_schedule,
    "rng": pins.check_splitmix64,
    "p11": pins.check_p11_detect,
    "p12": lambda O: pins.check_p12_direct_location(O, us=range(0, 4096, 5)),
    "p13": lambda O: pins.check_p13_vote(O, _sig),
    "p14": pins.check_p14_verify,
    "p15": pins.check_p15_home_bucket,
    "p16": pins.check_p16_eta_floor,
}

MUTANTS = [
    # gather: offset applied with the wrong sign (Eq. 7)
    ("idx = (sigma * (t - T)) % N", "idx = (sigma * (t + T)) % N", ["p1", "p3"]),
    # gather: sigma applied after the shift instead of before
    ("idx = (sigma * (t - T)) % N", "idx = (sigma * t - T) % N", ["p1", "p3"]),
    # bucket DFT normalised by 1/B (Eq. 1) instead of 1/N
    ("return np.fft.fft(y) / N", "return np.fft.fft(y) / B", ["p1", "p2"]),
    # fold index transposed to the sample index
    ("    b = t % B\n", "    b = idx % B\n", ["p2", "p6"]),
    # window: boxcar frequency doubled
    ("np.sin(math.pi * lt / N)", "np.sin(2 * math.pi * lt / N)", ["p4"]),
    # window: centre tap wrong
    ("G[0] = float(L)", "G[0] = float(L) + 1.0", ["p4"]),
    # window: Gaussian too wide (drops the factor 2 in the width rule)
    ("s_t = h / math.sqrt(2.0 * math.log(1.0 / delta))", "s_t = h / math.sqrt(math.log(1.0 / delta))", ["p4"]),
    # window spectrum: negative-time half not mirrored
    ("g[N - h:] = G_half[1:][::-1]", "g[N - h:] = G_half[1:]", ["p4", "p3"]),
    # transition half-width: erfc^-1 argument off by 2
    ("erfcinv(2.0 * delta)", "erfcinv(delta / 2.0)", ["p4"]),
    # subtraction: phase sign flipped
    ("out[j, i % B] -= v * np.exp(-1j * TWO_PI * p / N) * g",
     "out[j, i % B] -= v * np.exp(1j * TWO_PI * p / N) * g", ["p5"]),
    # subtraction: window spectrum index off by one
    ("g = it.Ghat[abs(i * L - u)]", "g = it.Ghat[max(abs(i * L - u) - 1, 0)]", ["p5"]),
    # subtraction: reach limited to the home bucket
    ("        for i in bucket_range(u, L, it.D):\n            g = it.Ghat",
     "        for i in bucket_range(u, L, L // 2 - 1):\n            g = it.Ghat", ["p5"]),
    # phase difference conjugated on the wrong operand (Eq. 16 sign)
    ("z = yhat[0, i] * np.conj(yhat[j, i])", "z = np.conj(yhat[0, i]) * yhat[j, i]", ["p7"]),
    # block location: extension applied in the wrong direction
    ("a = a + ((2 * best_b * qd - qn) * ln) // (2 * qd * l)",
     "a = a + ((2 * best_b * qd + qn) * ln) // (2 * qd * l)", ["p7"]),
    # block location: block start used instead of block centre
    ("num = ((2 * l * a + (2 * b + 1) * ln) * tau) % M2", "num = ((2 * l * a + (2 * b) * ln) * tau) % M2", ["p7"]),
    # first region not extended by the transition half-width
    ("a = i * L - L // 2 - e\n", "a = i * L - L // 2\n", ["p7"]),
    # schedule: region multiplier too large (phases wrap)
    ("        tau = N // ln\n", "        tau = 2 * (N // ln)\n", ["p7", "sched"]),
    # schedule: region shrinks by l/q instead of l/(1+q)
    ("nxt = math.ceil((1 + q) * ln / l) + 1", "nxt = math.ceil(q * ln / l) + 1", ["p7", "sched"]),
    # estimate: phase correction with the wrong sign (Eq. 14)
    ("yhat[j, i] * np.exp(1j * TWO_PI * ((it.T[j] * u) % N) / N) / g",
     "yhat[j, i] * np.exp(-1j * TWO_PI * ((it.T[j] * u) % N) / N) / g", ["p8"]),
    # estimate: window spectrum not divided out
    ("((it.T[j] * u) % N) / N) / g", "((it.T[j] * u) % N) / N)", ["p8"]),
    # frequency from position with sigma instead of sigma^-1
    ("f = (it.sigma_inv * u) % N", "f = (it.sigma * u) % N", ["p9"]),
    # accumulation overwrites instead of adding (Sec. 3.1 step 5)
    ("rec[f] = rec.get(f, 0j) + v", "rec[f] = v", ["p9"]),
    # detection: round-to-round magnitude test dropped (collisions pass)
    ("return (p0 >= thr) & (p0 > 0) & consistent", "return (p0 >= thr) & (p0 > 0)", ["p11", "p9"]),
    # round offsets: reference round shifted like the others
    ("T = [tau0] + [(tau0 + taus[j]) % N for j in range(1, R + 1)]",
     "T = [tau0] + [(taus[j]) % N for j in range(1, R + 1)]", ["p9"]),
    # RNG: wrong mixing constant
    ("0xBF58476D1CE4E5B9", "0xBF58476D1CE4E5B8", ["rng"]),
    # direct location: truncation instead of rounding
    ("return math.floor(theta[1] * N / TWO_PI + 0.5) % N", "return math.floor(theta[1] * N / TWO_PI) % N", ["p12"]),
    # direct location: the offset of the second round
    ("lens, taus, kinds = [0, Lm + 2 * e], [0, 1], [BLK, DIRECT]",
     "lens, taus, kinds = [0, Lm + 2 * e], [0, 2], [BLK, DIRECT]", ["p12"]),
    # vote: a strict majority instead of at least half of the loops
    ("if 2 * len(vs) >= loops:", "if 2 * len(vs) > loops:", ["p13"]),
    # vote: mean over the loops instead of the median
    ("out[f] = complex(np.median(a.real), np.median(a.imag))",
     "out[f] = complex(np.mean(a.real), np.mean(a.imag))", ["p13"]),
    # vote: loops also subtract what earlier loops located
    ("ysub = yhat if vote else subtract(yhat, rec, it, N)",
     "ysub = subtract(yhat, {f: vs[0] for f, vs in votes.items()} if vote else rec, it, N)", ["p13"]),
    # vote: B halves per loop as in the iterative method
    ('Bm = B if combine == "vote" else max(B >> (m - 1), b_min)', "Bm = max(B >> (m - 1), b_min)", ["p13"]),
    # verify: the per-round phase test (Eq. 18 bound) dropped
    ("        if circ_dist(theta[j], TWO_PI * ((it.taus[j] * u) % N) / N) > math.pi / l:\n            return False\n",
     "        pass\n", ["p14", "p7"]),
    # verify: tolerance of a whole block (2 pi / l) instead of half a block
    ("((it.taus[j] * u) % N) / N) > math.pi / l:", "((it.taus[j] * u) % N) / N) > 2 * math.pi / l:", ["p14"]),
    # verify: tolerance a quarter block
    ("((it.taus[j] * u) % N) / N) > math.pi / l:", "((it.taus[j] * u) % N) / N) > 0.5 * math.pi / l:", ["p14"]),
    # verify: the home-bucket check dropped (any bucket that locates u keeps it)
    ("    if home_bucket(u, it.L, it.B) != i:\n        return False\n", "", ["p14", "p15", "p7"]),
    # verify: accepted wherever the window reaches (L/2 + e) instead of the home range
    ("    if home_bucket(u, it.L, it.B) != i:\n        return False\n",
     "    if min(abs(i * it.L - u), N - abs(i * it.L - u)) > it.D:\n        return False\n", ["p14", "p15", "p7"]),
    # home bucket: halves rounded down instead of up
    ("return ((u + L // 2) // L) % B", "return ((u + L // 2 - 1) // L) % B", ["p14", "p7"]),
    # home bucket: the floor of u / L (no rounding to the nearest centre)
    ("return ((u + L // 2) // L) % B", "return (u // L) % B", ["p14", "p7"]),
    # detection: the relative floor eta dropped
    ("thr = max(2.0 * math.log(B) * nu, eta * eta * float(p0.max()))", "thr = 2.0 * math.log(B) * nu", ["p16"]),
    # detection: the noise threshold dropped (only the relative floor left)
    ("thr = max(2.0 * math.log(B) * nu, eta * eta * float(p0.max()))", "thr = eta * eta * float(p0.max())", ["p16"]),
    # detection: the noise threshold without the union bound over B buckets
    ("thr = max(2.0 * math.log(B) * nu, eta * eta * float(p0.max()))",
     "thr = max(2.0 * nu, eta * eta * float(p0.max()))", ["p16"]),
    # detection: the floor applied to magnitudes instead of powers
    ("thr = max(2.0 * math.log(B) * nu, eta * eta * float(p0.max()))",
     "thr = max(2.0 * math.log(B) * nu, eta * float(p0.max()))", ["p16", "p9"]),
]


@pytest.mark.parametrize("old,new,checks", MUTANTS, ids=[f"m{i:02d}" for i in range(len(MUTANTS))])
def test_planted_mistake_is_caught(old, new, checks):
    O = mutated_oracle(old, new)
    caught = []
    for name in checks:
        try:
            CHECKS[name](O)
        except AssertionError as exc:
            caught.append((name, str(exc)[:80]))
    assert caught, f"no pin caught the mutation {old!r} -> {new!r}"


def test_unmutated_oracle_passes_the_same_checks():
    O = importlib.import_module("oracle.sfft_oracle")
    for name in ("p1", "p2", "p5", "p6", "p8", "sched", "rng", "p14", "p15", "p16"):
        CHECKS[name](O)
