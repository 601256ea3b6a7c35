"""Pins that tie the FP64 oracle to the paper and to plain mathematics.

Every check takes the oracle module as an argument, so the mutation tests can
run the same checks against a deliberately broken copy and show that each
planted mistake is caught.  The checks use brute-force definitions (an
explicit O(N^2) DFT matrix, direct cosine sums, closed forms, exhaustive
enumeration), never the oracle's own library calls.
"""

from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
from scipy.special import erf, erfc

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------- helpers --
def dft_matrix(N: int) -> np.ndarray:
    """F_N[j, k] = omega^{jk} / N with omega = exp(-2 pi i / N) (Eq. 1)."""
    j = np.arange(N)
    return np.exp(-2j * np.pi * np.outer(j, j) / N) / N


def brute_dft(x: np.ndarray) -> np.ndarray:
    """xhat = F_N x (Eq. 2) by an explicit matrix-vector product."""
    return dft_matrix(x.shape[0]) @ x


def brute_window_spectrum(N: int, G_half: np.ndarray) -> np.ndarray:
    """Ghat_k for every k in [0, N) by the direct cosine sum of the even,
    real window: (1/N) (G_0 + 2 sum_{t=1..h} G_t cos(2 pi k t / N))."""
    h = len(G_half) - 1
    k = np.arange(N)[:, None]
    t = np.arange(1, h + 1)[None, :]
    return (G_half[0] + 2.0 * (G_half[1:][None, :] * np.cos(TWO_PI * ((k * t) % N) / N)).sum(axis=1)) / N


def rng(seed):
    return np.random.default_rng(seed)


def random_signal(N, seed):
    r = rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


def full_flat_window(N: int) -> np.ndarray:
    """G = 1 on every residue mod N, written as taps |t| <= N/2 where the two
    taps at +-N/2 (the same residue) carry 1/2 each."""
    G = np.ones(N // 2 + 1)
    G[-1] = 0.5
    return G


# ------------------------------------------------------------------ pins --
def check_p1_permutation(O, N=64, seeds=range(3)):
    """P1 (Eq. 7-8): with a window that is 1 everywhere and B = N,
    HashToBins is the DFT of the permuted signal, and
    DFT(x_{sigma(. - tau)})_i = xhat_{sigma^-1 i} omega^{tau i}."""
    G = full_flat_window(N)
    for s in seeds:
        x = random_signal(N, 100 + s)
        xhat = brute_dft(x)
        r = rng(200 + s)
        sigma = int(2 * r.integers(0, N // 2) + 1)
        tau = int(r.integers(0, N))
        sinv = pow(sigma, -1, N)
        got = O.hash_to_bins(x, sigma, tau, G, N)
        i = np.arange(N)
        want = xhat[(sinv * i) % N] * np.exp(-2j * np.pi * ((tau * i) % N) / N)
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        assert err < 1e-13, f"P1 permutation identity off by {err:.3g}"


def check_p2_subsampling(O, N=128, Bs=(4, 8, 32), seeds=range(2)):
    """P2 (Eq. 11-12 with the 1/N reading): with a window that is 1
    everywhere, yhat[i] = xhat'[iL], the permuted spectrum subsampled by L."""
    G = full_flat_window(N)
    for B in Bs:
        L = N // B
        for s in seeds:
            x = random_signal(N, 300 + s)
            r = rng(400 + s)
            sigma = int(2 * r.integers(0, N // 2) + 1)
            tau = int(r.integers(0, N))
            xp = x[(sigma * (np.arange(N) - tau)) % N]
            want = brute_dft(xp)[np.arange(B) * L]
            got = O.hash_to_bins(x, sigma, tau, G, B)
            err = np.max(np.abs(got - want)) / np.max(np.abs(want))
            assert err < 1e-13, f"P2 subsampling identity (B={B}) off by {err:.3g}"


def check_p3_lemma1_single_tone(O, N=1024, B=32, w=None, delta=1e-8, seeds=range(4)):
    """P3 (Lemma 1, Eq. 13-14, exact form): a single coefficient v at f gives,
    in every bucket i and every round j, yhat_j[i] = v omega^{T_j u}
    Ghat_{(iL-u) mod N} with u = sigma f mod N; and HashToBins is linear."""
    if w is None:
        w = (B * int(math.log2(N))) | 1
    P = O.make_plan(N, 1, B, w, 1, 16, 1, delta, seed=7)
    it = P.iters[0]
    Gfull = brute_window_spectrum(N, it.G)
    L = N // B
    total = np.zeros((it.R + 1, B), dtype=complex)
    xsum = np.zeros(N, dtype=complex)
    for s in seeds:
        r = rng(500 + s)
        f = int(r.integers(0, N))
        v = complex(r.standard_normal(), r.standard_normal())
        x = v * np.exp(2j * np.pi * f * np.arange(N) / N)
        xsum += x
        u = (it.sigma * f) % N
        i = np.arange(B)
        for j in range(it.R + 1):
            got = O.hash_to_bins(x, it.sigma, it.T[j], it.G, B)
            want = v * np.exp(-2j * np.pi * ((it.T[j] * u) % N) / N) * Gfull[(i * L - u) % N]
            total[j] += want
            err = np.max(np.abs(got - want)) / abs(v)
            assert err < 1e-13, f"P3 single tone (round {j}) off by {err:.3g}"
    for j in range(it.R + 1):
        got = O.hash_to_bins(xsum, it.sigma, it.T[j], it.G, B)
        err = np.max(np.abs(got - total[j])) / np.max(np.abs(total[j]))
        assert err < 1e-12, f"P3 superposition off by {err:.3g}"


def check_p4_window(O, cases=((1024, 32, 1e-8), (4096, 64, 1e-6), (2048, 16, 1e-10))):
    """P4 (Sec. 2.3, Eq. 9): (a) G_t / gaussian_t is the inverse DFT of the
    half-edge boxcar; (b) the tabulated Ghat equals the direct cosine sum;
    (c) Ghat follows the erf closed form of a boxcar convolved with a
    Gaussian to within the truncation bound delta / (pi ln(1/delta));
    (d) leakage |Ghat_k| <= delta past L/2 + d_delta; (e) flatness
    |1 - Ghat_k| <= delta inside L/2 - d_delta, when that band exists."""
    for N, B, delta in cases:
        L = N // B
        w = (B * int(math.log2(N))) | 1
        G, info = O.flat_window(N, B, w, delta)
        h, s_t, s_f, d = info["h"], info["s_t"], info["s_f"], info["d_delta"]
        assert info["e"] == math.ceil(d) and h == (w - 1) // 2
        # d_delta is where the one-sided Gaussian tail of the transition
        # falls to delta: erfc(d / (sqrt(2) s_f)) / 2 = delta.
        assert abs(0.5 * erfc(d / (math.sqrt(2) * s_f)) / delta - 1) < 1e-9, "P4 transition width"
        assert abs(s_f * 2 * math.pi * s_t / N - 1) < 1e-14
        assert abs(math.exp(-h * h / (2 * s_t * s_t)) / delta - 1) < 1e-12, "P4 Gaussian not at delta at h"
        # (a) boxcar inverse DFT, Eq. 2 normalisation: H_t = sum_k Hhat_k e^{+2 pi i k t / N}
        k = np.arange(N)
        kk = np.minimum(k, N - k)
        Hhat = np.where(kk < L // 2, 1.0, np.where(kk == L // 2, 0.5, 0.0))
        H = (np.exp(2j * np.pi * np.outer(np.arange(h + 1), k) / N) @ Hhat).real
        gauss = np.exp(-np.arange(h + 1) ** 2 / (2 * s_t * s_t))
        err = np.max(np.abs(G - H * gauss)) / L
        assert err < 1e-12, f"P4a window formula off by {err:.3g}"
        # (b) table against the direct cosine sum
        Gfull = brute_window_spectrum(N, G)
        kmax = L // 2 + info["e"]
        tab = O.window_spectrum(N, G, kmax)
        assert tab.shape == (kmax + 1,)
        err = np.max(np.abs(tab - Gfull[:kmax + 1]))
        assert err < 1e-13, f"P4b Ghat table off by {err:.3g}"
        # (c) closed form.  By Poisson summation the DFT of the sampled,
        # untruncated Gaussian is the unit-mass Gaussian density phi of width
        # s_f sampled at the integers, so Ghat = (half-edge boxcar) * phi as a
        # discrete convolution, up to the truncation of the time Gaussian at
        # h, which costs at most delta / (pi ln(1/delta)).  The erf form is
        # the continuum limit of that sum; the trapezoid (Euler-Maclaurin)
        # error adds at most 2 max|phi'| / 12 < 0.05 / s_f^2.
        ks = kk.astype(float)
        bound = delta / (math.pi * math.log(1 / delta))
        m = np.arange(-(L // 2), L // 2 + 1)
        c = np.ones(m.size)
        c[0] = c[-1] = 0.5
        phi = lambda z: np.exp(-z * z / (2 * s_f * s_f)) / (math.sqrt(2 * math.pi) * s_f)
        disc = np.array([np.sum(c * (phi(kv - m) + phi(kv - m - N) + phi(kv - m + N))) for kv in ks])
        err = np.max(np.abs(Gfull - disc))
        assert err <= 1.05 * bound + 1e-14, f"P4c boxcar*Gaussian form off by {err:.3g} > {bound:.3g}"
        closed = 0.5 * (erf((L / 2 + ks) / (math.sqrt(2) * s_f)) + erf((L / 2 - ks) / (math.sqrt(2) * s_f)))
        err = np.max(np.abs(Gfull - closed))
        assert err <= bound + 0.05 / s_f ** 2, f"P4c erf form off by {err:.3g}"
        # (d) leakage
        stop = ks >= L / 2 + d
        assert stop.any()
        assert np.max(np.abs(Gfull[stop])) <= delta + 1.05 * bound, "P4d leakage above delta"
        # (e) flatness
        flat = ks <= L / 2 - d
        if flat.any():
            assert np.max(np.abs(1 - Gfull[flat])) <= delta + 1.05 * bound, "P4e passband not flat"


def check_p5_subtraction(O, N=2048, B=64, delta=1e-8, seed=11):
    """P5 (Sec. 3.1 steps 2-3): subtracting recovered coefficients in bucket
    space equals bucketizing the signal with those coefficients removed:
    HashToBins(x - x_rec) = HashToBins(x) - Update(rec), up to the
    coefficients' reach beyond L/2 + e (at most delta each)."""
    w = (B * int(math.log2(N))) | 1
    P = O.make_plan(N, 8, B, w, 1, 16, 1, delta, seed=seed)
    it = P.iters[0]
    r = rng(seed)
    x = random_signal(N, seed + 1)
    fs = r.choice(N, size=6, replace=False)
    vs = r.standard_normal(6) + 1j * r.standard_normal(6)
    rec = {int(f): complex(v) for f, v in zip(fs, vs)}
    n = np.arange(N)
    xrec = sum(v * np.exp(2j * np.pi * f * n / N) for f, v in rec.items())
    yx = np.stack([O.hash_to_bins(x, it.sigma, it.T[j], it.G, B) for j in range(it.R + 1)])
    yd = np.stack([O.hash_to_bins(x - xrec, it.sigma, it.T[j], it.G, B) for j in range(it.R + 1)])
    got = O.subtract(yx, rec, it, N)
    err = np.max(np.abs(got - yd))
    tol = 2 * delta * sum(abs(v) for v in rec.values()) + 1e-12 * np.max(np.abs(yx))
    assert err <= tol, f"P5 subtraction off by {err:.3g} > {tol:.3g}"
    # and the empty update changes nothing
    assert np.array_equal(O.subtract(yx, {}, it, N), yx)


def check_p6_bucket_fft(O, N=256, B=16, seed=5):
    """P6: the B-point transform inside HashToBins against an O(B^2) DFT of
    the folded vector, both built by explicit loops from Eq. 7, 10, 11."""
    r = rng(seed)
    x = random_signal(N, seed)
    h = 40
    G = r.standard_normal(h + 1)
    sigma, T = 77, 19
    y = np.zeros(B, dtype=complex)
    for t in range(-h, h + 1):
        y[t % B] += G[abs(t)] * x[(sigma * (t - T)) % N]
    want = np.array([sum(y[b] * np.exp(-2j * np.pi * i * b / B) for b in range(B)) for i in range(B)]) / N
    got = O.hash_to_bins(x, sigma, T, G, B)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    assert err < 1e-13, f"P6 bucket DFT off by {err:.3g}"


def _single_tone_yhat(it, u, v, N, i):
    """The exact Lemma 1 value of a lone coefficient in bucket i, all rounds."""
    dist = abs(i * it.L - u)
    dist = min(dist, N - dist)
    g = it.Ghat[dist]
    return np.array([v * np.exp(-2j * np.pi * ((it.T[j] * u) % N) / N) * g for j in range(it.R + 1)])


def check_p7_location(O, N=4096, B=64, lq=((16, Fraction(1)), (4, Fraction(1, 4))), us=None,
                      delta=1e-8, seed=3):
    """P7 (Sec. 3.2, Eq. 16): a lone noiseless coefficient is located
    exactly, at every permuted position u (exhaustive by default) and from
    every bucket whose extended region reaches it; verification accepts it
    in the bucket whose range [iL - L/2, iL + L/2) holds u (Lemma 1) and
    nowhere else, and the result does not depend on the offset tau0."""
    w = (B * int(math.log2(N))) | 1
    for l, q in lq:
        P = O.make_plan(N, 1, B, w, 1, l, q, delta, seed=seed)
        it = P.iters[0]
        assert it.kinds[-1] == O.ENUM and all(k == O.BLK for k in it.kinds[1:-1])
        v = complex(0.6, -0.8)
        for u in (range(N) if us is None else us):
            for i_unwrapped in O.bucket_range(u, it.L, it.D):
                i = i_unwrapped % B
                col = _single_tone_yhat(it, u, v, N, i)
                yh = np.zeros((it.R + 1, B), dtype=complex)
                yh[:, i] = col
                th = O.phases(yh, i)
                got = O.locate(th, i, it, N, l, q)
                assert got == u, f"P7 (l={l}, q={q}) u={u} bucket {i}: located {got}"
                # the range of bucket i: iL - L/2 <= u < iL + L/2 (circularly)
                off = (u - i * it.L + it.L // 2) % N
                assert O.verify(th, u, i, it, N, l) == (off < it.L), f"P7 verify of u={u} in bucket {i}"
        # tau0 invariance on a sample of positions
        it2 = O.make_plan(N, 1, B, w, 1, l, q, delta, seed=seed + 1000).iters[0]
        it2 = type(it)(**{**it.__dict__, "tau0": it2.tau0,
                          "T": [(it2.tau0 + it.taus[j]) % N if j else it2.tau0 for j in range(it.R + 1)]})
        for u in range(0, N, 97):
            i = ((u + it.L // 2) // it.L) % B
            yh = np.zeros((it.R + 1, B), dtype=complex)
            yh[:, i] = _single_tone_yhat(it2, u, v, N, i)
            assert O.locate(O.phases(yh, i), i, it2, N, l, q) == u


def check_p12_direct_location(O, N=4096, B=64, delta=1e-8, seed=5, us=None):
    """P12 (the two-round location of sFFT3.0, Eq. 16 with tau = 1): the plan
    has one location step with offsets tau0 and tau0 + 1; a lone noiseless
    coefficient is located exactly at every permuted position u from every
    bucket that reaches it, and verification accepts it.  For phases off the
    grid the located position is the nearest position by brute force over
    all N (checked away from exact halves)."""
    w = (B * int(math.log2(N))) | 1
    P = O.make_plan(N, 1, B, w, 1, 16, 1, delta, seed=seed, location="direct")
    it = P.iters[0]
    assert it.R == 1 and it.taus[1] == 1 and it.kinds[1] == O.DIRECT
    assert it.T[1] == (it.T[0] + 1) % N
    v = complex(-0.28, 0.96)
    for u in (range(N) if us is None else us):
        for i_unwrapped in O.bucket_range(u, it.L, it.D):
            i = i_unwrapped % B
            yh = np.zeros((2, B), dtype=complex)
            yh[:, i] = _single_tone_yhat(it, u, v, N, i)
            th = O.phases(yh, i)
            got = O.locate(th, i, it, N, 16, Fraction(1))
            assert got == u, f"P12 u={u} bucket {i}: located {got}"
            off = (u - i * it.L + it.L // 2) % N
            assert O.verify(th, u, i, it, N, 16) == (off < it.L), f"P12 verify of u={u} in bucket {i}"
    r = rng(seed)
    grid = 2 * math.pi * np.arange(N) / N
    for _ in range(200):
        frac = r.uniform(-0.49, 0.49)
        c = int(r.integers(N))
        theta = (2 * math.pi * (c + frac) / N) % (2 * math.pi)
        d = np.abs(((grid - theta) + math.pi) % (2 * math.pi) - math.pi)
        best = int(np.argmin(d))
        th = [0.0, theta]
        assert O.locate(th, 0, it, N, 16, Fraction(1)) == best == c % N


def check_p8_estimate(O, N=4096, B=64, delta=1e-8, seed=9, n=200):
    """P8 (Eq. 14 with the median over rounds): a lone coefficient's value
    comes back from any bucket that holds it."""
    w = (B * int(math.log2(N))) | 1
    P = O.make_plan(N, 1, B, w, 1, 16, 1, delta, seed=seed)
    it = P.iters[0]
    r = rng(seed)
    for _ in range(n):
        u = int(r.integers(0, N))
        v = complex(r.standard_normal(), r.standard_normal())
        for i_unwrapped in O.bucket_range(u, it.L, it.D):
            i = i_unwrapped % B
            yh = np.zeros((it.R + 1, B), dtype=complex)
            yh[:, i] = _single_tone_yhat(it, u, v, N, i)
            got = O.estimate(yh, i, u, it, N)
            assert abs(got - v) <= 1e-12 * abs(v), f"P8 estimate {got} != {v}"


def check_p8b_median_rule(O):
    """Median of complex values (reading of the 'median estimation'): real
    and imaginary parts separately, mean of the two middle values for an
    even count; an outlier round does not move the estimate."""
    N, B = 1024, 32
    P = O.make_plan(N, 1, B, (B * 10) | 1, 1, 16, 1, 1e-8, seed=1)
    it = P.iters[0]
    u = 5 * it.L + 3
    i = 5
    v = complex(1.0, 2.0)
    yh = np.zeros((it.R + 1, B), dtype=complex)
    yh[:, i] = _single_tone_yhat(it, u, v, N, i)
    if it.R + 1 >= 3:
        yh[1, i] *= 7.0           # one corrupted round
        got = O.estimate(yh, i, u, it, N)
        assert abs(got - v) < 1e-9 * abs(v) or (it.R + 1) % 2 == 0


def check_p13_vote(O, make_signal):
    """P13 (the cross-iteration vote over loops, the one-shot framework of
    Sec. 1 and the opening of Sec. 3).  (a) A vote worked by hand: with 4
    loops, a frequency located by 3 loops keeps the per-part median of its
    3 values, one located by 2 loops the mean of the two middle values, one
    located by 1 loop is dropped.  (b) Every loop of a vote plan has the full
    B buckets and w taps.  (c) An exactly K-sparse planted signal at
    K/B = 1/32 comes back (support equal, values within 10 K delta of the
    truth): with nothing subtracted, a coefficient's estimate in one loop
    carries the leakage of any other coefficient within reach of its bucket,
    which at this sparsity happens in few loops, and the median over the
    loops drops them.  This fails if a loop subtracts what earlier loops
    found, since later loops then see nothing and the vote drops it.  (d) A single loop is the iterative
    method's single iteration: same support, same values."""
    got = O.combine_votes({3: [1 + 1j, 2 + 5j, 3 - 1j], 7: [4j], 9: [1 + 0j, 2 + 2j]}, 4)
    assert set(got) == {3, 9}, f"P13 vote kept {sorted(got)}"
    assert got[3] == 2 + 1j and got[9] == 1.5 + 1j, f"P13 vote values {got}"
    N, K, B, w, M, delta = 2 ** 14, 16, 512, 7169, 8, 1e-8
    P = O.make_plan(N, K, B, w, M, 16, 1, delta, seed=132, combine="vote")
    assert all(it.B == B and it.w == w for it in P.iters), "P13 vote plan must keep B and w"
    x, sup, vals = make_signal(N, K, 131)
    idx, val, _ = O.sfft(x, P)
    assert np.array_equal(idx, np.sort(sup)), f"P13 vote support: {len(idx)} of {K}"
    truth = dict(zip(sup.tolist(), vals))
    err = max(abs(v - truth[f]) for f, v in zip(idx.tolist(), val))
    assert err <= 10 * K * delta, f"P13 vote value error {err:.3g}"
    one_v = O.sfft(x, O.make_plan(N, K, B, w, 1, 16, 1, delta, seed=133, combine="vote"))
    one_s = O.sfft(x, O.make_plan(N, K, B, w, 1, 16, 1, delta, seed=133))
    assert np.array_equal(one_v[0], one_s[0]) and np.array_equal(one_v[1], one_s[1]), "P13 single loop"


def check_p9_end_to_end(O, cases, make_signal, location="multiscale"):
    """P9: an exactly K-sparse planted signal comes back: the support equals
    the planted support and values are within 10 K delta of the truth;
    Parseval N sum |v|^2 = sum |x|^2 holds to 1e-6."""
    for (N, K, B, w, M, l, q, delta, sseed, pseed) in cases:
        x, sup, vals = make_signal(N, K, sseed)
        P = O.make_plan(N, K, B, w, M, l, q, delta, seed=pseed, location=location)
        idx, val, info = O.sfft(x, P)
        assert np.array_equal(idx, np.sort(sup)), f"P9 support mismatch at N={N}, K={K}, (l,q)=({l},{q})"
        truth = dict(zip(sup.tolist(), vals))
        err = max(abs(v - truth[f]) for f, v in zip(idx.tolist(), val))
        assert err <= 10 * K * delta, f"P9 value error {err:.3g}"
        pars = abs(N * np.sum(np.abs(val) ** 2) - np.sum(np.abs(x) ** 2)) / np.sum(np.abs(x) ** 2)
        assert pars < 1e-6, f"P9 Parseval off by {pars:.3g}"


def check_p10_samples(O, N=4096, B=64, M=4):
    """P10 (Sec. 2.4 and Sec. 3.1 cost model): one execute reads
    sum_m (R_m + 1) w_m samples; counted by observing every gather."""
    w = (B * 12) | 1
    P = O.make_plan(N, 4, B, w, M, 16, 1, 1e-8, seed=2)
    count = [0]
    orig = O.hash_to_bins

    def counting(x, sigma, T, G, Bm):
        count[0] += 2 * (len(G) - 1) + 1
        return orig(x, sigma, T, G, Bm)

    O.hash_to_bins = counting
    try:
        x = random_signal(N, 1)
        O.sfft(x, P)
    finally:
        O.hash_to_bins = orig
    want = sum((it.R + 1) * it.w for it in P.iters)
    assert count[0] == want == O.samples_per_signal(P)


def check_schedule(O):
    """Schedule (Sec. 3.2): regions shrink by (1+q)/l per block step, tau_j =
    floor(N/len_j), the last step enumerates at most max(l, ...) positions,
    and the number of steps is about log_{l/(q+1)} of the first length."""
    for (N, L, e, l, q) in [(2 ** 22, 2048, 741, 16, Fraction(1)), (2 ** 14, 32, 25, 4, Fraction(1, 4)),
                            (2 ** 20, 128, 51, 2, Fraction(1, 2)), (2 ** 20, 128, 51, 16, Fraction(1, 8))]:
        lens, taus, kinds = O.location_schedule(N, L, e, l, q)
        assert lens[1] == L + 2 * e
        for j in range(1, len(lens)):
            assert taus[j] == N // lens[j]
            if kinds[j] == O.BLK:
                assert lens[j + 1] == math.ceil((1 + q) * lens[j] / l) + 1
                assert lens[j + 1] < lens[j]
        assert kinds[-1] == O.ENUM
        R = len(lens) - 1
        ideal = math.log(lens[1]) / math.log(l / (1 + q))
        assert R <= ideal + 3, (R, ideal)


def check_splitmix64(O):
    """SplitMix64 published test vector: seed 1234567 gives these outputs."""
    g = O.SplitMix64(1234567)
    got = [g.next() for _ in range(5)]
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert got == want, got


def check_p11_detect(O, N=4096, B=64, delta=1e-8, seed=21):
    """Detection (the build's reading of the isolation assumption of Sec.
    3.2): a bucket with one coefficient is active; a bucket where two
    coefficients collide, so that its magnitude swings from round to round by
    more than rho, is not; empty buckets are not; the rule is invariant to a
    common scale of the input."""
    w = (B * int(math.log2(N))) | 1
    P = O.make_plan(N, 2, B, w, 1, 4, Fraction(1, 4), delta, seed=seed)
    it = P.iters[0]
    assert it.R >= 2
    L = it.L
    yh = np.zeros((it.R + 1, B), dtype=complex)
    lone_i = 5
    yh[:, lone_i] = _single_tone_yhat(it, lone_i * L + 3, complex(0.8, 0.6), N, lone_i)
    # two equal coefficients in bucket 20: pick offsets whose round phases differ
    coll_i = 20
    r = rng(seed)
    for _ in range(1000):
        d1, d2 = (int(v) for v in r.integers(-(L // 4), L // 4, size=2))
        col = (_single_tone_yhat(it, coll_i * L + d1, 1.0, N, coll_i)
               + _single_tone_yhat(it, coll_i * L + d2, 1.0, N, coll_i))
        mag = np.abs(col)
        if np.max(np.abs(mag - mag[0])) > 2 * P.rho * mag[0] and mag[0] > 0.5:
            break
    else:
        raise AssertionError("could not build a colliding bucket")
    yh[:, coll_i] = col
    act = O.detect(yh, B, P.eta, P.rho)
    assert act[lone_i], "P11 lone coefficient not detected"
    assert not act[coll_i], "P11 collision bucket passed the singleton screen"
    assert act.sum() == 1, "P11 empty bucket detected"
    assert np.array_equal(O.detect(yh * 1e-3, B, P.eta, P.rho), act)
    assert not O.detect(np.zeros_like(yh), B, P.eta, P.rho).any()


def _exact_phases(it, u, v, N, i):
    """Round phases of bucket i for a lone noiseless coefficient at u, taken
    from its exact Lemma 1 bucket values (P3's closed form)."""
    yh = np.zeros((it.R + 1, it.B), dtype=complex)
    yh[:, i] = _single_tone_yhat(it, u, v, N, i)
    return [0.0] + [math.atan2((yh[0, i] * np.conj(yh[j, i])).imag, (yh[0, i] * np.conj(yh[j, i])).real)
                    % TWO_PI for j in range(1, it.R + 1)]


def check_p14_verify(O, N=4096, B=64, lq=((16, Fraction(1)), (4, Fraction(1, 4))), delta=1e-8, seed=17):
    """P14 (Eq. 18 bound, Sec. 3.2): a location is trusted only while every
    round's phase error is at most half a block, pi/l, and only in the
    bucket whose range holds the position (Lemma 1: u in [iL - L/2,
    iL + L/2)).  For lone coefficients at many positions, from their home
    bucket, verify accepts the exact phases; it accepts a phase error of
    (1 - 1e-9) pi/l in any one round, of either sign, and rejects
    (1 + 1e-9) pi/l in any one round.  At the edges of the range, with exact
    phases, iL - L/2 and iL + L/2 - 1 are kept and iL + L/2 and
    iL - L/2 - 1 are rejected (they belong to the neighbours)."""
    w = (B * int(math.log2(N))) | 1
    r = rng(seed)
    v = complex(0.6, 0.8)
    for l, q in lq:
        it = O.make_plan(N, 1, B, w, 1, l, q, delta, seed=seed).iters[0]
        tol = math.pi / l
        L = it.L
        for u in r.choice(N, size=40, replace=False).tolist():
            i = ((u + L // 2) // L) % B
            th = _exact_phases(it, u, v, N, i)
            assert O.verify(th, u, i, it, N, l), f"P14 exact phases rejected (u={u}, i={i})"
            for j in range(1, it.R + 1):
                for sgn in (1.0, -1.0):
                    inside = list(th)
                    inside[j] = (th[j] + sgn * tol * (1 - 1e-9)) % TWO_PI
                    assert O.verify(inside, u, i, it, N, l), f"P14 error inside pi/l rejected (l={l}, j={j})"
                    outside = list(th)
                    outside[j] = (th[j] + sgn * tol * (1 + 1e-9)) % TWO_PI
                    assert not O.verify(outside, u, i, it, N, l), \
                        f"P14 error beyond pi/l accepted (l={l}, j={j}, sign {sgn})"
        # the edges of bucket i's range, with the exact phases bucket i sees
        for i in (0, 5, B - 1):
            for off, keep in ((-(L // 2), True), (L // 2 - 1, True), (L // 2, False), (-(L // 2) - 1, False)):
                u = (i * L + off) % N
                ok = O.verify(_exact_phases(it, u, v, N, i), u, i, it, N, l)
                assert ok == keep, f"P14 position {off:+d} from the centre of bucket {i}: verify {ok}"


def check_p15_home_bucket(O, N=4096, B=64, delta=1e-8, seed=19):
    """P15 (one position seen by two buckets; Eq. 14 error propagation): a
    lone coefficient v at u between the centres of buckets i (distance 10)
    and i + 1 (distance L - 10), both within the window's reach, is located
    from both.  Each bucket carries an error c, placed in every round so
    that it shifts every round's Eq. 14 estimate by the same amount
    c / Ghat: the estimate of bucket k is then exactly v + c / Ghat_{d_k}.
    The one candidate must be the home bucket's, within |c| / Ghat_10 (1e-12
    relative), not the other's, which is off by |c| / Ghat_{L-10}, orders of
    magnitude more: a position deep in a bucket's transition band, where
    Ghat falls toward delta, would turn any error of that bucket into a
    huge false coefficient."""
    w = (B * int(math.log2(N))) | 1
    P = O.make_plan(N, 1, B, w, 1, 16, 1, delta, seed=seed)
    it = P.iters[0]
    L = it.L
    v = complex(-0.8, 0.6)
    c = complex(3e-7, -4e-7)
    for i, offset in ((7, 10), (30, L - 10), (B - 1, 10)):
        u = (i * L + offset) % N
        near = i if offset < L // 2 else (i + 1) % B
        far = (i + 1) % B if offset < L // 2 else i
        d_near, d_far = min(offset, L - offset), L - min(offset, L - offset)
        assert d_far <= it.D, "the farther bucket must reach the coefficient"
        g_near, g_far = it.Ghat[d_near], it.Ghat[d_far]
        assert g_far < 0.05 * g_near and g_far > 10 * P.eta
        yh = np.zeros((it.R + 1, B), dtype=complex)
        for k in (near, far):
            yh[:, k] = _single_tone_yhat(it, u, v, N, k)
            # an error that Eq. 14 turns into the same shift c / Ghat in every round
            yh[:, k] += np.array([c * np.exp(-2j * np.pi * ((it.T[j] * u) % N) / N) for j in range(it.R + 1)])
        cands, active, located = O.reconstruct(yh, it, P)
        assert active[near] and active[far], "P15 both buckets must pass detection"
        assert located[near] == u and located[far] == -1, "P15 only the home bucket keeps u"
        f = (it.sigma_inv * u) % N
        assert list(cands) == [f], f"P15 one candidate per position, got {sorted(cands)}"
        want = v + c / g_near
        assert abs(cands[f] - want) <= 1e-12 * abs(v), \
            f"P15 kept the farther bucket's estimate ({abs(cands[f] - v):.3g} from v)"
        assert abs(c / g_far) > 10 * abs(cands[f] - v), "P15 the farther estimate must be far worse"


def check_p16_eta_floor(O, N=4096, B=64, delta=1e-8, seed=23):
    """P16 (the relative detection floor eta of the detection reading): in
    one iteration, a strong lone coefficient (1.0), a weaker one (3e-3) and
    a weak one (3e-5, below eta = 1e-4 of the strongest) sit in separate
    buckets above a noise floor of 1e-9 in every bucket.  The weak bucket
    clears the noise threshold 2 ln(B) median|yhat_0|^2 / ln 2 by far, but
    not the floor (eta max|yhat_0|)^2: the two others are detected, it is
    not.  With eta = 0 it is detected too.  Scaling all values keeps the
    decisions."""
    w = (B * int(math.log2(N))) | 1
    P = O.make_plan(N, 2, B, w, 1, 4, Fraction(1, 4), delta, seed=seed)
    it = P.iters[0]
    L = it.L
    r = rng(seed)
    yh = 1e-9 * (r.standard_normal((it.R + 1, B)) + 1j * r.standard_normal((it.R + 1, B)))
    yh[:, 10] += _single_tone_yhat(it, 10 * L, 1.0 + 0j, N, 10)
    yh[:, 40] += _single_tone_yhat(it, 40 * L + 1, complex(0, 3e-5), N, 40)
    # 3e-3 of the strongest: above the floor (a power ratio of eta^2 = 1e-8)
    yh[:, 25] += _single_tone_yhat(it, 25 * L - 2, complex(-3e-3, 0), N, 25)
    p0 = np.abs(yh[0]) ** 2
    assert p0[40] > 1e3 * 2 * math.log(B) * np.median(p0) / math.log(2), "weak bucket must clear the noise threshold"
    act = O.detect(yh, B, P.eta, P.rho)
    assert act[10] and act[25] and not act[40], f"P16 eta floor: active buckets {np.flatnonzero(act).tolist()}"
    assert act.sum() == 2
    assert np.array_equal(O.detect(yh * 1e4, B, P.eta, P.rho), act)
    no_floor = O.detect(yh, B, 0.0, P.rho)
    assert no_floor[10] and no_floor[25] and no_floor[40], "P16 without the floor all three are lone coefficients"
    # The noise threshold: buckets of pure noise whose magnitude is the same
    # in every round (so the round-to-round test cannot reject them) and
    # whose power is exponentially distributed with mean mu.  The median
    # power is mu ln 2, so nu = mu and the threshold 2 ln(B) mu is exceeded
    # with probability exp(-2 ln B) = 1/B^2 per bucket: across B buckets a
    # noise bucket passes with probability 1/B.  All of them sit far above
    # the eta floor of the strongest bucket, a lone coefficient of 1.0.
    for B2 in (64, 256):
        it2 = O.make_plan(N, 2, B2, (B2 * int(math.log2(N))) | 1, 1, 4, Fraction(1, 4), delta, seed=seed).iters[0]
        mag = np.sqrt(r.exponential(2e-6, size=B2))
        ph = r.uniform(0, TWO_PI, size=(it2.R + 1, B2))
        yn = mag[None, :] * np.exp(1j * ph)
        yn[:, 3] = _single_tone_yhat(it2, 3 * it2.L, 1.0 + 0j, N, 3)
        act = O.detect(yn, B2, P.eta, P.rho)
        assert act[3] and act.sum() == 1, f"P16 noise buckets detected: {np.flatnonzero(act).tolist()}"
        assert O.detect(yn, B2, 0.0, P.rho).sum() == 1
