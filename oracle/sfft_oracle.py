"""FP64 CPU oracle for the sFFT4.0 hot path (multiscale sparse FFT).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import or call this module.  It
shares no code with the HIP library: it computes its own plan (window, window
spectrum, location schedule, random draws) from the paper's definitions and
runs the method step by step in float64 NumPy, in the order the paper gives.

Paper: B. Li, Z. Jiang, J. Chen, "On Performance of Multiscale Sparse Fast
Fourier Transform Algorithm" (arXiv 2011.05698).

Conventions (Sec. 2.1, Eq. 1-2): omega_N = exp(-2 pi i / N) and the forward
DFT carries the 1/N factor, xhat_f = (1/N) sum_j x_j omega^{f j}.

Readings of passages the paper leaves silent or garbled (each one is listed
in the design notes):
  * Eq. 12 needs the 1/N factor: yhat = (1/N) FFT_B(y), which makes Eq. 12-14
    exact identities.
  * Eq. 16 sign: theta = arg(yhat_0 conj(yhat_j)) = 2 pi (tau_j u mod N)/N.
  * Window (Sec. 2.3): boxcar of width L with half-weight edges, times a
    Gaussian in time, truncated to |t| <= h = (w-1)/2; the Gaussian width is
    set so that the truncation level is delta.
  * Location (Sec. 3.2): extended first region L + 2e (e = window transition
    half-width), integer schedule tau_j = floor(N / len_j), rational block
    centres, floor for the region start, a final enumeration step.
  * Detection and verification rules are readings of their own (the paper
    assumes isolated buckets).  Verification accepts a located position only
    in its home bucket, the one whose range Lemma 1 and Eq. 14 assign it.
  * Estimation takes the median over the R+1 rounds of one iteration.
  * The two-round location of sFFT3.0, which the paper sets against sFFT4.0
    (Sec. 1, Sec. 3.1: R_m = 2 rounds), is read as offsets tau0 and tau0 + 1
    and the phase-to-position conversion u = round(theta N / 2 pi) mod N
    (Eq. 16 with tau = 1), then the same verification and estimation.
  * The cross-iteration vote (the one-shot framework that Sec. 1 and the opening
    of Sec. 3 set against the iterative one: several random bucketizations, a vote over
    them) is read as: every loop has the full B buckets and w taps, no loop
    subtracts, a frequency is kept when at least half of the loops located
    it, and its value is the median over those loops (real and imaginary
    parts separately).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np
from scipy.special import erfcinv

__all__ = [
    "SplitMix64", "Iteration", "Plan", "make_plan", "flat_window",
    "location_schedule", "hash_to_bins", "subtract", "detect", "locate",
    "verify", "estimate", "sfft", "circ_dist", "samples_per_signal",
    "window_spectrum", "bucket_range", "phases", "multiscale_upper_bound",
    "extension_lower_bound", "BLK", "ENUM", "DIRECT", "combine_votes", "reconstruct", "home_bucket",
]

TWO_PI = 2.0 * math.pi
MASK64 = (1 << 64) - 1
BLK, ENUM, DIRECT = 0, 1, 2


# --------------------------------------------------------------------------
# Random draws for sigma and tau (Sec. 2.2).  SplitMix64 as published by
# Steele, Lea and Flood (OOPSLA 2014): add the golden gamma, then two
# xor-shift-multiply mixing rounds and a final xor-shift.
# --------------------------------------------------------------------------
class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)


# --------------------------------------------------------------------------
# Flat window (Sec. 2.3, Eq. 9-10).
# --------------------------------------------------------------------------
def flat_window(N: int, B: int, w: int, delta: float):
    """Flat window G for bucket width L = N/B, support w (odd), level delta.

    G is the inverse DFT (Eq. 2 normalisation) of a width-L boxcar whose two
    edge bins carry weight 1/2, multiplied pointwise by a time-domain
    Gaussian exp(-t^2 / (2 s_t^2)) with s_t chosen so that the Gaussian has
    fallen to delta at the truncation point h = (w-1)/2.  By the product
    theorem (Eq. 4) Ghat is the boxcar convolved with a unit-sum Gaussian of
    width s_f = N / (2 pi s_t) bins, i.e. the Gaussian-convolved boxcar the
    paper describes.

    Returns (G_half, info): G_half[t] = G_t for t = 0..h (G is even), and
    info with s_t, s_f, d_delta (transition half-width where the Gaussian
    tail falls to delta) and e = ceil(d_delta).
    """
    L = N // B
    h = (w - 1) // 2
    s_t = h / math.sqrt(2.0 * math.log(1.0 / delta))
    t = np.arange(h + 1, dtype=np.float64)
    G = np.empty(h + 1, dtype=np.float64)
    G[0] = float(L)
    tt = t[1:]
    # sin(pi L t / N) with the argument reduced exactly: L t mod 2N.
    lt = (np.arange(1, h + 1, dtype=np.int64) * L) % (2 * N)
    G[1:] = (np.sin(math.pi * lt / N) * (np.cos(math.pi * tt / N) / np.sin(math.pi * tt / N))
             * np.exp(-(tt * tt) / (2.0 * s_t * s_t)))
    s_f = N / (TWO_PI * s_t)
    d_delta = math.sqrt(2.0) * s_f * float(erfcinv(2.0 * delta))
    e = int(math.ceil(d_delta))
    return G, dict(s_t=s_t, s_f=s_f, d_delta=d_delta, e=e, L=L, h=h)


def window_spectrum(N: int, G_half: np.ndarray, kmax: int) -> np.ndarray:
    """Ghat_k for k = 0..kmax: the DFT (Eq. 2, with the 1/N factor) of the
    window placed on the circle (G at t and at -t mod N).  G is real and
    even, so Ghat is real and even.  Computed with a dense real FFT of size N
    (a library FFT serving as the DFT of the definition)."""
    h = len(G_half) - 1
    g = np.zeros(N, dtype=np.float64)
    g[0] = G_half[0]
    g[1:h + 1] = G_half[1:]
    g[N - h:] = G_half[1:][::-1]
    spec = np.fft.rfft(g) / N
    return spec.real[:kmax + 1].copy()


# --------------------------------------------------------------------------
# Location schedule (Sec. 3.2, the multiscale block approach).
# --------------------------------------------------------------------------
def location_schedule(N: int, L: int, e: int, l: int, q: Fraction):
    """Region lengths len_j and multipliers tau_j for location steps j = 1..R.

    The first region is the bucket extended by the window's transition
    half-width on both sides (len_1 = L + 2e).  Each block step keeps one of
    l blocks plus q/2 blocks on either side, so the length shrinks by
    (1+q)/l; one is added to absorb the floor on the region start.  Once the
    region holds no more than l positions, or would stop shrinking, the last
    step enumerates its positions.  tau_j = floor(N / len_j) stretches the
    region over (almost) one full turn of phase.
    Returns lists indexed 1..R (index 0 unused: the reference round)."""
    lens, taus, kinds = [0], [0], [BLK]
    ln = L + 2 * e
    while True:
        tau = N // ln
        nxt = math.ceil((1 + q) * ln / l) + 1
        lens.append(ln)
        taus.append(tau)
        if ln <= l or nxt >= ln:
            kinds.append(ENUM)
            break
        kinds.append(BLK)
        ln = nxt
    return lens, taus, kinds


# --------------------------------------------------------------------------
# Plan (Sec. 3.1 schedule of iterations; Sec. 3.3 parameter rules).
# --------------------------------------------------------------------------
@dataclass
class Iteration:
    m: int
    B: int
    L: int
    w: int
    h: int
    e: int
    d_delta: float
    G: np.ndarray          # G_t, t = 0..h
    Ghat: np.ndarray       # Ghat_k, k = 0..L/2+e
    lens: list
    taus: list
    kinds: list
    R: int
    sigma: int
    sigma_inv: int
    tau0: int
    T: list                # round offsets T_j, j = 0..R

    @property
    def D(self) -> int:
        """Largest bucket-centre distance that still receives a coefficient."""
        return self.L // 2 + self.e


@dataclass
class Plan:
    N: int
    K: int
    B: int
    w: int
    loops: int
    l: int
    q: Fraction
    delta: float
    seed: int
    eta: float
    rho: float
    b_min: int
    combine: str = "sum"
    iters: list = field(default_factory=list)


def make_plan(N, K, B, w, loops, l, q, delta=1e-6, seed=0, b_min=16, eta=1e-4, rho=0.25,
              location="multiscale", combine="sum") -> Plan:
    """Per-iteration parameters: B_m = max(B >> (m-1), b_min) buckets (the
    paper halves B per iteration), w_m = floor(w B_m / B) | 1 taps, a fresh
    odd sigma_m and offset tau0_m per iteration from SplitMix64(seed).
    location = "multiscale" (sFFT4.0, Sec. 3.2) or "direct" (the two-round
    location of sFFT3.0: one step with tau_1 = 1).  combine = "sum" (the
    iterative framework, Sec. 3.1) or "vote" (the one-shot vote over loops:
    every loop keeps B_m = B and w_m = w)."""
    assert location in ("multiscale", "direct")
    assert combine in ("sum", "vote")
    assert N & (N - 1) == 0 and B & (B - 1) == 0
    q = Fraction(q)
    if w % 2 == 0:
        w += 1
    rng = SplitMix64(seed)
    P = Plan(N, K, B, w, loops, l, q, delta, seed, eta, rho, b_min, combine)
    for m in range(1, loops + 1):
        Bm = B if combine == "vote" else max(B >> (m - 1), b_min)
        Lm = N // Bm
        wm = (w * Bm // B) | 1
        G, info = flat_window(N, Bm, wm, delta)
        e = info["e"]
        Ghat = window_spectrum(N, G, Lm // 2 + e)
        if location == "direct":
            lens, taus, kinds = [0, Lm + 2 * e], [0, 1], [BLK, DIRECT]
        else:
            lens, taus, kinds = location_schedule(N, Lm, e, l, q)
        R = len(lens) - 1
        sigma = 2 * (rng.next() % (N // 2)) + 1
        tau0 = rng.next() % N
        T = [tau0] + [(tau0 + taus[j]) % N for j in range(1, R + 1)]
        P.iters.append(Iteration(m, Bm, Lm, wm, info["h"], e, info["d_delta"], G, Ghat,
                                 lens, taus, kinds, R, sigma, pow(sigma, -1, N), tau0, T))
    return P


def samples_per_signal(P: Plan) -> int:
    """Samples one execute reads: each of the R_m+1 rounds of iteration m
    reads w_m samples (the cost model of Sec. 2.4 and Sec. 3.1)."""
    return sum((it.R + 1) * it.w for it in P.iters)


# --------------------------------------------------------------------------
# HashToBins: frequency bucketization (Sec. 2.4, Lemma 1, Eq. 13).
# --------------------------------------------------------------------------
def hash_to_bins(x: np.ndarray, sigma: int, T: int, G_half: np.ndarray, B: int) -> np.ndarray:
    """yhat = F_B U_L Q_L S_T P_sigma x.

    Permutation (Eq. 7): x'_t = x[sigma (t - T) mod N].  Window (Eq. 10):
    x''_t = G_t x'_t for |t| <= h.  Aliasing (Eq. 11): y_b = sum of x''_t over
    t = b mod B.  B-point DFT with the 1/N factor (Eq. 12 reading):
    yhat[i] = (1/N) sum_b y_b exp(-2 pi i i b / B), which equals the
    filtered permuted spectrum at iL."""
    N = x.shape[0]
    h = len(G_half) - 1
    t = np.arange(-h, h + 1, dtype=np.int64)
    idx = (sigma * (t - T)) % N
    vals = G_half[np.abs(t)] * x[idx]
    b = t % B
    y = (np.bincount(b, weights=vals.real, minlength=B)
         + 1j * np.bincount(b, weights=vals.imag, minlength=B))
    return np.fft.fft(y) / N


def bucket_range(u: int, L: int, D: int):
    """Unwrapped bucket indices i with |iL - u| <= D."""
    lo = -((D - u) // L)          # ceil((u - D) / L)
    hi = (u + D) // L
    return range(lo, hi + 1)


def subtract(yhat: np.ndarray, rec: dict, it: Iteration, N: int) -> np.ndarray:
    """Remove already-recovered coefficients in bucket space (Sec. 3.1,
    iteration steps 2-3): for (f, v) with u = sigma f mod N, every bucket i
    whose centre iL lies within L/2 + e of u holds v omega^{T_j u} Ghat_{iL-u}
    in round j (Eq. 14), which is subtracted."""
    out = yhat.copy()
    B, L = it.B, it.L
    for f, v in rec.items():
        u = (it.sigma * f) % N
        for i in bucket_range(u, L, it.D):
            g = it.Ghat[abs(i * L - u)]
            for j in range(it.R + 1):
                p = (it.T[j] * u) % N
                out[j, i % B] -= v * np.exp(-1j * TWO_PI * p / N) * g
    return out


# --------------------------------------------------------------------------
# Reconstruction within one iteration (Sec. 3.2).
# --------------------------------------------------------------------------
def detect(yhat: np.ndarray, B: int, eta: float, rho: float) -> np.ndarray:
    """Singleton screen (the paper assumes an isolated coefficient per
    bucket; this rule is the build's reading).  nu = median |yhat_0|^2 / ln 2
    estimates the per-bucket noise power; bucket i is active if
    |yhat_0[i]|^2 >= max(2 ln(B) nu, (eta max|yhat_0|)^2), is non-zero, and
    its magnitude is the same in every round to within rho."""
    p0 = np.abs(yhat[0]) ** 2
    nu = np.median(p0) / math.log(2.0)
    thr = max(2.0 * math.log(B) * nu, eta * eta * float(p0.max()))
    mag = np.abs(yhat)
    consistent = np.all(np.abs(mag - mag[0]) <= rho * mag[0], axis=0)
    return (p0 >= thr) & (p0 > 0) & consistent


def circ_dist(a: float, b: float) -> float:
    """Circular distance between two angles in radians."""
    d = abs(a - b) % TWO_PI
    return min(d, TWO_PI - d)


def phases(yhat: np.ndarray, i: int) -> list:
    """theta_j = arg(yhat_0[i] conj(yhat_j[i])) in [0, 2 pi) for j = 1..R:
    the two-round phase difference of Eq. 15-16, equal to 2 pi (tau_j u mod N)/N
    for a lone coefficient at permuted position u."""
    th = [0.0]
    for j in range(1, yhat.shape[0]):
        z = yhat[0, i] * np.conj(yhat[j, i])
        th.append(math.atan2(z.imag, z.real) % TWO_PI)
    return th


def locate(theta: list, i: int, it: Iteration, N: int, l: int, q: Fraction) -> int:
    """Multiscale block location of the lone coefficient of bucket i.

    Region [a, a + len_j), first region centred on the bucket and extended by
    e on both sides.  Block step: split into l blocks of len_j/l positions;
    the block whose centre position p, seen through tau_j (phase
    2 pi (p tau_j mod N)/N), is closest to theta_j wins (smallest index on a
    tie); the new region starts q/2 blocks before it (floor).  Last step:
    the single position of the region whose phase is closest (smallest
    position on a tie).  Returns u in [0, N)."""
    L, e = it.L, it.e
    if it.kinds[1] == DIRECT:
        # theta_1 = 2 pi u / N: the nearest position, halves rounded up
        return math.floor(theta[1] * N / TWO_PI + 0.5) % N
    a = i * L - L // 2 - e
    qn, qd = q.numerator, q.denominator
    M2 = 2 * l * N
    for j in range(1, it.R + 1):
        ln, tau = it.lens[j], it.taus[j]
        if it.kinds[j] == BLK:
            best_b, best_d = 0, math.inf
            for b in range(l):
                # centre a + (b + 1/2) ln / l, times tau, mod N, as a fraction of 2lN
                num = ((2 * l * a + (2 * b + 1) * ln) * tau) % M2
                d = circ_dist(TWO_PI * num / M2, theta[j])
                if d < best_d:
                    best_b, best_d = b, d
            # a <- floor(a + (b* - q/2) ln / l)
            a = a + ((2 * best_b * qd - qn) * ln) // (2 * qd * l)
        else:
            best_c, best_d = a, math.inf
            for c in range(a, a + ln):
                d = circ_dist(TWO_PI * ((c * tau) % N) / N, theta[j])
                if d < best_d:
                    best_c, best_d = c, d
            return best_c % N
    raise AssertionError("schedule must end with an enumeration step")


def home_bucket(u: int, L: int, B: int) -> int:
    """The bucket that holds position u: the i with u in [iL - L/2, iL + L/2)
    (the bucket range of Lemma 1 and Eq. 14, halves rounded up)."""
    return ((u + L // 2) // L) % B


def verify(theta: list, u: int, i: int, it: Iteration, N: int, l: int) -> bool:
    """Accept u only if bucket i is its home bucket (Eq. 14 estimates a
    coefficient from the bucket whose range [iL - L/2, iL + L/2) holds it;
    the location searched a wider region, L + 2e, so that leakage from the
    transition band cannot alias) and every round's phase agrees with it to
    within pi/l (the Eq. 18 bound on the phase error)."""
    if home_bucket(u, it.L, it.B) != i:
        return False
    for j in range(1, it.R + 1):
        if circ_dist(theta[j], TWO_PI * ((it.taus[j] * u) % N) / N) > math.pi / l:
            return False
    return True


def estimate(yhat: np.ndarray, i: int, u: int, it: Iteration, N: int) -> complex:
    """Eq. 14 per round, xhat_f = yhat_j[i] omega^{-T_j u} / Ghat_{iL-u}, and
    the median over the R+1 rounds, real and imaginary parts separately
    (mean of the two middle values for an even count)."""
    dist = abs(i * it.L - u)
    dist = min(dist, N - dist)
    g = it.Ghat[dist]
    est = np.array([yhat[j, i] * np.exp(1j * TWO_PI * ((it.T[j] * u) % N) / N) / g
                    for j in range(it.R + 1)])
    return complex(np.median(est.real), np.median(est.imag))


def combine_votes(votes: dict, loops: int) -> dict:
    """The vote over loops: votes maps a frequency to the values that the
    loops which located it estimated.  A frequency is kept when at least
    half of the loops located it (2 n >= loops); its value is the median of
    its n values, real and imaginary parts separately (mean of the two
    middle values for an even n)."""
    out = {}
    for f, vs in votes.items():
        if 2 * len(vs) >= loops:
            a = np.asarray(vs, dtype=np.complex128)
            out[f] = complex(np.median(a.real), np.median(a.imag))
    return out


def reconstruct(ysub: np.ndarray, it: Iteration, P: Plan):
    """One iteration's reconstruction (Sec. 3.2) from its bucket values after
    subtraction: singleton detection, location and verification of every
    active bucket, and the Eq. 14 median estimate of each located position.
    Verification accepts a position only from its home bucket, so each
    position yields at most one candidate.  Returns (cands {f: v}, active
    mask, located position per bucket or -1)."""
    N = P.N
    active = detect(ysub, it.B, P.eta, P.rho)
    located = np.full(it.B, -1, dtype=np.int64)
    cands = {}
    for i in np.flatnonzero(active):
        i = int(i)
        th = phases(ysub, i)
        u = locate(th, i, it, N, P.l, P.q)
        if not verify(th, u, i, it, N, P.l):
            continue
        located[i] = u
        f = (it.sigma_inv * u) % N
        cands[f] = estimate(ysub, i, u, it, N)
    return cands, active, located


# --------------------------------------------------------------------------
# The whole method (Sec. 3.1: iterations; output is the K largest, Sec. 2.1).
# --------------------------------------------------------------------------
def sfft(x: np.ndarray, P: Plan, trace: bool = False):
    """Run all iterations on x (complex, length N).  Returns (idx, val, info)
    where idx (sorted ascending) and val hold at most K recovered
    coefficients: the K largest |v| of the accumulated result (ties to the
    smaller index, exact zeros dropped)."""
    N = P.N
    x = np.asarray(x, dtype=np.complex128)
    assert x.shape == (N,)
    rec: dict = {}
    votes: dict = {}
    vote = P.combine == "vote"
    info = dict(iters=[])
    for it in P.iters:
        yhat = np.stack([hash_to_bins(x, it.sigma, it.T[j], it.G, it.B) for j in range(it.R + 1)])
        ysub = yhat if vote else subtract(yhat, rec, it, N)
        cands, active, located = reconstruct(ysub, it, P)
        for f, v in cands.items():
            if vote:
                votes.setdefault(f, []).append(v)
            else:
                rec[f] = rec.get(f, 0j) + v
        if trace:
            info["iters"].append(dict(yhat=yhat, ysub=ysub, active=active, located=located,
                                      cands=dict(cands), rec=dict(rec)))
    if vote:
        rec = combine_votes(votes, P.loops)
    items = [(f, v) for f, v in rec.items() if v != 0]
    items.sort(key=lambda fv: (-abs(fv[1]), fv[0]))
    items = sorted(items[:P.K])
    idx = np.array([f for f, _ in items], dtype=np.int64)
    val = np.array([v for _, v in items], dtype=np.complex128)
    info["rec_size"] = len(rec)
    info["samples"] = samples_per_signal(P)
    return idx, val, info


# --------------------------------------------------------------------------
# Parameter bounds of Sec. 3.2 (Eq. 18-19).
# --------------------------------------------------------------------------
def multiscale_upper_bound(max_dphi: float) -> float:
    """Eq. 18: the located block contains u only if the phase error stays
    within half a block, so l <= pi / max(dPhi)."""
    return math.pi / max_dphi


def extension_lower_bound(max_dphi: float, l: float) -> float:
    """Eq. 19: the extended region (q/2 blocks per side) absorbs the phase
    error only if q >= max(dPhi) l / pi."""
    return max_dphi * l / math.pi
