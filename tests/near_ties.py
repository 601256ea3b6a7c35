"""Classification of support mismatches between the GPU path and the oracle.

Test infrastructure over the oracle's trace (oracle.sfft(..., trace=True)).
On noisy inputs the GPU (FP32 bucket values and decisions) and the oracle
(FP64) can take a decision differently when it sits within rounding of its
threshold.  For every frequency in the symmetric difference of the two
supports this module finds the smallest decision margin the oracle met on
the buckets that frequency reaches, in every iteration:

  * detection: the bucket's round-0 magnitude against the threshold of the
    detection rule (noise threshold and relative floor);
  * round-to-round consistency: | |y_j| - |y_0| | against rho |y_0|;
  * location: the gap between the best and the second-best block (or
    position) in circular phase distance, at every step;
  * verification: each round's phase distance against pi / l;
  * top-K: the frequency's magnitude against the K-th largest.

A margin is the smallest perturbation of the bucket values, relative to
their size before the subtraction (the scale FP32 rounds at), that flips
the decision.  A mismatch is a near-tie when one of its margins is below
`tol` (1e-5), or when it shares a bucket in some iteration with a
mismatch that is one (a flipped decision changes what later iterations
subtract from every bucket the coefficient reaches).  Everything else is
reported as unexplained.
"""

from __future__ import annotations

import math

import numpy as np

import oracle.sfft_oracle as O

TWO_PI = 2.0 * math.pi


def _block_gaps(theta, i, it, N, l, q):
    """Phase gaps (radians) between the best and second-best candidate of
    every location step for bucket i, following the oracle's schedule."""
    L, e = it.L, it.e
    a = i * L - L // 2 - e
    qn, qd = q.numerator, q.denominator
    M2 = 2 * l * N
    gaps = []
    for j in range(1, it.R + 1):
        ln, tau = it.lens[j], it.taus[j]
        if it.kinds[j] == O.BLK:
            d = sorted((O.circ_dist(TWO_PI * (((2 * l * a + (2 * b + 1) * ln) * tau) % M2) / M2, theta[j]), b)
                       for b in range(l))
            gaps.append(d[1][0] - d[0][0])
            a = a + ((2 * d[0][1] * qd - qn) * ln) // (2 * qd * l)
        elif it.kinds[j] == O.ENUM:
            d = sorted(O.circ_dist(TWO_PI * ((c * tau) % N) / N, theta[j]) for c in range(a, a + ln))
            if len(d) > 1:
                gaps.append(d[1] - d[0])
            break
        else:  # direct: u = round(theta N / 2 pi); the margin is the distance to a half position
            x = theta[1] * N / TWO_PI
            gaps.append(abs((x - math.floor(x)) - 0.5) * TWO_PI / N * 2.0)
            break
    return gaps


def bucket_margin(tr, it, P, i):
    """Smallest relative decision margin of bucket i in one traced iteration."""
    ysub, yhat = tr["ysub"], tr["yhat"]
    N = P.N
    scale = float(np.max(np.abs(yhat[:, i]))) or 1e-300
    p0 = np.abs(ysub[0]) ** 2
    thr = max(2.0 * math.log(it.B) * float(np.median(p0)) / math.log(2.0), P.eta ** 2 * float(p0.max()))
    mag = np.abs(ysub[:, i])
    margins = [abs(mag[0] - math.sqrt(thr)) / max(scale, math.sqrt(thr))]
    if mag[0] > 0:
        margins.append(float(np.min(np.abs(np.abs(mag[1:] - mag[0]) - P.rho * mag[0]))) / scale
                       if len(mag) > 1 else math.inf)
    if tr["active"][i]:
        th = O.phases(ysub, i)
        # an angle decision flips when the bucket values move by about
        # gap * |y| (relative to the unsubtracted scale)
        small = float(np.min(mag)) / scale
        margins += [g * small for g in _block_gaps(th, i, it, N, P.l, P.q)]
        u = O.locate(th, i, it, N, P.l, P.q)
        for j in range(1, it.R + 1):
            dj = O.circ_dist(th[j], TWO_PI * ((it.taus[j] * u) % N) / N)
            margins.append(abs(dj - math.pi / P.l) * small)
    return min(margins)


def classify(gidx, gval, oidx, oval, info, P, tol=1e-5):
    """Returns dict(near_tie=[...], unexplained=[...], margins={f: m}) for
    the symmetric difference of the GPU and oracle supports."""
    N = P.N
    diff = sorted(set(int(f) for f in gidx) ^ set(int(f) for f in oidx))
    if not diff:
        return dict(near_tie=[], unexplained=[], margins={})
    # top-K margin: distance of |v| to the K-th largest magnitude of the oracle's store
    rec = info["iters"][-1]["rec"] if info["iters"] else {}
    mags = sorted((abs(v) for v in rec.values() if v != 0), reverse=True)
    kth = mags[P.K - 1] if len(mags) >= P.K else 0.0
    gmap = {int(f): v for f, v in zip(gidx, gval)}
    margins, touched = {}, {}
    for f in diff:
        m_best = math.inf
        v = rec.get(f, gmap.get(f, 0j))
        if kth > 0:
            m_best = abs(abs(v) - kth) / kth
        for tr, it in zip(info["iters"], P.iters):
            u = (it.sigma * f) % N
            bs = [b % it.B for b in O.bucket_range(u, it.L, it.D)]
            touched.setdefault(f, []).append((it.m, frozenset(bs)))
            for b in bs:
                m_best = min(m_best, bucket_margin(tr, it, P, b))
        margins[f] = m_best
    near = {f for f in diff if margins[f] < tol}
    changed = True
    while changed:  # collision cascade: shares a bucket of one iteration with a near tie
        changed = False
        for f in diff:
            if f in near:
                continue
            for g in list(near):
                if any(mf == mg and (bf & bg) for mf, bf in touched[f] for mg, bg in touched[g]):
                    near.add(f)
                    changed = True
                    break
    return dict(near_tie=sorted(near), unexplained=sorted(set(diff) - near), margins=margins)


def per_coefficient(gidx, gval, oidx, oval):
    """Per-coefficient relative error |v_gpu - v_oracle| / |v_oracle| over the
    common support: (max, median, array)."""
    common, gi, oi = np.intersect1d(gidx, oidx, return_indices=True)
    if len(common) == 0:
        return 0.0, 0.0, np.zeros(0)
    e = np.abs(np.asarray(gval)[gi] - np.asarray(oval)[oi]) / np.maximum(np.abs(np.asarray(oval)[oi]), 1e-300)
    return float(e.max()), float(np.median(e)), e
