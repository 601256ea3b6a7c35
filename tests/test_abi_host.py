"""C-ABI checks that need no GPU: every declared symbol is exported, the
host-only plan matches the oracle's plan exactly (integers) or to FP64
rounding (tables), and invalid parameters are rejected synchronously."""

import ctypes
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import oracle.sfft_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfft.h")

sfft = pytest.importorskip("paper_2011_05698_amd.sfft", reason="libsfft.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfft_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(sfft.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in sfft.h but not exported"
    assert sorted(sfft.EXPORTED) == names


PLANS = [
    # N, K, B, w, loops, l, q, delta, seed
    (2 ** 14, 50, 512, 7169, 8, 16, Fraction(1), 1e-8, 102),
    (2 ** 14, 50, 512, 7169, 8, 4, Fraction(1, 4), 1e-8, 102),
    (2 ** 20, 1000, 8192, 163841, 12, 2, Fraction(1, 2), 1e-6, 202),
    (2 ** 20, 1000, 8192, 163841, 12, 16, Fraction(1, 8), 1e-6, 202),
    (2 ** 22, 1000, 2048, 45057, 12, 16, Fraction(1), 1e-6, 602),
    (2 ** 12, 10, 128, 1536, 6, 8, Fraction(3, 2), 1e-7, 5),
]


@pytest.mark.parametrize("combine", ["sum", "vote"])
@pytest.mark.parametrize("location", ["multiscale", "direct"])
@pytest.mark.parametrize("case", PLANS, ids=lambda c: f"N{c[0]}_B{c[2]}_l{c[5]}_q{c[6]}")
def test_plan_matches_oracle(case, location, combine):
    N, K, B, w, M, l, q, delta, seed = case
    P = O.make_plan(N, K, B, w, M, l, q, delta, seed=seed, location=location, combine=combine)
    p = sfft.Plan(N, K, B, w, M, l, q, delta=delta, seed=seed, host_only=True, location=location,
                  combine=combine)
    assert p.samples == O.samples_per_signal(P)
    off = 0
    for m, it in enumerate(P.iters):
        g = p.iteration(m)
        assert (g["B"], g["L"], g["w"], g["h"], g["e"], g["R"]) == (it.B, it.L, it.w, it.h, it.e, it.R)
        assert (g["sigma"], g["sigma_inv"], g["tau0"]) == (it.sigma, it.sigma_inv, it.tau0)
        assert g["T"] == it.T
        assert g["tau"][1:] == it.taus[1:] and g["len"][1:] == it.lens[1:]
        assert g["y_offset"] == off
        assert g["last_kind"] == it.kinds[-1]  # 1: enumeration, 2: direct conversion
        off += (it.R + 1) * it.B
        assert abs(g["d_delta"] - it.d_delta) <= 1e-9 * it.d_delta
        G, Ghat = p.tables(m)
        assert np.max(np.abs(G - it.G)) <= 1e-13 * it.L
        assert np.max(np.abs(Ghat - it.Ghat)) <= 1e-12
    assert p.yhat_elems == off


def test_invalid_parameters_rejected():
    bad = [
        dict(N=1000), dict(N=2 ** 31), dict(B=24), dict(B=2 ** 13), dict(K=0), dict(K=600),
        dict(w=100), dict(w=2 ** 14), dict(loops=0), dict(l=3), dict(l=1), dict(q=0.0), dict(q=0.3),
        dict(l=2, q=1.0), dict(delta=0.5), dict(delta=0.0), dict(combine=2),
    ]
    base = dict(N=2 ** 14, K=50, B=512, w=7169, loops=8, l=16, q=1.0, delta=1e-8, combine=0)
    for b in bad:
        a = {**base, **b}
        o = sfft.sfft_default_options()
        o.delta, o.combine, o.flags = a["delta"], a["combine"], sfft.SFFT_PLAN_HOST_ONLY
        with pytest.raises(sfft.SfftError) as ei:
            sfft.sfft_plan(a["N"], a["K"], a["B"], a["w"], a["loops"], a["l"], a["q"], o)
        assert ei.value.status in (1, 2), b


def test_paper_literal_parameter_pairs_are_rejected():
    """The literal (multiscale, extension) pairs of the workload list shrink
    nothing under the paper's region rule (factor (1+q)/l >= 1): rejected."""
    for l, q in [(2, 4.0), (1, 2.0), (2, 2.0), (4, 4.0), (4, 8.0)]:
        with pytest.raises(sfft.SfftError):
            sfft.Plan(2 ** 14, 50, 512, 7169, 8, l, q, host_only=True)


def test_unsupported_bucket_count():
    """The bucket DFT holds B values in 128 KiB of LDS: B <= 16384 for the
    FP32 and FP16 forms, B <= 8192 for complex128."""
    sfft.Plan(2 ** 20, 100, 16384, 16384 * 20 + 1, 2, 16, 1.0, host_only=True)
    sfft.Plan(2 ** 20, 100, 8192, 8192 * 20 + 1, 2, 16, 1.0, dtype="c128", host_only=True)
    with pytest.raises(sfft.SfftError) as ei:
        sfft.Plan(2 ** 22, 100, 32768, 32768 * 22 + 1, 2, 16, 1.0, host_only=True)
    assert ei.value.status == 2
    with pytest.raises(sfft.SfftError) as ei:
        sfft.Plan(2 ** 20, 100, 16384, 16384 * 20 + 1, 2, 16, 1.0, dtype="c128", host_only=True)
    assert ei.value.status == 2


def test_host_only_plan_cannot_execute():
    p = sfft.Plan(2 ** 14, 50, 512, 7169, 8, 16, 1.0, host_only=True)
    with pytest.raises(sfft.SfftError) as ei:
        sfft.sfft_hash_to_bins(p.handle, None, 1.0, None, stream=0)
    assert ei.value.status in (1, 6)


def test_status_strings():
    for s in range(7):
        assert sfft.sfft_status_string(s)
