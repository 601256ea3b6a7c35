"""The recovery kernel's body on the CPU (tests/emu): no GPU is touched.

tests/emu/hip_emu.h emulates the HIP device code the recovery uses (one host
thread per work item, barriers, DPP moves per wavefront of 64 threads);
tests/emu/recover_emu.cpp runs recover_body.h, the code the GPU kernels
run, on one signal whose bucket values come from the oracle's HashToBins
(built twice: plain host arithmetic, and with fused multiply-adds wherever
the compiler can contract, as the GPU compiler does),
with every buffer it reads or writes (bucket values, workspace, plan
tables, outputs, the workgroup's LDS) placed against an inaccessible guard
page, past its end in one run and before its start in another.  Any access
outside a buffer stops the program and names the buffer; a barrier or wave
move that not every thread reaches is reported as well.  The result must be
the oracle's support, with values within the GPU tests' tolerance.

The program runs the kernel body in both workgroup shapes (256 threads, and
512 threads with twice the LDS) and requires the same bits from both; the
denser N = 2^16 case is one where a team size that followed the shape would
change them.

The first case is the end-to-end case whose first GPU run, with an earlier
recovery kernel since replaced, faulted the GPU (complex128, (l, q) =
(16, 1)); the others are its siblings, larger shapes, and the direct
location and vote options.
"""

import hashlib
import os
import shutil
import subprocess
import struct
from fractions import Fraction

import numpy as np
import pytest

import oracle.sfft_oracle as O
from paper_2011_05698_amd.signals import SignalSpec, make_signal

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_05698_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")
BUILD = os.path.join(ROOT, "_build", "emu")

DTYPES = {"c64": 0, "c128": 1}


FLAVOURS = {
    # plain host arithmetic, and fused multiply-adds wherever the compiler can
    # contract (as the GPU compiler does): decisions must not hinge on either
    "plain": ["-O2"],
    "fma": ["-O2", "-mfma", "-ffp-contract=fast"],
}
# host AddressSanitizer and UndefinedBehaviorSanitizer: every thread's
# private arrays (the kernel's registers and scratch) are host stack arrays,
# which the guard pages do not cover and these do
SANITIZED = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]


# the fold's FP16 storage form needs a host compiler with _Float16: ROCm's clang
HOST_CLANG = "/opt/rocm/llvm/bin/clang++"


def _build(main, flavour):
    """Builds an emulation program once per source state (host compiler, no HIP)."""
    srcs = [os.path.join(EMU, f) for f in ("recover_emu.cpp", "emu_selftest.cpp", "fold_emu.cpp", "ilv_emu.cpp",
                                           "hip_emu.h", "guarded.h")]
    srcs += [os.path.join(EMU, "include", "hip", "hip_runtime.h"), os.path.join(CSRC, "plan.cpp"),
             os.path.join(ROOT, "include", "sfft.h")]
    srcs += [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".h")]
    flags = SANITIZED if flavour == "sanitized" else FLAVOURS[flavour]
    h = hashlib.sha256(" ".join(flags).encode())
    for f in srcs:
        h.update(open(f, "rb").read())
    exe = os.path.join(BUILD, f"{main}_{flavour}_{h.hexdigest()[:16]}")
    if os.path.exists(exe):
        return exe
    gxx = HOST_CLANG if main in ("fold_emu", "ilv_emu") else shutil.which("g++")
    if not gxx or not os.path.exists(gxx):
        pytest.skip(f"host compiler for {main} not found")
    os.makedirs(BUILD, exist_ok=True)
    tmp = f"{exe}.{os.getpid()}.tmp"  # parallel test workers may build the same program
    extra = [os.path.join(CSRC, "plan.cpp")] if main in ("recover_emu", "fold_emu", "ilv_emu") else []
    subprocess.run([gxx, "-std=c++17", *flags, "-g", "-pthread", "-Wno-unknown-pragmas",
                    "-I", os.path.join(EMU, "include"), "-I", EMU, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(EMU, main + ".cpp"), *extra, "-o", tmp], check=True, capture_output=True)
    os.replace(tmp, exe)
    return exe


def test_emulation_reports_faults_and_divergence():
    """The emulation itself: a write one element past or before a guarded
    buffer stops the program and names the buffer; a wave move that one
    lane skips is reported; the kernel's DPP team sums, wave extrema and
    wave scan equal their definitions."""
    exe = _build("emu_selftest", "plain")
    for what, byte in (("fault-after", "400"), ("fault-before", "-4")):
        r = subprocess.run([exe, what], capture_output=True, text=True, timeout=60)
        assert r.returncode == 86, (what, r.returncode, r.stdout, r.stderr)
        assert f"access at byte {byte} of self-test buffer" in r.stderr
    env = dict(os.environ, EMU_BARRIER_TIMEOUT_S="2")
    r = subprocess.run([exe, "diverge"], capture_output=True, text=True, timeout=60, env=env)
    assert r.returncode == 87 and "barrier not reached by every thread" in r.stderr, (r.returncode, r.stderr)
    r = subprocess.run([exe, "dpp"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and "dpp: 0 mismatches" in r.stdout, (r.stdout, r.stderr)


def oracle_buckets(x, P):
    """Bucket values of every round of every iteration, in the plan's layout."""
    return np.concatenate([np.concatenate([O.hash_to_bins(x, it.sigma, it.T[j], it.G, it.B) for j in range(it.R + 1)])
                           for it in P.iters])


def run_emulated(tmp_path, y, N, K, B, w, M, l, q, delta, seed, dtype, guard_mode, flavour, location=0, combine=0,
                 env=None):
    exe = _build("recover_emu", flavour)
    inp, out = tmp_path / f"in{guard_mode}.bin", tmp_path / f"out{guard_mode}_{flavour}.bin"
    y = np.asarray(y, dtype=np.complex128)
    with open(inp, "wb") as f:
        f.write(struct.pack("<qqqqiiddQiiiiq", N, K, B, w, M, l, float(q), delta, seed, DTYPES[dtype], location,
                            combine, guard_mode, len(y)))
        f.write(np.stack([y.real, y.imag], axis=1).astype("<f8").tobytes())
    r = subprocess.run([exe, str(inp), str(out)], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, f"exit {r.returncode}: {r.stdout[-2000:]} {r.stderr[-2000:]}"
    data = open(out, "rb").read()
    c = struct.unpack_from("<q", data)[0]
    rec = np.frombuffer(data[8:], dtype=np.dtype([("f", "<i8"), ("re", "<f8"), ("im", "<f8")]), count=c)
    return rec["f"].copy(), rec["re"] + 1j * rec["im"]


CASES = [
    # N, K, B, w, loops, l, q, delta, dtype, signal seed, plan seed, location, combine
    (2 ** 14, 50, 512, 7169, 8, 16, Fraction(1), 1e-8, "c128", 101, 102, "multiscale", "sum"),
    (2 ** 14, 50, 512, 7169, 8, 4, Fraction(1, 4), 1e-8, "c128", 101, 102, "multiscale", "sum"),
    (2 ** 14, 50, 512, 7169, 8, 16, Fraction(1), 1e-8, "c64", 101, 102, "multiscale", "sum"),
    (2 ** 16, 200, 512, 8193, 10, 16, Fraction(1), 1e-6, "c64", 9, 10, "multiscale", "sum"),
    (2 ** 16, 200, 512, 8193, 10, 16, Fraction(1), 1e-6, "c128", 9, 10, "multiscale", "sum"),
    (2 ** 16, 400, 1024, 16385, 10, 16, Fraction(1), 1e-6, "c64", 19, 20, "multiscale", "sum"),
    (2 ** 14, 50, 512, 7169, 8, 16, Fraction(1), 1e-6, "c64", 131, 132, "direct", "sum"),
    (2 ** 14, 50, 512, 7169, 8, 16, Fraction(1), 1e-6, "c128", 141, 142, "multiscale", "vote"),
]


@pytest.mark.parametrize("flavour", sorted(FLAVOURS))
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}_K{c[1]}_l{c[5]}_q{c[6]}_{c[8]}_{c[11]}_{c[12]}")
def test_emulated_recovery_in_bounds_and_exact(tmp_path, case, flavour):
    N, K, B, w, M, l, q, delta, dt, ss, ps, loc, comb = case
    x, sup, _ = make_signal(SignalSpec(N, K, ss))
    P = O.make_plan(N, K, B, w, M, l, q, delta, seed=ps, location=loc, combine=comb)
    y = oracle_buckets(x, P)
    if dt == "c64":
        y = y.astype(np.complex64)
    oidx, oval, _ = O.sfft(x, P)
    if loc == "multiscale" and comb == "sum":
        assert np.array_equal(oidx, np.sort(sup))
    tol = 1e-10 if dt == "c128" else 1e-4
    codes = dict(location={"multiscale": 0, "direct": 1}[loc], combine={"sum": 0, "vote": 1}[comb])
    for mode in (0, 1):  # guard pages after, then before, every buffer
        gidx, gval = run_emulated(tmp_path, y, N, K, B, w, M, l, q, delta, ps, dt, mode, flavour, **codes)
        assert np.array_equal(gidx, oidx), set(gidx) ^ set(oidx)
        err = np.linalg.norm(gval - oval) / np.linalg.norm(oval)
        assert err <= tol, err
        assert np.max(np.abs(gval - oval) / np.abs(oval)) <= 10 * tol


FOLD_CASES = [
    # N, K, B, w, loops, l, q, delta, plan seed, dtypes x Kahan, (tiles, union tiles) or None
    (2 ** 14, 40, 512, 7169, 8, 16, "1", 1e-6, 900, [(d, k) for d in (0, 1, 2) for k in (0, 1)], None),
    (2 ** 20, 200, 2048, 40961, 12, 4, "0.25", 1e-6, 61, [(0, 0), (1, 1)], None),
    # the metric plan: rounds 0..2 of the iterations with B = 2048..256 unite
    # (offsets 0, tau_1, tau_2 step by less than w; tau_3 - tau_2 > w): 8 + 4
    # + 2 + 1 union tiles, and the tile count falls from 89 to 59
    (2 ** 22, 1000, 2048, 45057, 12, 16, "1", 1e-6, 602, [(0, 0), (2, 0)], (59, 15)),
]


@pytest.mark.parametrize("flavour", sorted(FLAVOURS))
@pytest.mark.parametrize("case", FOLD_CASES, ids=lambda c: f"N{c[0]}_B{c[2]}_l{c[5]}")
def test_emulated_fold_union_tiles_bit_exact(case, flavour):
    """The per-signal fold's union tiles (rounds whose windows overlap round
    0's, gathered once) give every bucket value bit for bit what one-round
    tiles give, for 8, 16 and 24 taps in flight, in complex64, complex128
    and FP16 storage, with and without Kahan summation; every item is
    written and every access stays inside its buffer (guard pages after,
    then before, every buffer).  The last case is the metric plan
    (N = 2^22, B = 2048, w = 45057, 12 iterations)."""
    exe = _build("fold_emu", flavour)
    N, K, B, w, M, l, q, delta, seed, forms, counts = case
    for dtype, kahan in forms:
        for mode in (0, 1):
            args = [str(a) for a in (N, K, B, w, M, l, q, delta, seed, dtype, kahan, mode)]
            r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300)
            assert r.returncode == 0, (args, r.returncode, r.stdout[-2000:], r.stderr[-2000:])
            assert r.stdout.startswith("FOLD OK") and " union 0 " not in r.stdout, r.stdout
            if counts:
                assert f"tiles {counts[0]} union {counts[1]} " in r.stdout, r.stdout


ILV_CASES = [
    # dtype, Kahan, signals, ld, guard mode, most signals per lane
    (0, 0, 100, 102, 0, 2),   # complex64, two groups of 64 (the last ragged): one workgroup per two tiles
    (2, 1, 100, 102, 1, 2),   # FP16 pairs with per-signal scales, Kahan; ld not a multiple of 4
    (2, 0, 200, 204, 0, 4),   # FP16 pairs, four groups (the last ragged): one workgroup per four tiles
    (2, 0, 100, 101, 1, 1),   # odd ld: one signal per lane
    (0, 0, 65, 66, 1, 1),     # odd signal count
    (1, 1, 5, 5, 0, 1),       # complex128: always one signal per lane
]


@pytest.mark.parametrize("case", ILV_CASES, ids=lambda c: f"d{c[0]}_k{c[1]}_n{c[2]}_ld{c[3]}_g{c[4]}")
def test_emulated_position_major_fold_bit_exact(case):
    """The position-major fold body, with one, two and four adjacent signals
    per lane, gives every signal's bucket values bit for bit what the
    per-signal fold gives on a contiguous copy of that signal, for 8, 16
    and 24 taps in flight; every item is written and every access stays
    inside its buffer (guard pages after or before every buffer).  L > 1
    signals per lane run exactly where the library allows them (two for
    complex64, two or four for FP16 pairs; ld, the signal count and the
    group count multiples of L)."""
    exe = _build("ilv_emu", "plain")
    dtype, kahan, nsig, ld, mode, lanes = case
    args = [str(a) for a in (2 ** 12, 10, 128, 1793, 4, 16, 1, 1e-6, 900, dtype, kahan, mode, nsig, ld)]
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (args, r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert r.stdout.startswith("ILV OK") and r.stdout.rstrip().endswith(f"lanes {lanes}"), r.stdout


def test_emulated_recovery_sanitized(tmp_path):
    """The case whose first GPU run, with an earlier recovery kernel, faulted
    the GPU (complex128, (l, q) = (16, 1), N = 2^14, K = 50, delta = 1e-8,
    plan seed 102), through the current kernel body built with host
    AddressSanitizer and UndefinedBehaviorSanitizer on top of the guard
    pages: no access outside any array (private ones included) and no
    undefined behaviour, in both workgroup shapes and both guard modes, and
    the oracle's support and values."""
    N, K, B, w, M, l, q, delta, dt, ss, ps, loc, comb = CASES[0]
    x, sup, _ = make_signal(SignalSpec(N, K, ss))
    P = O.make_plan(N, K, B, w, M, l, q, delta, seed=ps)
    y = oracle_buckets(x, P)
    oidx, oval, _ = O.sfft(x, P)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:exitcode=97:detect_stack_use_after_return=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    for mode in (0, 1):
        gidx, gval = run_emulated(tmp_path, y, N, K, B, w, M, l, q, delta, ps, dt, mode, "sanitized", env=env)
        assert np.array_equal(gidx, oidx)
        assert np.linalg.norm(gval - oval) / np.linalg.norm(oval) <= 1e-10
