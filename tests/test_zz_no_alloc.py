"""sfft_execute_noalloc (the entry point for callers that cannot allocate)
against sfft_execute, through the C ABI (needs an MI355X).

The two calls run the same kernels on the same plan, so their outputs must
be identical bit for bit; two calls in a row, the second on a smaller plan,
check that the shared static workspace carries nothing from one call into
the next.  A plan whose workspace exceeds the static array is refused
before anything is enqueued."""

from fractions import Fraction

import numpy as np
import pytest

from paper_2011_05698_amd.signals import SignalSpec, make_signal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 16 << 20


@pytest.fixture(scope="module")
def sf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_05698_amd import sfft
    return sfft


def _both(sf, plan, x, dtype):
    """Outputs of sfft_execute and of sfft_execute_noalloc on the same input."""
    vdt = torch.complex128 if dtype == "c128" else torch.complex64
    xd = torch.from_numpy(x.astype(np.complex128 if dtype == "c128" else np.complex64)).to("cuda")
    outs = []
    for fn in (sf.sfft_execute, sf.sfft_execute_noalloc):
        # poison the outputs so that entries a call leaves untouched compare equal only if both leave them
        idx = torch.full((plan.K,), -7, dtype=torch.int64, device="cuda")
        val = torch.full((plan.K,), 3.0 + 5.0j, dtype=vdt, device="cuda")
        cnt = torch.full((1,), -9, dtype=torch.int64, device="cuda")
        fn(plan.handle, xd, 1.0, idx, val, cnt)
        torch.cuda.synchronize()
        outs.append((idx.cpu().numpy(), val.cpu().numpy(), int(cnt.item())))
    return outs


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_matches_execute(sf, dtype):
    # a larger plan, then a smaller one: the second call must not see the first's workspace
    cases = [(2 ** 18, 300, 1024, 18433, 10, 21), (2 ** 12, 10, 128, 1537, 6, 7)]
    for N, K, B, w, M, ss in cases:
        plan = sf.Plan(N, K, B, w, M, 16, Fraction(1), delta=1e-6, seed=ss + 1, dtype=dtype)
        assert plan.workspace_bytes <= SCRATCH_BYTES
        x, sup, _ = make_signal(SignalSpec(N, K, ss))
        (ia, va, ca), (ib, vb, cb) = _both(sf, plan, x, dtype)
        assert ca == cb and ca == K
        assert np.array_equal(ia, ib)
        assert np.array_equal(va.view(np.uint8), vb.view(np.uint8))
        assert np.array_equal(np.sort(ia[:ca]), np.sort(sup))
        plan.close()


def test_noalloc_refuses_oversized_workspace(sf):
    # N = 2^24, B = 16384, 15 iterations: the bucket values alone exceed 16 MiB in complex128
    plan = sf.Plan(2 ** 24, 8192, 8192, (8192 * 24) | 1, 40, 16, Fraction(1), delta=1e-6, seed=5,
                   dtype="c128", b_min=8192)
    assert plan.workspace_bytes > SCRATCH_BYTES
    x = torch.zeros(2 ** 24, dtype=torch.complex128, device="cuda")
    idx = torch.zeros(plan.K, dtype=torch.int64, device="cuda")
    val = torch.zeros(plan.K, dtype=torch.complex128, device="cuda")
    cnt = torch.full((1,), -9, dtype=torch.int64, device="cuda")
    with pytest.raises(sf.SfftError) as e:
        sf.sfft_execute_noalloc(plan.handle, x, 1.0, idx, val, cnt)
    assert e.value.status == 5  # SFFT_ERR_CAPACITY
    torch.cuda.synchronize()
    assert int(cnt.item()) == -9  # nothing was enqueued
