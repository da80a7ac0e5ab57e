"""The allocation-free LU entry point (nlf_getrf_batched_noalloc) against the allocating one
(nlf_getrf_batched): the same factors, pivots, permutations and info flags, bit for bit, on
two calls in a row with the second one smaller (the fixed scratch keeps the first call's
contents), in both precisions; the pivots also against the oracle's LU; and a size beyond
the fixed scratch refused on the host."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1801_09794_amd as nl  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    nl.lib()
    yield
    torch.cuda.synchronize()


def factor(fn, mats, dt):
    batch, n = len(mats), mats[0].shape[0]
    A = torch.stack([nl.to_colmajor(M, "cuda", dt) for M in mats])
    ipiv = torch.full((batch, n), -7, dtype=torch.int32, device="cuda")
    perm = torch.full((batch, n), -7, dtype=torch.int32, device="cuda")
    info = torch.full((batch,), -7, dtype=torch.int32, device="cuda")
    fn(A, ipiv, perm, info)
    torch.cuda.synchronize()
    return A, ipiv, perm, info


@pytest.mark.parametrize("dt", [torch.complex128, torch.complex64])
def test_noalloc_equals_allocating_entry_point(dt):
    rng = np.random.default_rng(2024)
    for n, batch in [(1000, 6), (520, 3)]:         # the second call is smaller
        mats = [wl.cn(rng, (n, n)) for _ in range(batch)]
        print("noalloc case: dtype %s n %d batch %d" % (dt, n, batch), flush=True)
        got = factor(nl.nlf_getrf_batched_noalloc, mats, dt)
        want = factor(nl.nlf_getrf_batched, mats, dt)
        for g, w in zip(got, want):
            assert torch.equal(g, w)
        assert np.all(got[3].cpu().numpy() == 0)
        if dt == torch.complex128:
            _, piv0 = dense.lu_partial_pivot(mats[0])
            assert np.array_equal(got[1][0].cpu().numpy(), piv0)
    # a third, tiny call with an exact zero pivot at column 17 of the first matrix
    A = np.eye(40, dtype=complex)
    A[:, 17] = 0.0
    got = factor(nl.nlf_getrf_batched_noalloc, [A, np.eye(40, dtype=complex)], dt)
    want = factor(nl.nlf_getrf_batched, [A, np.eye(40, dtype=complex)], dt)
    assert got[3].cpu().numpy().tolist() == want[3].cpu().numpy().tolist() == [18, 0]
    assert torch.equal(got[1], want[1]) and torch.equal(got[2], want[2])


def test_noalloc_refuses_more_than_its_scratch():
    n = 8192
    batch = nl.NLF_NOALLOC_SCRATCH_INTS // (4 * n) + 1      # 33 matrices of 8192: one too many
    small = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = nl.lib().nlf_getrf_batched_noalloc(nl.NLF_C128, n, batch, small.data_ptr(), n, n * n,
                                            small.data_ptr(), small.data_ptr(), small.data_ptr(), None)
    assert st == nl.NLF_ERR_ARG
    assert b"exceed the fixed scratch" in nl.lib().nlfeast_last_error(None)
