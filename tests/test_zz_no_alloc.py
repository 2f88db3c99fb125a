"""The allocation-free compaction (sdc_select_noalloc) against the
context's sdc_select, through the C ABI: bit-exact index lists and counts on
two calls in a row (the second with a smaller input, so the shared scratch
holds the first call's values), plus the empty input, theta <= 0, an entry
outside amax (count -1, output untouched) and the size limit (rejected on the
host before anything is enqueued)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from workloads import config1  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(rng, N, n, theta):
    """An ascending random list of n rows and correction maxima with ties at
    theta, NaNs and values on both sides."""
    idx = np.sort(rng.choice(N, n, replace=False)).astype(np.int32)
    amax = rng.uniform(0.0, 2.0 * theta, N)
    amax[rng.choice(N, N // 10, replace=False)] = theta   # ties: kept
    amax[rng.choice(N, N // 50, replace=False)] = np.nan  # dropped
    return idx, amax


def test_noalloc_select_matches_context_select():
    from paper_2311_07206_amd import Solver, select_noalloc
    P = config1(n=96, theta=1e-7)
    s = Solver.from_problem(P)
    rng = np.random.default_rng(41)
    # two calls in a row, the second smaller; several blocks and a ragged tail each
    for n, theta in ((7000, 1e-7), (1500, 3e-7)):
        idx, amax = _case(rng, P.N, n, theta)
        print(f"[no-alloc select] n_in={n} theta={theta}", flush=True)
        a = torch.tensor(amax, device=DEV)
        i = torch.tensor(idx, device=DEV)
        want = s.select(a, i, theta).cpu().numpy()
        out = torch.full((n,), -7, dtype=torch.int32, device=DEV)
        cnt = torch.full((1,), -9, dtype=torch.int64, device=DEV)
        select_noalloc(a, i, theta, out, cnt)
        torch.cuda.synchronize()
        k = int(cnt.item())
        assert k == want.size and 0 < k < n
        assert np.array_equal(out[:k].cpu().numpy(), want)
        assert np.all(out[k:].cpu().numpy() == -7)
        host = idx[(amax[idx] >= theta)]
        assert np.array_equal(want, host)
    # theta <= 0 keeps every entry (NaN included)
    out = torch.zeros(idx.size, dtype=torch.int32, device=DEV)
    select_noalloc(a, i, 0.0, out, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == idx.size and np.array_equal(out.cpu().numpy(), idx)
    # an empty list
    select_noalloc(a, i[:0], theta, out, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    s.close()


def test_noalloc_select_flags_entries_outside_amax_and_rejects_large_sizes():
    from paper_2311_07206_amd import _lib, select_noalloc
    a = torch.ones(1000, dtype=torch.float64, device=DEV)
    i = torch.tensor(np.r_[np.arange(600), 1000, np.arange(601, 700)].astype(np.int32), device=DEV)
    out = torch.full((i.numel(),), -3, dtype=torch.int32, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    select_noalloc(a, i, 0.5, out, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == -1 and np.all(out.cpu().numpy() == -3)
    lib = _lib.load()
    st = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    p = ctypes.c_void_p
    rc = lib.sdc_select_noalloc(0, st, p(a.data_ptr()), a.numel(), p(i.data_ptr()), _lib.NOALLOC_MAX_IN + 1, 0.5,
                                p(out.data_ptr()), p(cnt.data_ptr()))
    assert rc == -1
    rc = lib.sdc_select_noalloc(0, st, p(a.data_ptr()), a.numel(), p(i.data_ptr()), -1, 0.5, p(out.data_ptr()),
                                p(cnt.data_ptr()))
    assert rc == -1
    rc = lib.sdc_select_noalloc(0, st, p(a.data_ptr()), a.numel(), p(i.data_ptr()), 10, 0.5, None, p(cnt.data_ptr()))
    assert rc == -1
    with pytest.raises(ValueError):
        select_noalloc(a, i, 0.5, out[:10], cnt)
