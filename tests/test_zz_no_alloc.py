"""ks_symv_noalloc (the symmetric product with its tile partials in the
library's fixed device array) against ks_symv with a caller workspace, through
the C ABI: two calls in a row, the second on a smaller, ragged system, each
equal bit for bit to ks_symv on the same input (same kernels), and each
within the componentwise rounding bound of the oracle's row sums."""
import ctypes

import numpy as np
import pytest

import oracle
from workloads import spd_problem

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _ws(n, device):
    import torch

    from paper_1511_07207_amd import _native as N

    sz = ctypes.c_size_t(0)
    assert N.lib().ks_symv_workspace_bytes(n, ctypes.byref(sz)) == 0
    return torch.empty(sz.value, dtype=torch.uint8, device=device), sz.value


def _run_both(n, lda, seed, device):
    import torch

    from paper_1511_07207_amd import _native as N

    L = N.lib()
    p = spd_problem(n, 1e3, seed=seed, config_id=0)
    Ah = np.full((n, lda), np.nan)
    Ah[:, :n] = np.tril(p.A)
    Ah[:, :n] += np.triu(np.full((n, n), np.nan), 1)  # above the diagonal: never read into y
    A = torch.from_numpy(Ah).to(device)
    xh = np.random.default_rng(seed).standard_normal(n)
    x = torch.from_numpy(xh).to(device)
    y_ref = torch.full((n,), np.nan, dtype=torch.float64, device=device)
    y = torch.full((n,), np.nan, dtype=torch.float64, device=device)
    ws, wsb = _ws(n, device)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.ks_symv(n, lda, A.data_ptr(), x.data_ptr(), y_ref.data_ptr(), ws.data_ptr(), wsb,
                     stream) == 0
    assert L.ks_symv_noalloc(n, lda, A.data_ptr(), x.data_ptr(), y.data_ptr(), stream) == 0
    torch.cuda.synchronize()
    yr, yn = y_ref.cpu().numpy(), y.cpu().numpy()
    assert np.array_equal(yr.view(np.int64), yn.view(np.int64))
    # against the oracle's row sums of the full symmetric matrix
    Af = np.tril(p.A) + np.tril(p.A, -1).T
    yo = oracle.matvec(Af, xh)
    bound = 2 * n * U * (np.abs(Af) @ np.abs(xh)) + 1e-300
    assert np.all(np.abs(yn - yo) <= bound)


@pytest.mark.parametrize("n1,n2", [(3000, 700), (1031, 257)])
def test_symv_noalloc_two_calls(device, n1, n2):
    print(f"ks_symv_noalloc n={n1} then n={n2}", flush=True)
    # leading dimensions padded past n, even (rows 16-byte aligned, as ks_symv requires)
    _run_both(n1, n1 + 6 + n1 % 2, 11, device)
    _run_both(n2, n2 + 2 + n2 % 2, 12, device)


def test_symv_noalloc_full_size_then_small(device):
    """The largest order the array holds, then a small one."""
    import torch

    from paper_1511_07207_amd import _native as N

    print("ks_symv_noalloc n=32768 then n=300", flush=True)
    n = 32768
    g = torch.Generator(device=device).manual_seed(3)
    A = torch.randn((n, n), dtype=torch.float64, device=device, generator=g)
    x = torch.randn(n, dtype=torch.float64, device=device, generator=g)
    y_ref = torch.full((n,), np.nan, dtype=torch.float64, device=device)
    y = torch.full((n,), np.nan, dtype=torch.float64, device=device)
    ws, wsb = _ws(n, device)
    L = N.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.ks_symv(n, n, A.data_ptr(), x.data_ptr(), y_ref.data_ptr(), ws.data_ptr(), wsb,
                     stream) == 0
    assert L.ks_symv_noalloc(n, n, A.data_ptr(), x.data_ptr(), y.data_ptr(), stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(y_ref.view(torch.int64), y.view(torch.int64))
    del ws, A
    torch.cuda.empty_cache()
    _run_both(300, 300, 13, device)


def test_symv_noalloc_rejects_beyond_maximum(device):
    from paper_1511_07207_amd import _native as N

    L = N.lib()
    # refused on the host before any device call (the pointers are never read)
    assert L.ks_symv_noalloc(32769, 32769, 16, 16, 16, None) == N.KS_ETOOLARGE
    assert L.ks_symv_noalloc(0, 1, 16, 16, 16, None) == N.KS_EINVAL
