"""Kernel-level parity on the GPU: GEMV (all storage types), conversions,
read ceiling.  References: the CPU oracle's matrix-vector product in binary64,
and a numpy statement of the rounding rule."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

RAGGED = [1, 2, 63, 64, 65, 257, 1000, 4097]


def _torch():
    import torch

    return torch


def bf16_rne_bits(a64: np.ndarray) -> np.ndarray:
    """binary64 -> binary32 (nearest even) -> bfloat16 (nearest even), as bits."""
    f = a64.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    r = np.where(nan, ((u >> 16) | 0x40) & 0xFFFF, r)
    return r.astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("n", RAGGED)
@pytest.mark.parametrize("pad", [0, 6])
def test_gemv_fp64(device, n, pad):
    torch = _torch()
    from paper_1511_07207_amd import krylov

    print(f"gemv fp64 n={n} pad={pad}", flush=True)
    rng = np.random.default_rng(n + pad)
    lda = n + pad
    lda += lda % 2  # 16-byte rows
    Ah = rng.standard_normal((n, lda))
    v = rng.standard_normal(n)
    A = torch.from_numpy(Ah).to(device)
    y = krylov.gemv(A, torch.from_numpy(v).to(device), n=n, lda=lda)
    torch.cuda.synchronize()
    ref = oracle.matvec(np.ascontiguousarray(Ah[:, :n]), v)
    bound = 2 * n * 2.0 ** -53 * (np.abs(Ah[:, :n]) @ np.abs(v)) + 1e-300
    assert np.all(np.abs(y.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("n", RAGGED)
def test_gemv_fp32_and_bf16(device, n):
    torch = _torch()
    from paper_1511_07207_amd import krylov

    print(f"gemv fp32/bf16 n={n}", flush=True)
    rng = np.random.default_rng(100 + n)
    Ah = rng.standard_normal((n, n))
    A = torch.from_numpy(Ah).to(device)
    lda = ((n + 7) // 8) * 8
    v32 = rng.standard_normal(n).astype(np.float32)
    vt = torch.from_numpy(v32).to(device)
    for dtype in (torch.float32, torch.bfloat16):
        Al = krylov.convert(A, dtype, lda_dst=lda)
        y = krylov.gemv(Al, vt, n=n, lda=lda)
        torch.cuda.synchronize()
        if dtype == torch.float32:
            Aref = Al.cpu().numpy()[:, :n].astype(np.float64)
            assert np.array_equal(Aref, Ah.astype(np.float32).astype(np.float64))
        else:
            bits = Al.view(torch.int16).cpu().numpy().view(np.uint16)[:, :n]
            assert np.array_equal(bits, bf16_rne_bits(Ah))
            Aref = bf16_bits_to_f64(bits)
        ref = oracle.matvec(np.ascontiguousarray(Aref), v32.astype(np.float64))
        bound = 2 * n * 2.0 ** -24 * (np.abs(Aref) @ np.abs(v32.astype(np.float64))) + 1e-30
        assert np.all(np.abs(y.cpu().numpy().astype(np.float64) - ref) <= bound), dtype


def test_convert_special_values(device):
    torch = _torch()
    from paper_1511_07207_amd import krylov

    vals = np.array([0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9,
                     3.0e38, -3.4e38, 1e-40, np.inf, -np.inf, np.nan, 65504.0, 2.0 ** -133,
                     1.0 + 2.0 ** -24, 1.0 + 2.0 ** -24 + 2.0 ** -40])
    n = 4
    Ah = np.zeros((n, n))
    Ah.flat[: vals.size] = vals
    A = torch.from_numpy(Ah).to(device)
    Ab = krylov.convert(A, torch.bfloat16)
    Af = krylov.convert(A, torch.float32)
    torch.cuda.synchronize()
    bits = Ab.view(torch.int16).cpu().numpy().view(np.uint16)
    assert np.array_equal(bits, bf16_rne_bits(Ah))
    f = Af.cpu().numpy()
    assert np.array_equal(f.view(np.uint32), Ah.astype(np.float32).view(np.uint32))


def test_gemv_deterministic(device):
    torch = _torch()
    from paper_1511_07207_amd import krylov

    rng = np.random.default_rng(7)
    n = 3000
    A = torch.from_numpy(rng.standard_normal((n, n))).to(device)
    v = torch.from_numpy(rng.standard_normal(n)).to(device)
    y1 = krylov.gemv(A, v).clone()
    y2 = krylov.gemv(A, v)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


def test_read_ceiling_runs(device):
    torch = _torch()
    from paper_1511_07207_amd import krylov

    buf = torch.ones(1 << 22, dtype=torch.float32, device=device)
    sink = torch.zeros(1, dtype=torch.float64, device=device)
    krylov.read_ceiling(buf, sink)
    torch.cuda.synchronize()
    assert sink.item() == 0.0
