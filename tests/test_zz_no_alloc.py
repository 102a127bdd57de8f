"""mtgp_fft_noalloc (the FFT entry point that allocates nothing and stages its
spectrum in a static device array) against mtgp_fft with a caller-supplied
scratch buffer: the same kernels, so the outputs must agree bit for bit.
Two calls in a row, the second on a smaller input, so a stale array would
show; then sizes beyond the static array are refused before any work."""
import ctypes

import pytest
import torch

from paper_2603_16014_amd import _lib

pytestmark = pytest.mark.gpu

F64, F32 = 0, 1


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _with_scratch(x, log2n, dtype, bitrev):
    lib = _lib.load()
    batch = x.numel() >> log2n
    X = torch.full((2 * x.numel(),), float("nan"), dtype=x.dtype, device="cuda")
    scratch = torch.empty(2 * x.numel(), dtype=x.dtype, device="cuda")
    _lib.check(lib.mtgp_fft(_ptr(x), _ptr(X), _ptr(scratch), batch, log2n, dtype, bitrev,
                            _stream()), "mtgp_fft")
    return X


def _noalloc(x, log2n, dtype, bitrev):
    lib = _lib.load()
    batch = x.numel() >> log2n
    X = torch.full((2 * x.numel(),), float("nan"), dtype=x.dtype, device="cuda")
    _lib.check(lib.mtgp_fft_noalloc(_ptr(x), _ptr(X), batch, log2n, dtype, bitrev, _stream()),
               "mtgp_fft_noalloc")
    return X


@pytest.mark.parametrize("dtype", [F64, F32])
def test_noalloc_fft_matches_scratch_fft_twice(dtype):
    tdt = torch.float64 if dtype == F64 else torch.float32
    g = torch.Generator(device="cpu").manual_seed(11)
    # (log2n, batch): a large multi-pass case filling most of the static
    # array, then a smaller multi-pass case, then a single-pass size
    cases = [(20, 2 if dtype == F64 else 4), (15, 3), (9, 5)]
    for bitrev in (0, 1):
        for log2n, batch in cases:
            print(f"noalloc fft: dtype {dtype} bitrev {bitrev} log2n {log2n} batch {batch}",
                  flush=True)
            x = torch.randn(batch << log2n, generator=g, dtype=torch.float64).to(tdt).cuda()
            want = _with_scratch(x, log2n, dtype, bitrev)
            got = _noalloc(x, log2n, dtype, bitrev)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (dtype, bitrev, log2n, batch)
            assert torch.isfinite(got).all()


def test_noalloc_fft_refuses_inputs_beyond_its_scratch():
    lib = _lib.load()
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    cap = 33554432
    # 2^21 complex doubles fill the array exactly; one more row does not fit
    assert (1 << 21) * 16 == cap
    rc = lib.mtgp_fft_noalloc(_ptr(x), _ptr(x), 2, 21, F64, 0, _stream())
    assert rc == -6
    rc = lib.mtgp_fft_noalloc(_ptr(x), _ptr(x), 1, 23, F32, 0, _stream())
    assert rc == -6
    assert b"static scratch" in lib.mtgp_strerror(-6)
    # batch 0 does nothing
    assert lib.mtgp_fft_noalloc(None, None, 0, 20, F64, 0, _stream()) == 0
    torch.cuda.synchronize()


def test_noalloc_fft_at_capacity():
    """batch * n complex doubles exactly filling the static array."""
    g = torch.Generator(device="cpu").manual_seed(12)
    x = torch.randn(1 << 21, generator=g, dtype=torch.float64).cuda()
    want = _with_scratch(x, 21, F64, 0)
    got = _noalloc(x, 21, F64, 0)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
