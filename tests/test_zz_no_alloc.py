"""fft2_exec_noalloc (the entry point for callers that cannot allocate)
against fft2_exec, through the C ABI: bit-identical results on two calls in
a row, the second with a smaller image, in place (where the static scratch
image is used) and out of place, FP32 and split BF16; images above
FFT2_NOALLOC_MAX_POINTS are rejected."""
import numpy as np
import pytest

from paper_1505_08019_amd import fft2 as F
from paper_1505_08019_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to("cuda:0")


def _noalloc(p, x, out, stream):
    return F.lib().fft2_exec_noalloc(p.handle, x.data_ptr(), out.data_ptr(), stream.cuda_stream)


def _exec(p, x, out, stream):
    return F.lib().fft2_exec(p.handle, x.data_ptr(), out.data_ptr(), stream.cuda_stream)


@pytest.mark.parametrize("precision", [F.PREC_FP32, F.PREC_SPLIT_BF16], ids=["fp32", "split_bf16"])
@pytest.mark.parametrize("direction", [F.FORWARD, F.INVERSE], ids=["forward", "inverse"])
def test_noalloc_matches_exec_two_calls(precision, direction):
    s = torch.cuda.current_stream()
    # the largest accepted image first, then a smaller one of another shape:
    # the second call's result must not depend on what the first left behind
    for k, (M, N) in enumerate([(2048, 2048), (512, 1024)]):
        x = _dev(inputs.smooth_image(M, N, cfg_seed=5, index=k))
        with F.Plan(M, N, direction, precision) as p:
            want = torch.empty_like(x)
            assert _exec(p, x, want, s) == F.SUCCESS
            got = torch.full_like(x, float("nan"))
            assert _noalloc(p, x, got, s) == F.SUCCESS  # out of place
            y = x.clone()
            assert _noalloc(p, y, y, s) == F.SUCCESS    # in place: the static scratch image
            want_ip = x.clone()
            assert _exec(p, want_ip, want_ip, s) == F.SUCCESS
            torch.cuda.synchronize()
            assert torch.equal(got, want), (M, N)
            assert torch.equal(y, want_ip), (M, N)
            assert torch.equal(y, want), (M, N)


def test_noalloc_rejects_large_images():
    M, N = 4096, 2048  # 2^23 values > FFT2_NOALLOC_MAX_POINTS
    assert M * N > F.NOALLOC_MAX_POINTS
    x = torch.zeros((M, N), dtype=torch.complex64, device="cuda:0")
    with F.Plan(M, N) as p:
        s = torch.cuda.current_stream()
        assert _noalloc(p, x, x, s) == F.ERR_INVALID_SIZE
        assert "at most" in F.last_error()[1]
    assert F.lib().fft2_exec_noalloc(None, x.data_ptr(), x.data_ptr(), s.cuda_stream) == F.ERR_INVALID_VALUE
    torch.cuda.synchronize()
