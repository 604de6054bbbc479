"""2D DCT-II / DCT-III (fft2_plan_dct / fft2_exec_dct) against the FP64
oracle's dct2 / idct2, through the C ABI.  Bars: relative L2 <= 2e-6 (FP32
butterflies), <= 5e-6 (split BF16)."""
import numpy as np
import pytest

import oracle
from paper_1505_08019_amd import fft2 as F
from paper_1505_08019_amd import inputs
from paper_1505_08019_amd.metrics import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _real(kind, rows, cols, index=0):
    return np.ascontiguousarray(inputs.image(kind, rows, cols, cfg_seed=4, index=index).real, dtype=np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


SHAPES = [(1, 2), (2, 2), (1, 16), (16, 1 * 2), (4, 8), (8, 4), (16, 16), (64, 64), (32, 256), (256, 32),
          (512, 512), (1024, 1024), (2048, 1024)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
@pytest.mark.parametrize("kind", ["uniform", "smooth"])
def test_dct2_matches_oracle(shape, kind):
    x = _real(kind, *shape, index=shape[0] + 3 * shape[1])
    want = oracle.dct2(x)
    with F.DctPlan(*shape) as p:
        got = p.exec(_dev(x))
        torch.cuda.synchronize()
    assert rel_l2(got.cpu().numpy(), want) <= 2e-6


@pytest.mark.parametrize("shape", [(1, 2), (2, 4), (16, 16), (64, 128), (1024, 512)], ids=lambda s: "%dx%d" % s)
def test_idct2_matches_oracle(shape):
    X = oracle.dct2(_real("smooth", *shape, index=9)).astype(np.float32)
    want = oracle.idct2(X)
    with F.DctPlan(*shape, direction=F.INVERSE) as p:
        got = p.exec(_dev(X))
        torch.cuda.synchronize()
    assert rel_l2(got.cpu().numpy(), want) <= 2e-6


@pytest.mark.parametrize("shape", [(8, 8), (256, 256), (2048, 2048)], ids=lambda s: "%dx%d" % s)
def test_dct_round_trip(shape):
    x = _real("uniform", *shape)
    xd = _dev(x)
    with F.DctPlan(*shape) as pf, F.DctPlan(*shape, direction=F.INVERSE) as pi:
        y = pi.exec(pf.exec(xd))
        torch.cuda.synchronize()
    assert rel_l2(y.cpu().numpy(), x) <= 2e-6


def test_dct_closed_forms_and_split():
    """A constant image gives 4 M N c at (0, 0) only; the split-BF16 form is
    within its 5e-6 bar."""
    M, N = 128, 256
    with F.DctPlan(M, N) as p:
        X = p.exec(torch.full((M, N), 5.0, device="cuda:0")).cpu().numpy()
    want = np.zeros((M, N))
    want[0, 0] = 4 * M * N * 5.0
    assert np.abs(X - want).max() <= 2e-6 * want[0, 0]
    x = _real("smooth", 1024, 1024, index=2)
    with F.DctPlan(1024, 1024, precision=F.PREC_SPLIT_BF16) as p:
        got = p.exec(_dev(x)).cpu().numpy()
    assert rel_l2(got, oracle.dct2(x)) <= 5e-6


def test_dct_errors():
    L = F.lib()
    assert L.fft2_plan_dct(8, 1, F.FORWARD, F.PREC_FP32) is None
    assert F.last_error()[0] == F.ERR_INVALID_SIZE
    x = torch.zeros((64, 64), dtype=torch.float32, device="cuda:0")
    y = torch.zeros((64, 64), dtype=torch.float32, device="cuda:0")
    s = torch.cuda.current_stream().cuda_stream
    with F.DctPlan(64, 64) as p:
        assert L.fft2_exec_dct(p.handle, x.data_ptr() + 4, y.data_ptr(), s) == F.ERR_ALIGNMENT
        assert L.fft2_exec_dct(p.handle, x.data_ptr(), x.data_ptr() + 8, s) == F.ERR_ALIAS
        assert L.fft2_exec_dct(None, x.data_ptr(), y.data_ptr(), s) == F.ERR_INVALID_VALUE
    torch.cuda.synchronize()
