"""Parity of the FP32 HIP path with the FP64 oracle, through the C ABI.

Bar: relative L2 error <= 2e-6 against the oracle; integer work (the
bit-reversal scramble) and the exact closed forms (delta, constant) bit-exact.
"""
import numpy as np
import pytest

import oracle
from paper_1505_08019_amd import fft2 as F
from paper_1505_08019_amd import inputs
from paper_1505_08019_amd.metrics import rel_l2
from tests import _bruteforce

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 2e-6


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to("cuda:0")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rev_np(n, bits):
    i = np.arange(n, dtype=np.int64)
    r = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        r |= ((i >> b) & 1) << (bits - 1 - b)
    return r


def _gpu_fft(x, direction=F.FORWARD):
    rows, cols = x.shape
    with F.Plan(rows, cols, direction) as p:
        return _host(p.exec(_dev(x)))


SHAPES = [(1, 1), (1, 2), (2, 1), (2, 2), (4, 8), (8, 4), (16, 16), (1, 1024), (1024, 1), (64, 64),
          (32, 128), (128, 32), (8, 512), (256, 256), (512, 512), (128, 1024), (1024, 128),
          (1024, 1024), (2048, 512), (512, 2048), (4096, 64), (64, 4096), (16384, 16), (16, 16384),
          (2, 16384), (16384, 2), (1, 16384), (16384, 1), (2048, 2048)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
def test_forward_matches_oracle(shape):
    x = inputs.uniform_pixels(*shape, cfg_seed=1, index=shape[0] * 7 + shape[1])
    want = oracle.fft2(x, threads=0)
    got = _gpu_fft(x)
    assert rel_l2(got, want) <= TOL, F.describe_schedule(*shape)


@pytest.mark.parametrize("shape", [(1, 1), (2, 2), (16, 64), (256, 256), (1024, 1024), (64, 4096), (4096, 64)],
                         ids=lambda s: "%dx%d" % s)
def test_inverse_matches_oracle(shape):
    g = np.random.default_rng(shape[0] + 3 * shape[1])
    x = (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)
    want = oracle.fft2(x, +1, threads=0)
    got = _gpu_fft(x, F.INVERSE)
    assert rel_l2(got, want) <= TOL


def test_bruteforce_8x8_crop():
    """Config 1: top-left 8x8 crop of the seeded 256x256 image vs eq. (1) term by term."""
    crop = inputs.uniform_pixels(256, 256, cfg_seed=1)[:8, :8]
    want = np.array(_bruteforce.dft2(crop.astype(np.complex128).tolist()))
    assert rel_l2(_gpu_fft(crop), want) <= TOL


def test_config1_256():
    x = inputs.uniform_pixels(256, 256, cfg_seed=1)
    assert rel_l2(_gpu_fft(x), oracle.fft2(x)) <= TOL


@pytest.mark.parametrize("kind", ["uniform", "smooth"])
def test_config2_1024_round_trip(kind):
    """Config 2: 1024x1024 forward then inverse, both pixel distributions."""
    x = inputs.image(kind, 1024, 1024, cfg_seed=2)
    want = oracle.fft2(x, threads=0)
    with F.Plan(1024, 1024, F.FORWARD) as pf, F.Plan(1024, 1024, F.INVERSE) as pi:
        X = pf.exec(_dev(x))
        y = pi.exec(X)
        Xh, yh = _host(X), _host(y)
    assert rel_l2(Xh, want) <= TOL
    assert rel_l2(yh, x) <= TOL


@pytest.mark.parametrize("shape", [(1, 1), (4, 8), (64, 32), (256, 256), (1024, 1024), (8192, 8192)],
                         ids=lambda s: "%dx%d" % s)
def test_delta_exact(shape):
    x = torch.zeros(shape, dtype=torch.complex64, device="cuda:0")
    x[0, 0] = 1
    with F.Plan(*shape) as p:
        X = p.exec(x)
    torch.cuda.synchronize()
    assert torch.equal(X, torch.ones(shape, dtype=torch.complex64, device="cuda:0"))


@pytest.mark.parametrize("shape", [(1, 1), (2, 16), (64, 32), (1024, 1024), (4096, 4096)],
                         ids=lambda s: "%dx%d" % s)
def test_constant_exact(shape):
    c = 173.0
    x = torch.full(shape, c, dtype=torch.complex64, device="cuda:0")
    with F.Plan(*shape) as p:
        X = p.exec(x)
    want = torch.zeros(shape, dtype=torch.complex64, device="cuda:0")
    want[0, 0] = c * shape[0] * shape[1]
    torch.cuda.synchronize()
    assert torch.equal(X, want)


@pytest.mark.parametrize("shape", [(8, 8), (2, 16384), (64, 64), (256, 512), (1024, 1024), (16384, 16),
                                   (8192, 8192), (8192, 16384)], ids=lambda s: "%dx%d" % s)
def test_scramble_bit_exact(shape):
    """Stage (0, 0): out[r, c] = rev(r) + i rev(c) for x[r, c] = r + i c (sec. 3.2)."""
    M, N = shape
    bm, bn = M.bit_length() - 1, N.bit_length() - 1
    r = torch.arange(M, device="cuda:0", dtype=torch.float32)[:, None].expand(M, N)
    c = torch.arange(N, device="cuda:0", dtype=torch.float32)[None, :].expand(M, N)
    x = torch.complex(r, c).contiguous()
    rr = torch.from_numpy(_rev_np(M, bm).astype(np.float32)).to("cuda:0")[:, None].expand(M, N)
    cc = torch.from_numpy(_rev_np(N, bn).astype(np.float32)).to("cuda:0")[None, :].expand(M, N)
    want = torch.complex(rr, cc)
    with F.Plan(M, N) as p:
        got = p.exec_partial(x, 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(got, want)


@pytest.mark.parametrize("shape", [(64, 64), (256, 512), (1024, 1024), (32, 2048)], ids=lambda s: "%dx%d" % s)
def test_stage_snapshots(shape):
    """Each (row_stages, col_stages) snapshot against the oracle's snapshot."""
    M, N = shape
    bm, bn = M.bit_length() - 1, N.bit_length() - 1
    x = inputs.uniform_pixels(M, N, cfg_seed=3)
    xd = _dev(x)
    cases = sorted({(s, t) for s in (0, 1, 2, bn // 2, bn - 1, bn) for t in (0, 1, 2, 3, bm // 2, bm)
                    if 0 <= s <= bn and 0 <= t <= bm and (t == 0 or s == bn)})
    with F.Plan(M, N) as p:
        for s, t in cases:
            got = _host(p.exec_partial(xd, s, t))
            want = oracle.fft2(x, row_stages=s, col_stages=t)
            assert rel_l2(got, want) <= TOL, (s, t)


def test_in_place_equals_out_of_place():
    x = inputs.smooth_image(512, 1024, cfg_seed=2)
    with F.Plan(512, 1024) as p:
        a = p.exec(_dev(x))
        b = _dev(x)
        p.exec(b, out=b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_deterministic():
    x = _dev(inputs.uniform_pixels(2048, 2048, cfg_seed=2))
    with F.Plan(2048, 2048) as p:
        a = p.exec(x)
        b = p.exec(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_side_stream_and_concurrent_plan_use():
    x = _dev(inputs.uniform_pixels(1024, 1024, cfg_seed=2))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with F.Plan(1024, 1024) as p:
        out1 = torch.empty_like(x)
        out2 = torch.empty_like(x)
        p.exec(x, out1, stream=s1)
        p.exec(x, out2, stream=s2)
        ref = p.exec(x)
    torch.cuda.synchronize()
    assert torch.equal(out1, ref) and torch.equal(out2, ref)


def test_error_codes():
    x = torch.zeros((64, 64), dtype=torch.complex64, device="cuda:0")
    y = torch.zeros((64, 64), dtype=torch.complex64, device="cuda:0")
    with F.Plan(64, 64) as p:
        h = p.handle
        s = torch.cuda.current_stream().cuda_stream
        L = F.lib()
        assert L.fft2_exec(h, x.data_ptr() + 4, y.data_ptr(), s) == F.ERR_ALIGNMENT
        assert L.fft2_exec(h, x.data_ptr(), x.data_ptr() + 8, s) == F.ERR_ALIAS
        assert L.fft2_exec(h, 0, y.data_ptr(), s) == F.ERR_INVALID_VALUE
        assert L.fft2_exec(None, x.data_ptr(), y.data_ptr(), s) == F.ERR_INVALID_VALUE
    assert F.lib().fft2_plan(3, 64, -1, 0) is None
    assert F.last_error()[0] == F.ERR_INVALID_SIZE
    torch.cuda.synchronize()


def _sampled_check(x, X, n_cols=3, seed=0):
    """Sampled outputs of a large image against the plain double sum.

    Returns (rms, dc): the RMS error over random bins of n_cols random output
    columns divided by the RMS of all outputs (||x|| by Parseval), which
    estimates the whole output's relative L2 error without the DC bin's
    weight; and the relative L2 error over the k2 = 0 column, where the large
    partial sums of the pixel mean meet, against its own values."""
    M, N = x.shape
    g = np.random.default_rng(seed)
    k2 = np.repeat(g.integers(1, N, size=n_cols), 256)
    k1 = g.integers(0, M, size=k2.size)
    err = X[k1, k2] - oracle.dft2_at(x, k1, k2)
    rms = np.sqrt(np.mean(np.abs(err) ** 2)) / np.linalg.norm(x.astype(np.complex128))
    d1 = np.concatenate([[0], g.integers(1, M, size=255)])
    d2 = np.zeros_like(d1)
    dc = rel_l2(X[d1, d2], oracle.dft2_at(x, d1, d2))
    return rms, dc


@pytest.mark.parametrize("n", [4096, 8192])
@pytest.mark.parametrize("kind", ["uniform", "smooth"])
def test_config3_large_full(n, kind):
    """Config 3 at full size, every output bin against the full FP64 oracle,
    plus the forward/inverse round trip and Parseval."""
    x = inputs.image(kind, n, n, cfg_seed=3)
    xd = _dev(x)
    with F.Plan(n, n, F.FORWARD) as pf, F.Plan(n, n, F.INVERSE) as pi:
        X = pf.exec(xd)
        y = pi.exec(X)
        torch.cuda.synchronize()
        e_rt = (torch.linalg.vector_norm((y - xd).to(torch.complex128)) /
                torch.linalg.vector_norm(xd.to(torch.complex128))).item()
        ex = torch.sum(torch.abs(xd.to(torch.complex128)) ** 2).item() * n * n
        eX = torch.sum(torch.abs(X.to(torch.complex128)) ** 2).item()
        Xh = X.cpu().numpy()
        del X, y, xd
    want = oracle.fft2(x, threads=0)
    err = rel_l2(Xh, want)
    print("fp32 %dx%d %s: rel_l2 %.3e, round trip %.3e" % (n, n, kind, err, e_rt), flush=True)
    assert err <= TOL
    assert e_rt <= TOL
    assert abs(ex - eX) / eX <= 1e-5
    # the sampled checker agrees with the full comparison
    rms, dc = _sampled_check(x, Xh, n_cols=2)
    assert rms <= TOL and dc <= TOL


def test_three_pass_full():
    """8192 x 16384 needs three passes; every output bin against the full
    FP64 oracle."""
    M, N = 8192, 16384
    assert len(F.describe_schedule(M, N).split()) == 3
    x = inputs.uniform_pixels(M, N, cfg_seed=3)
    with F.Plan(M, N) as p:
        Xh = _host(p.exec(_dev(x)))
    err = rel_l2(Xh, oracle.fft2(x, threads=0))
    print("fp32 %dx%d uniform: rel_l2 %.3e" % (M, N, err), flush=True)
    assert err <= TOL


def test_odd_element_offset_views():
    """Buffers need only 8-byte alignment: images that start at an odd
    complex64 element (8 mod 16 bytes) give the same bits as aligned ones,
    out of place, in place, and through the filter request."""
    for (M, N) in [(64, 64), (1024, 1024), (512, 2048), (4096, 4096)]:
        x = _dev(inputs.uniform_pixels(M, N, cfg_seed=2))
        buf_in = torch.zeros(M * N + 1, dtype=torch.complex64, device="cuda:0")
        buf_out = torch.zeros(M * N + 1, dtype=torch.complex64, device="cuda:0")
        xi = buf_in[1:].view(M, N)
        xo = buf_out[1:].view(M, N)
        assert xi.data_ptr() % 16 == 8 and xo.data_ptr() % 16 == 8
        xi.copy_(x)
        with F.Plan(M, N) as p:
            want = p.exec(x)
            p.exec(xi, xo)
            torch.cuda.synchronize()
            assert torch.equal(xo, want), (M, N)
            assert buf_out[0].item() == 0  # nothing written before the view
            p.exec(xi, out=xi)
            torch.cuda.synchronize()
            assert torch.equal(xi, want), (M, N)
            xi.copy_(x)
            fw = p.exec_filter(x, 0.2)
            p.exec_filter(xi, 0.2, out=xo)
            torch.cuda.synchronize()
            assert torch.equal(xo, fw), (M, N)
    L = F.lib()
    h = torch.zeros(64, 64, dtype=torch.complex64, device="cuda:0")
    with F.Plan(8, 8) as p:
        s = torch.cuda.current_stream().cuda_stream
        assert L.fft2_exec(p.handle, h.data_ptr() + 4, h.data_ptr() + 4096, s) == F.ERR_ALIGNMENT
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1024, 4096, 8192])
def test_in_place_large(n):
    """In-place calls stage the row pass through scratch: no cross-workgroup race."""
    x = _dev(inputs.uniform_pixels(n, n, cfg_seed=2))
    with F.Plan(n, n) as p:
        a = p.exec(x)
        b = x.clone()
        p.exec(b, out=b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_exec_pass_sequence_equals_exec():
    x = _dev(inputs.uniform_pixels(1024, 2048, cfg_seed=2))
    with F.Plan(1024, 2048) as p:
        want = p.exec(x)
        out = torch.empty_like(x)
        for i in range(p.info()[0]):
            p.exec_pass(i, x, out)
        torch.cuda.synchronize()
        assert torch.equal(out, want)


def test_largest_size_16384():
    """The largest accepted size, 16384 x 16384 (2 GiB per image, three
    passes): a delta at the origin gives all ones exactly, and sampled
    columns of a uniform-pixel image match the plain sum."""
    n = 16384
    with F.Plan(n, n) as p:
        d = torch.zeros((n, n), dtype=torch.complex64, device="cuda:0")
        d[0, 0] = 1.0
        X = p.exec(d)
        torch.cuda.synchronize()
        assert bool(torch.all(X == 1.0).item())
        del d, X
        x = inputs.uniform_pixels(n, n, cfg_seed=3)
        Xh = _host(p.exec(_dev(x)))
    g = np.random.default_rng(1)
    # Uniformly drawn outputs (four random columns): their RMS error against
    # the RMS of all outputs, which Parseval gives as ||x||, estimates the
    # whole output's relative L2 error.
    k2 = np.repeat(g.integers(0, n, size=4), 256)
    k1 = g.integers(0, n, size=k2.size)
    err = Xh[k1, k2] - oracle.dft2_at(x, k1, k2)
    assert np.sqrt(np.mean(np.abs(err) ** 2)) / np.linalg.norm(x.astype(np.complex128)) <= TOL
    # The DC column, where the large partial sums of the pixel mean meet,
    # against its own values (DC included).
    k1 = np.concatenate([[0], g.integers(1, n, size=1023)])
    k2 = np.zeros_like(k1)
    assert rel_l2(Xh[k1, k2], oracle.dft2_at(x, k1, k2)) <= TOL


def test_stream_capture():
    """Under HIP stream capture the out-of-place transform records kernel nodes
    only (its graph replays equal the eager result, with eager work between
    replays); calls that would take a stream-ordered scratch image (in place,
    the MFMA-form filter without a workspace, real transforms) refuse with
    FFT2_ERR_UNSUPPORTED instead of recording an allocation."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    vp = ctypes.c_void_p
    hip.hipStreamCreate.argtypes = [ctypes.POINTER(vp)]
    hip.hipStreamBeginCapture.argtypes = [vp, ctypes.c_int]
    hip.hipStreamEndCapture.argtypes = [vp, ctypes.POINTER(vp)]
    hip.hipGraphInstantiate.argtypes = [ctypes.POINTER(vp), vp, vp, vp, ctypes.c_size_t]
    hip.hipGraphLaunch.argtypes = [vp, vp]
    hip.hipStreamSynchronize.argtypes = [vp]
    hip.hipGraphExecDestroy.argtypes = [vp]
    hip.hipGraphDestroy.argtypes = [vp]
    hip.hipStreamDestroy.argtypes = [vp]
    relaxed = 2  # hipStreamCaptureModeRelaxed
    x = _dev(inputs.uniform_pixels(1024, 1024, cfg_seed=2))
    y = torch.zeros_like(x)
    xs = x.clone()
    st = vp()
    assert hip.hipStreamCreate(ctypes.byref(st)) == 0
    torch.cuda.synchronize()
    L = F.lib()
    with F.Plan(1024, 1024) as p, F.Plan(1024, 1024, F.FORWARD, F.PREC_SPLIT_BF16) as ps, \
            F.RealPlan(64, 64) as pr:
        want = p.exec(x)
        torch.cuda.synchronize()
        assert hip.hipStreamBeginCapture(st, relaxed) == 0
        rc_ok = L.fft2_exec(p.handle, x.data_ptr(), y.data_ptr(), st)
        rc_inplace = L.fft2_exec(p.handle, xs.data_ptr(), xs.data_ptr(), st)
        rc_filter = L.fft2_exec_filter(ps.handle, x.data_ptr(), xs.data_ptr(), ctypes.c_float(0.3), st)
        rc_real = L.fft2_exec_real(pr.handle, x.data_ptr(), xs.data_ptr(), st)
        graph, gexec = vp(), vp()
        assert hip.hipStreamEndCapture(st, ctypes.byref(graph)) == 0
        assert (rc_ok, rc_inplace, rc_filter, rc_real) == (F.SUCCESS, F.ERR_UNSUPPORTED, F.ERR_UNSUPPORTED,
                                                          F.ERR_UNSUPPORTED)
        assert "fft2_exec_noalloc" in F.last_error()[1] or F.last_error()[0] == F.ERR_UNSUPPORTED
        assert hip.hipGraphInstantiate(ctypes.byref(gexec), graph, None, None, 0) == 0
        for rep in range(3):
            y.zero_()
            torch.cuda.synchronize()
            assert hip.hipGraphLaunch(gexec, st) == 0
            assert hip.hipStreamSynchronize(st) == 0
            assert torch.equal(y, want), rep
            p.exec(x, xs)  # eager work between replays
            torch.cuda.synchronize()
        hip.hipGraphExecDestroy(gexec)
        hip.hipGraphDestroy(graph)
    hip.hipStreamDestroy(st)
    assert torch.equal(xs, want)


@pytest.mark.parametrize("shape", [(64, 64), (256, 256), (1024, 1024), (512, 2048), (64, 4096), (4096, 4096)],
                         ids=lambda s: "%dx%d" % s)
def test_every_schedule_bit_identical(shape):
    """Every candidate schedule of a shape (row-pass depth, register bits,
    lane swaps, ping-pong LDS buffers, two or three passes) runs the same
    butterflies on the same operands: all give the default plan's bits,
    forward and inverse."""
    x = _dev(inputs.smooth_image(*shape, cfg_seed=2))
    cands = F.schedule_candidates(*shape)
    assert len(cands) > 1
    for direction in (F.FORWARD, F.INVERSE):
        with F.Plan(*shape, direction) as p:
            want = p.exec(x)
        for c in cands:
            with F.Plan(*shape, direction, schedule=c) as q:
                got = q.exec(x)
                torch.cuda.synchronize()
            assert torch.equal(got, want), (direction, c)
