"""Ragged batches in one persistent launch, through the C ABI.

Each image of a batch must be bit-identical to the same image transformed
alone (the schedule depends only on shape, precision and direction), and
match the FP64 oracle; HIP-graph replays must equal the eager launch."""
import numpy as np
import pytest

import oracle
from paper_1505_08019_amd import fft2 as F
from paper_1505_08019_amd import inputs
from paper_1505_08019_amd.metrics import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to("cuda:0")


def _alone(x, precision, direction=F.FORWARD):
    r, c = x.shape
    with F.Plan(r, c, direction, precision) as p:
        return p.exec(x)


SMALL = [(64, 64), (128, 512), (512, 128), (16, 16), (1024, 1024), (64, 2048), (2048, 64), (256, 256), (8, 256),
         (4, 64), (1, 512), (32, 32), (512, 512), (2048, 2048), (128, 128), (1024, 256)]


@pytest.mark.parametrize("precision", [F.PREC_FP32, F.PREC_SPLIT_BF16], ids=["fp32", "split_bf16"])
@pytest.mark.parametrize("direction", [F.FORWARD, F.INVERSE], ids=["fwd", "inv"])
def test_small_batch_matches_alone(precision, direction):
    shapes = SMALL
    xs = [_dev(inputs.uniform_pixels(r, c, cfg_seed=4, index=i)) for i, (r, c) in enumerate(shapes)]
    outs = [torch.empty_like(x) for x in xs]
    with F.Batch(shapes, direction, precision) as b:
        b.exec(xs, outs)
        assert b.status() == 0
    torch.cuda.synchronize()
    for i, (x, y) in enumerate(zip(xs, outs)):
        assert torch.equal(y, _alone(x, precision, direction)), shapes[i]
    # a few against the oracle
    tol = 2e-6 if precision == F.PREC_FP32 else 5e-6
    for i in (0, 4, 9, 13):
        want = oracle.fft2(xs[i].cpu().numpy(), direction, threads=0)
        assert rel_l2(outs[i].cpu().numpy(), want) <= tol, shapes[i]


def test_graph_replay_equals_eager():
    shapes = SMALL[:8]
    xs = [_dev(inputs.smooth_image(r, c, cfg_seed=4, index=i)) for i, (r, c) in enumerate(shapes)]
    eager = [torch.empty_like(x) for x in xs]
    outs = [torch.empty_like(x) for x in xs]
    # b replays a graph on its own buffers; be does the eager work in between
    # (a replay with no buffers reuses the batch's last ones).
    with F.Batch(shapes) as b, F.Batch(shapes) as be:
        be.exec(xs, eager)
        torch.cuda.synchronize()
        for rep in range(4):
            for y in outs:
                y.zero_()
            torch.cuda.synchronize()
            b.exec(xs if rep == 0 else None, outs if rep == 0 else None, graph=True)
            torch.cuda.synchronize()
            for e, y in zip(eager, outs):
                assert torch.equal(e, y), rep
            # eager work between replays
            be.exec(xs, eager)
            _alone(xs[3], F.PREC_FP32)
            torch.cuda.synchronize()
            if rep == 1:
                # change an input in place: replays and eager runs must follow it
                xs[0].mul_(2)
                be.exec(xs, eager)
        assert b.status() == 0 and be.status() == 0
        # buffers given to a replay re-target it
        other = [torch.zeros_like(x) for x in xs]
        b.exec(xs, other, graph=True)
        torch.cuda.synchronize()
        for e, y in zip(eager, other):
            assert torch.equal(e, y)


def test_tuned_batch_is_bit_identical():
    shapes = [(256, 256), (1024, 512), (64, 4096)]
    xs = [_dev(inputs.uniform_pixels(r, c, cfg_seed=4, index=i)) for i, (r, c) in enumerate(shapes)]
    a = [torch.empty_like(x) for x in xs]
    t = [torch.empty_like(x) for x in xs]
    with F.Batch(shapes) as b1, F.Batch(shapes, tuned_reps=3) as b2:
        b1.exec(xs, a)
        b2.exec(xs, t)
    torch.cuda.synchronize()
    for u, v in zip(a, t):
        assert torch.equal(u, v)


def test_batch_errors():
    assert F.batch_validate([(3, 64)]) == F.ERR_INVALID_SIZE
    assert F.batch_validate([(16384, 16384)], precision=F.PREC_SPLIT_BF16) == F.ERR_UNSUPPORTED
    x = _dev(inputs.uniform_pixels(64, 64, cfg_seed=4))
    with F.Batch([(64, 64)]) as b:
        with pytest.raises(F.FFT2Error):
            b.exec([x], [x])


@pytest.mark.parametrize("precision", [F.PREC_FP32, F.PREC_SPLIT_BF16], ids=["fp32", "split_bf16"])
@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
@pytest.mark.parametrize("side", [False, True], ids=["default_stream", "side_stream"])
def test_batch_stream_order(precision, graph, side):
    """The batch's lanes start after the work already on the caller's stream
    and finish before the work enqueued on it afterwards: inputs written by
    copies queued just before the call and outputs read by clones queued just
    after it, with no synchronisation in between, give each image's result.
    The caller's stream is torch's default stream or a stream of its own."""
    shapes = [(2048, 2048), (1024, 512), (512, 512), (64, 64), (1024, 1024), (128, 128), (512, 2048)]
    src = [_dev(inputs.uniform_pixels(r, c, cfg_seed=4, index=i)) for i, (r, c) in enumerate(shapes)]
    want = [_alone(x, precision) for x in src]
    xs = [torch.zeros_like(x) for x in src]
    outs = [torch.zeros_like(x) for x in src]
    st = torch.cuda.Stream() if side else torch.cuda.current_stream()
    with F.Batch(shapes, F.FORWARD, precision) as b:
        for rep in range(3):
            torch.cuda.synchronize()
            with torch.cuda.stream(st):
                for x, y in zip(xs, outs):
                    x.zero_()
                    y.zero_()
                for x, s_ in zip(xs, src):
                    x.copy_(s_)
                b.exec(xs if rep == 0 else None, outs if rep == 0 else None, st, graph=graph)
                got = [y.clone() for y in outs]
            torch.cuda.synchronize()
            assert b.status() == 0
            for i, (g_, w) in enumerate(zip(got, want)):
                assert torch.equal(g_, w), (rep, shapes[i])


def test_batch_buffer_overlap():
    """The jobs of a batch run concurrently: an output shared with another
    image, or reaching into another image's input, is refused; a shared
    input is allowed and gives every image the result it gives alone."""
    shapes = [(1024, 1024), (512, 512), (64, 64), (512, 512)]
    xs = [_dev(inputs.uniform_pixels(r, c, cfg_seed=4, index=i)) for i, (r, c) in enumerate(shapes)]
    outs = [torch.empty_like(x) for x in xs]
    big = torch.empty(1024 * 1024 + 16, dtype=torch.complex64, device="cuda:0")
    with F.Batch(shapes) as b:
        for bad_outs, bad_ins in (
                ([outs[0], outs[1], outs[2], outs[1]], xs),                       # two images, one output
                ([outs[0], big[8:8 + 512 * 512].view(512, 512), outs[2], outs[3]],
                 [big[:1024 * 1024].view(1024, 1024)] + xs[1:]),                 # output inside another input
                ([outs[0], outs[1], outs[2], xs[1]], xs)):                        # output = another image's input
            with pytest.raises(F.FFT2Error) as ei:
                b.exec(bad_ins, bad_outs)
            assert ei.value.code == F.ERR_ALIAS
        shared = [xs[0], xs[1], xs[2], xs[1]]
        b.exec(shared, outs)
        torch.cuda.synchronize()
        assert b.status() == 0
    for x, y in zip(shared, outs):
        assert torch.equal(y, _alone(x, F.PREC_FP32))


@pytest.mark.parametrize("precision", [F.PREC_FP32, F.PREC_SPLIT_BF16], ids=["fp32", "split_bf16"])
def test_direct_and_persistent_mix(precision):
    """Large images and shapes outside the persistent menu run as their own
    pass kernels in the same batch; new buffers rebuild a captured graph."""
    shapes = [(1024, 1024), (64, 8), (16, 4096), (4096, 16), (64, 64), (512, 1024), (1, 1), (8, 8), (256, 128)]
    if precision == F.PREC_FP32:
        shapes += [(8192, 64), (2, 16384)]
    xs = [_dev(inputs.uniform_pixels(r, c, cfg_seed=4, index=i)) for i, (r, c) in enumerate(shapes)]
    alone = [_alone(x, precision) for x in xs]
    for graph in (False, True):
        with F.Batch(shapes, F.FORWARD, precision) as b:
            for rep in range(3):
                outs = [torch.zeros_like(x) for x in xs]
                b.exec(xs, outs, graph=graph)
                torch.cuda.synchronize()
                assert b.status() == 0
                for i, (y, a) in enumerate(zip(outs, alone)):
                    assert torch.equal(y, a), (graph, rep, shapes[i])


@pytest.mark.parametrize("precision", [F.PREC_FP32, F.PREC_SPLIT_BF16], ids=["fp32", "split_bf16"])
def test_config4_ragged_512(precision):
    """Config 4: 512 images, sides log-uniform 64..2048, a quarter rectangular,
    uniform pixels: the small ones in one persistent launch, the large ones
    as their own pass kernels."""
    shapes = inputs.ragged_shapes(512)
    xs = [_dev(inputs.uniform_pixels(r, c, cfg_seed=4, index=i)) for i, (r, c) in enumerate(shapes)]
    outs = [torch.empty_like(x) for x in xs]
    with F.Batch(shapes, F.FORWARD, precision) as b:
        items, wgs, lds = b.info()
        print("config 4: %d work items, %d persistent workgroups, %d B LDS" % (items, wgs, lds), flush=True)
        b.exec(xs, outs)
        assert b.status() == 0
    torch.cuda.synchronize()
    for i in range(len(shapes)):
        assert torch.equal(outs[i], _alone(xs[i], precision)), (i, shapes[i])
    tol = 2e-6 if precision == F.PREC_FP32 else 5e-6
    g = np.random.default_rng(0)
    for i in g.choice(len(shapes), size=4, replace=False):
        want = oracle.fft2(xs[i].cpu().numpy(), threads=0)
        assert rel_l2(outs[i].cpu().numpy(), want) <= tol, shapes[i]
