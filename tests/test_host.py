"""CPU-only checks of the library boundary: it loads, exports every symbol the
header declares, validates arguments and picks pass schedules without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1505_08019_amd import fft2 as F
from paper_1505_08019_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "fft2.h")).read()
    return sorted(set(re.findall(r"\b(fft2_[a-z_0-9]+)\s*\(", txt)))


def test_header_lists_match_binding():
    assert _header_functions() == sorted(F.EXPORTS)


def test_library_exports_every_symbol():
    lib = F.lib()
    for name in _header_functions():
        assert hasattr(lib, name), name


def test_validate():
    assert F.validate(1024, 1024) == F.SUCCESS
    assert F.validate(1, 1) == F.SUCCESS
    assert F.validate(16384, 16384) == F.SUCCESS
    assert F.validate(3, 4) == F.ERR_INVALID_SIZE
    assert F.validate(0, 4) == F.ERR_INVALID_SIZE
    assert F.validate(32768, 4) == F.ERR_INVALID_SIZE
    assert F.validate(4, -8) == F.ERR_INVALID_SIZE
    assert F.validate(4, 4, 0) == F.ERR_INVALID_VALUE
    assert F.validate(4, 4, -1, 7) == F.ERR_INVALID_VALUE
    code, text = F.last_error()
    assert code == F.ERR_INVALID_VALUE and "precision" in text
    assert F.lib().fft2_error_string(F.ERR_ALIAS).decode()


def _passes(desc):
    return [dict(kind=m.group(1), **{k: int(v) for k, v in re.findall(r"(\w+)=(\d+)", m.group(2))})
            for m in re.finditer(r"(row|col)\(([^)]*)\)", desc)]


@pytest.mark.parametrize("bm", range(0, 15))
@pytest.mark.parametrize("bn", range(0, 15))
def test_schedule_covers_every_stage(bm, bn):
    """Every size has a schedule whose passes run each column stage exactly
    once, in order, and every row stage in the first pass."""
    ps = _passes(F.describe_schedule(1 << bm, 1 << bn))
    assert ps[0]["kind"] == "row" and ps[0]["bn"] == bn
    done = ps[0]["j"]
    for p in ps[1:]:
        assert p["kind"] == "col" and p["s_lo"] == done
        done += p["nz"]
        assert p["cb"] + p["nz"] <= 15
    assert done == bm
    assert ps[0]["bn"] + ps[0]["j"] <= 15
    assert len(ps) <= 3


def test_flagship_schedules():
    assert len(_passes(F.describe_schedule(1024, 1024))) == 2
    assert len(_passes(F.describe_schedule(8192, 8192))) == 2
    assert len(_passes(F.describe_schedule(64, 64))) == 1


def test_inputs_deterministic():
    a = inputs.uniform_pixels(64, 32, 1, 3)
    b = inputs.uniform_pixels(64, 32, 1, 3)
    c = inputs.uniform_pixels(64, 32, 1, 4)
    assert a.dtype == np.complex64 and np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.real.min() >= 0 and a.real.max() <= 255 and np.all(a.imag == 0)
    assert np.all(a.real == np.round(a.real))
    s = inputs.smooth_image(128, 64, 2, 0)
    assert np.array_equal(s, inputs.smooth_image(128, 64, 2, 0))
    shapes = inputs.ragged_shapes(512)
    assert shapes == inputs.ragged_shapes(512)
    sides = {r for r, c in shapes} | {c for r, c in shapes}
    assert sides <= {64, 128, 256, 512, 1024, 2048}
    rect = sum(1 for r, c in shapes if r != c)
    assert 0.15 < rect / 512 < 0.35
    tr = inputs.poisson_trace(5000.0, 2000)
    gaps = np.diff(tr["t"])
    assert abs(gaps.mean() * 5000.0 - 1.0) < 0.1
    assert set(np.unique(tr["precision"])) <= {0, 1}


def test_no_cpu_fallback_in_binding():
    """The product package (binding, build, kernels, host code) never imports,
    links or loads the oracle."""
    import re
    pkg = os.path.join(ROOT, "paper_1505_08019_amd")
    files = [os.path.join(pkg, f) for f in os.listdir(pkg) if f.endswith(".py")]
    files += [os.path.join(pkg, "csrc", f) for f in os.listdir(os.path.join(pkg, "csrc"))]
    pat = re.compile(r"import\s+oracle|from\s+oracle|liboracle|oracle/|fft2_oracle")
    for f in files:
        assert not pat.search(open(f, errors="replace").read()), f


def test_batch_validate_host():
    assert F.batch_validate([(64, 64), (2048, 512), (512, 2048)]) == F.SUCCESS
    assert F.batch_validate([(64, 64)], precision=F.PREC_SPLIT_BF16) == F.SUCCESS
    assert F.batch_validate([(4096, 4096)], precision=F.PREC_SPLIT_BF16) == F.SUCCESS
    assert F.batch_validate([(8192, 8192), (4096, 8192)], precision=F.PREC_SPLIT_BF16) == F.SUCCESS
    # shapes outside the persistent kernel's menu run as their own passes
    assert F.batch_validate([(64, 8), (64, 16384), (4096, 16), (1, 1)]) == F.SUCCESS
    assert F.batch_validate([(16384, 16384)], precision=F.PREC_SPLIT_BF16) == F.ERR_UNSUPPORTED
    assert F.batch_validate([(3, 64)]) == F.ERR_INVALID_SIZE
    assert F.batch_validate([]) == F.ERR_INVALID_VALUE
    assert F.batch_validate([(64, 64)], direction=0) == F.ERR_INVALID_VALUE
    assert F.batch_validate([(64, 64)], precision=F.PREC_FP16) == F.ERR_UNSUPPORTED
    assert F.batch_validate(inputs.ragged_shapes(512)) == F.SUCCESS
    assert F.batch_validate(inputs.ragged_shapes(512), precision=F.PREC_SPLIT_BF16) == F.SUCCESS


def test_serve_config_validation_host():
    """Pure host checks of a server configuration (no device is touched)."""
    v = F.serve_validate_config
    assert v(64 << 30, 4, 8, 0) == F.SUCCESS
    assert v(0, 4, 8, 0) == F.ERR_INVALID_VALUE
    assert v(64 << 30, 0, 8, 0) == F.ERR_INVALID_VALUE
    assert v(64 << 30, 65, 8, 0) == F.ERR_INVALID_VALUE
    assert v(64 << 30, 4, 0, 0) == F.ERR_INVALID_VALUE
    assert v(64 << 30, 4, 8, -1) == F.ERR_INVALID_VALUE
    assert v(64 << 30, 4, 8, 0, -5) == F.ERR_INVALID_VALUE
    assert v(64 << 30, 4, 8, 0, 0, -1) == F.ERR_INVALID_VALUE
    assert v(64 << 30, 4, 8, 0, 0, 4) == F.SUCCESS
    # four workspaces of 4096 x 4096 values (128 MiB each) exceed a 256 MiB budget
    assert v(256 << 20, 4, 8, 0) == F.ERR_BUDGET
    assert v(256 << 20, 4, 8, 0, 1 << 20) == F.SUCCESS
    assert F.lib().fft2_serve_validate_config(None) == F.ERR_INVALID_VALUE


def test_ping_pong_schedule_strings():
    """Ping-pong variants (two LDS buffers) are schedule candidates written
    with a 'p' after their register bits, and plan descriptions name them."""
    cands = F.schedule_candidates(1024, 1024)
    assert any("p" in c for c in cands) and any("p" not in c for c in cands)
    for c in cands:
        for part in c.split():
            reg = part.split(",")[1]
            assert reg.rstrip("p").isdigit()
