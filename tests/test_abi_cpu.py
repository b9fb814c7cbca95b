"""The C ABI on the CPU: the library loads, exports every declared symbol, and
rejects bad arguments before making any HIP call (so no GPU is needed)."""
import ctypes
import os
import re

import pytest

from paper_2105_09671_amd import _lib as L
from paper_2105_09671_amd import params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        names += re.findall(r"\b(ac_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libac.so not built")
    return L.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert "ac_step_2d" in names and "ac_step_3d" in names
    for n in names:
        assert hasattr(lib, n), "libac.so does not export %s" % n


def test_binding_covers_header():
    assert set(L.SIGNATURES) <= set(_declared_functions())


def test_version_and_strings(lib):
    assert lib.ac_version() >= 100
    for s in range(6):
        assert lib.ac_status_string(s)
    assert lib.ac_status_string(99) == b"unknown status"


# fake, 256-aligned device addresses: validation must fail (or succeed as a
# no-op) without dereferencing them or calling into HIP
A, B = 0x10000000, 0x20000000
H, DT = 1.0 / 64, 0.1 / 64 / 64
EPS = params.eps_m(H, 4)


def s2(lib, phi=A, work=B, nx=64, ny=64, h=H, dt=DT, eps=EPS, n=10, dtype=0):
    return lib.ac_step_2d(phi, work, nx, ny, h, dt, eps, n, dtype, None)


def s3(lib, phi=A, work=B, n3=(8, 8, 8), h=H, dt=DT, eps=EPS, n=10, dtype=0):
    return lib.ac_step_3d(phi, work, *n3, h, dt, eps, n, dtype, None)


def test_zero_steps_is_noop(lib):
    assert s2(lib, n=0) == L.AC_OK
    assert s3(lib, n=0) == L.AC_OK


@pytest.mark.parametrize("kw", [dict(phi=0), dict(work=0), dict(phi=A + 4), dict(work=B + 8),
                                dict(work=A), dict(work=A + 64 * 64 * 4 - 16), dict(nx=0),
                                dict(ny=-3), dict(h=0.0), dict(dt=-1.0), dict(eps=float("nan")),
                                dict(h=float("inf")), dict(n=-1), dict(dtype=7)])
def test_invalid_arguments_2d(lib, kw):
    assert s2(lib, **kw) == L.AC_ERR_INVALID_ARG
    assert lib.ac_last_error()


@pytest.mark.parametrize("kw", [dict(n3=(0, 4, 4)), dict(n3=(4, 4, -1)), dict(phi=0),
                                dict(work=A + 16), dict(eps=0.0), dict(n=-5)])
def test_invalid_arguments_3d(lib, kw):
    assert s3(lib, **kw) == L.AC_ERR_INVALID_ARG


def test_unstable_time_steps(lib):
    # r = dt/h^2 = 0.3 > 1/4 in 2D
    assert s2(lib, dt=0.3 * H * H) == L.AC_ERR_UNSTABLE
    # r = 0.2 > 1/6 in 3D
    assert s3(lib, dt=0.2 * H * H) == L.AC_ERR_UNSTABLE
    # alpha = dt/eps^2 too large: eps of one cell (m ~ 1.4)
    assert s2(lib, eps=H / 2) == L.AC_ERR_UNSTABLE
    assert b"alpha" in lib.ac_last_error()


def test_error_message_is_thread_local_and_cleared(lib):
    assert s2(lib, nx=0) == L.AC_ERR_INVALID_ARG
    assert lib.ac_last_error()
    assert s2(lib, n=0) == L.AC_OK
    assert lib.ac_last_error() == b""


def _inst_array(lib, specs):
    arr = (L.AcInstance2D * len(specs))()
    for i, s in enumerate(specs):
        arr[i] = L.AcInstance2D(*s)
    return arr


def test_batched_validation_before_hip(lib):
    good = [(A, B, 64, 64, H, DT, EPS), (A + 2 ** 20, B + 2 ** 20, 32, 16, H, DT, EPS)]
    arr = _inst_array(lib, good)
    assert lib.ac_step_batched(arr, 2, 0, 0, None) == L.AC_OK          # nsteps = 0
    assert lib.ac_step_batched(arr, 0, 10, 0, None) == L.AC_OK         # empty batch
    assert lib.ac_step_batched(None, 2, 10, 0, None) == L.AC_ERR_INVALID_ARG
    assert lib.ac_step_batched(arr, 2, -1, 0, None) == L.AC_ERR_INVALID_ARG
    assert lib.ac_step_batched(arr, 2, 10, 5, None) == L.AC_ERR_INVALID_ARG
    bad = _inst_array(lib, [good[0], (A + 2 ** 20, B + 2 ** 20, 0, 16, H, DT, EPS)])
    assert lib.ac_step_batched(bad, 2, 10, 0, None) == L.AC_ERR_INVALID_ARG
    assert b"instance 1" in lib.ac_last_error()
    unstable = _inst_array(lib, [good[0], (A + 2 ** 20, B + 2 ** 20, 32, 16, H, 0.3 * H * H, EPS)])
    assert lib.ac_step_batched(unstable, 2, 10, 0, None) == L.AC_ERR_UNSTABLE
    # instance 1's phi overlaps instance 0's phi
    overlap = _inst_array(lib, [good[0], (A + 1024, B + 2 ** 20, 32, 16, H, DT, EPS)])
    assert lib.ac_step_batched(overlap, 2, 10, 0, None) == L.AC_ERR_INVALID_ARG
    assert b"overlap" in lib.ac_last_error()


def test_tune_table_json_roundtrip(lib, tmp_path):
    lib.ac_tune_clear()
    assert lib.ac_tune_count() == 0
    src = tmp_path / "in.json"
    src.write_text('{"arch": "gfx950", "entries": [\n'
                   ' {"kind": 2, "dtype": 0, "cls": 22, "tb_depth": 8, "tile_x": 64, "tile_y": 64, "tile_z": 0, "kernel": 4},\n'
                   ' {"kind": 3, "dtype": 1, "cls": 24, "tb_depth": 3, "tile_x": 32, "tile_y": 16, "tile_z": 32, "kernel": 0}\n'
                   ']}\n')
    assert lib.ac_tune_load(str(src).encode()) == L.AC_OK
    assert lib.ac_tune_count() == 2
    out = tmp_path / "out.json"
    assert lib.ac_tune_save(str(out).encode()) == L.AC_OK
    lib.ac_tune_clear()
    assert lib.ac_tune_load(str(out).encode()) == L.AC_OK
    assert lib.ac_tune_count() == 2
    assert out.read_text() == src.read_text()
    # a table without the kernel field loads with the kernel left to the plan
    old = tmp_path / "old.json"
    old.write_text(src.read_text().replace(', "kernel": 4', "").replace(', "kernel": 0', ""))
    lib.ac_tune_clear()
    assert lib.ac_tune_load(str(old).encode()) == L.AC_OK
    assert lib.ac_tune_save(str(out).encode()) == L.AC_OK
    assert out.read_text() == src.read_text().replace('"kernel": 4', '"kernel": 0')
    bad = tmp_path / "bad.json"
    bad.write_text("{}")
    assert lib.ac_tune_load(str(bad).encode()) == L.AC_ERR_INVALID_ARG
    assert lib.ac_tune_load(b"/nonexistent/x.json") == L.AC_ERR_INVALID_ARG
    lib.ac_tune_clear()


# precision trace: FP32 pair A, B; FP64 pair C, D; rms and err slots R, E
C, D, R, E = 0x30000000, 0x40000000, 0x50000000, 0x60000000


def e2(lib, p32=A, w32=B, p64=C, w64=D, nx=64, ny=64, h=H, dt=DT, eps=EPS, n=10, rms=R, err=E):
    return lib.ac_err_2d(p32, w32, p64, w64, nx, ny, h, dt, eps, n, rms, err, None)


@pytest.mark.parametrize("kw", [dict(p64=A), dict(w64=B + 64), dict(p64=0), dict(w32=A),
                                dict(nx=0), dict(rms=0), dict(err=0), dict(eps=float("nan")),
                                dict(n=-1), dict(p32=A + 4)])
def test_precision_trace_rejects_bad_arguments(lib, kw):
    assert e2(lib, **kw) == L.AC_ERR_INVALID_ARG
    assert lib.ac_last_error()


def test_precision_trace_stability_gate(lib):
    assert e2(lib, dt=0.3 * H * H) == L.AC_ERR_UNSTABLE
    assert lib.ac_err_3d(A, B, C, D, 8, 8, 8, H, 0.2 * H * H, EPS, 10, R, E, None) == L.AC_ERR_UNSTABLE
    assert lib.ac_err_3d(A, B, C, D, 8, 0, 8, H, DT, EPS, 10, R, E, None) == L.AC_ERR_INVALID_ARG


def _inst3(phi, work, n3=(8, 8, 8), h=H, dt=DT, eps=EPS):
    return L.AcInstance3D(phi, work, *n3, h, dt, eps)


@pytest.mark.parametrize("bad", [dict(n3=(8, 0, 8)), dict(work=A + 16), dict(dt=0.2 * H * H),
                                 dict(eps=-1.0)])
def test_batched3d_validation_before_hip(lib, bad):
    kw = dict(phi=A, work=B)
    kw.update(bad)
    arr = (L.AcInstance3D * 2)(_inst3(C, D), _inst3(**kw))
    st = lib.ac_step_batched_3d(arr, 2, 10, 0, None, None, None)
    assert st in (L.AC_ERR_INVALID_ARG, L.AC_ERR_UNSTABLE)
    assert b"instance 1" in lib.ac_last_error()


def test_batched3d_rejects_overlap_between_instances(lib):
    arr = (L.AcInstance3D * 2)(_inst3(A, B), _inst3(C, A + 256))
    assert lib.ac_step_batched_3d(arr, 2, 10, 0, None, None, None) == L.AC_ERR_INVALID_ARG
    assert b"overlap" in lib.ac_last_error()


def test_autotune_one_call_validation_and_cache_hit(lib, tmp_path):
    """ac_autotune(dim, dtype, cache): bad dim / dtype fail before any HIP call;
    an existing cache that does not parse is refused and left as it was; a cache
    that already covers every representative size class of (dim, dtype) times
    nothing (no HIP call, so this runs without a GPU) and is written back."""
    lib.ac_tune_clear()
    assert lib.ac_autotune(1, 0, None) == L.AC_ERR_INVALID_ARG
    assert lib.ac_autotune(4, 0, None) == L.AC_ERR_INVALID_ARG
    assert lib.ac_autotune(2, 7, None) == L.AC_ERR_INVALID_ARG
    assert b"dtype" in lib.ac_last_error()
    junk = tmp_path / "junk.json"
    junk.write_text("not a table\n")
    assert lib.ac_autotune(2, 0, str(junk).encode()) == L.AC_ERR_INVALID_ARG
    assert junk.read_text() == "not a table\n"
    # size classes floor(log2(cells)): 512^2 -> 18, 2048^2 -> 22, 4096^2 -> 24;
    # 128^3 -> 21, 256^3 -> 24
    rows = [(2, 0, 18, 5, 64, 64, 0, 4), (2, 0, 22, 7, 64, 128, 0, 4), (2, 0, 24, 8, 128, 128, 0, 6),
            (3, 1, 21, 3, 64, 32, 32, 5), (3, 1, 24, 4, 64, 32, 64, 5)]
    cache = tmp_path / "cache.json"
    cache.write_text('{"arch": "gfx950", "entries": [\n' + ",\n".join(
        ' {"kind": %d, "dtype": %d, "cls": %d, "tb_depth": %d, "tile_x": %d, "tile_y": %d, '
        '"tile_z": %d, "kernel": %d}' % r for r in rows) + "\n]}\n")
    assert lib.ac_autotune(2, 0, str(cache).encode()) == L.AC_OK
    assert lib.ac_autotune(3, 1, str(cache).encode()) == L.AC_OK
    assert lib.ac_tune_count() == len(rows)
    text = cache.read_text()
    for r in rows:
        assert '"kind": %d, "dtype": %d, "cls": %d, "tb_depth": %d' % r[:4] in text
    lib.ac_tune_clear()


def test_surrogate_calls_reject_null_handle(lib):
    assert lib.ac_sur_backward(None, None, 1) == L.AC_ERR_INVALID_ARG
    assert lib.ac_sur_backward(None, A, 1) == L.AC_ERR_INVALID_ARG
    assert lib.ac_sur_forward(None, A, B, 1) == L.AC_ERR_INVALID_ARG
    assert lib.ac_sur_adam_step(None, 1e-3, 0.9, 0.999, 1e-8, 1) == L.AC_ERR_INVALID_ARG


def test_noalloc_judge_validation_before_hip(lib):
    """Size and pointer errors of the allocation-free judge come before any HIP
    call (batch above the static scratch's 16384 grids included)."""
    f = lib.ac_judge_2d_noalloc
    assert f(A, B, 16385, 64, 64, H, 3, C, D, None) == L.AC_ERR_INVALID_ARG
    assert b"16384" in lib.ac_last_error()
    assert f(A, B, 0, 64, 64, H, 3, C, D, None) == L.AC_ERR_INVALID_ARG
    assert f(A, B, 4, 64, 64, H, 17, C, D, None) == L.AC_ERR_INVALID_ARG
    assert f(0, B, 4, 64, 64, H, 3, C, D, None) == L.AC_ERR_INVALID_ARG
    assert f(A, B, 4, 64, 64, -1.0, 3, C, D, None) == L.AC_ERR_INVALID_ARG
