"""C-ABI contract checks that need no GPU: the HIP library loads and exports
every entry point declared in include/lr.h, the oracle exports the same call
shapes, and the binding refuses to work without the library or a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lr_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared("include/lr.h")
    for n in ("lr_create", "lr_set_state", "lr_step", "lr_run", "lr_get_fields", "lr_totals",
              "lr_destroy", "lr_bind_stream", "lr_last_error", "lr_debug_get", "lr_default_opts",
              "lr_set_state_device", "lr_batch_create", "lr_batch_submit", "lr_batch_step",
              "lr_batch_poll", "lr_batch_get_fields", "lr_batch_release", "lr_batch_destroy"):
        assert n in names


def test_hip_library_exports_every_declared_symbol():
    so = os.path.join(ROOT, "paper_2208_13409_amd", "liblr.so")
    if not os.path.exists(so):
        from paper_2208_13409_amd import build
        build.build()
    lib = ctypes.CDLL(so)
    for n in _declared("include/lr.h"):
        assert hasattr(lib, n), n


def test_oracle_exports_the_same_calls():
    from oracle import load
    lib = load()
    for n in _declared("include/lr.h"):
        if n in ("lr_bind_stream", "lr_profile", "lr_profile_read", "lr_kernel_count",
                 "lr_kernel_name", "lr_set_state_device", "lr_run_noalloc") or n.startswith("lr_batch_"):
            continue  # host-only oracle: no streams, kernels, device inputs or batches
        assert hasattr(lib, n.replace("lr_", "lr_ref_", 1)), n


def test_binding_has_no_fallback(monkeypatch, tmp_path):
    from paper_2208_13409_amd import lr
    monkeypatch.setattr(lr, "_LIB", None)
    monkeypatch.setattr(lr, "SO_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(FileNotFoundError):
        lr.Solver(4, 4, [1.4])


def test_argument_validation_without_device():
    """Bad sizes are rejected before any device call."""
    from paper_2208_13409_amd import lr
    lib = lr.load()
    o = lr.lr_default_opts()
    eos = (lr.lr_eos * 1)(lr.lr_eos(1.4, 0.0))
    h = ctypes.c_void_p()
    assert lib.lr_create(1, 4, 1, eos, None, ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    assert lib.lr_create(4, 4, 0, eos, None, ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    # more than 2^28 cells: beyond the 32-bit cell indexing
    assert lib.lr_create(1 << 15, (1 << 13) + 1, 1, eos, None, ctypes.byref(o),
                         ctypes.byref(h)) == lr.LR_EINVAL
    o.precision = 7
    assert lib.lr_create(4, 4, 1, eos, None, ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    bad = (lr.lr_eos * 1)(lr.lr_eos(1.4, -3.0))
    o = lr.lr_default_opts()
    assert lib.lr_create(4, 4, 1, bad, None, ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    o.mix_list = -1
    assert lib.lr_create(4, 4, 1, eos, None, ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    assert lib.lr_step(None, None) == lr.LR_EINVAL


def test_binding_exports_list_matches_header():
    from paper_2208_13409_amd import lr
    assert sorted(lr.EXPORTS) == _declared("include/lr.h")


def test_batch_argument_validation_without_device():
    """Batch options are checked before any device call; the footprint is
    host arithmetic and grows with the grid."""
    from paper_2208_13409_amd import lr
    lib = lr.load()
    o = lr.lr_batch_default_opts()
    assert o.chunk_steps % 2 == 0 and o.max_slots >= 1
    h = ctypes.c_void_p()
    o.chunk_steps = 3
    assert lib.lr_batch_create(ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    o = lr.lr_batch_default_opts()
    o.nmat = 0
    assert lib.lr_batch_create(ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    o = lr.lr_batch_default_opts()
    assert o.tile == lr.LR_TILE_32x8
    o.tile = lr.LR_NTILE
    assert lib.lr_batch_create(ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    f32 = lib.lr_batch_footprint(64, 64, 2, lr.LR_FP32)
    f64 = lib.lr_batch_footprint(64, 64, 2, lr.LR_FP64)
    big = lib.lr_batch_footprint(128, 128, 2, lr.LR_FP32)
    assert 0 < f32 < f64 and 3.5 * f32 < big < 4.5 * f32
    # the list of mixed cells is sized to need (1/16 of the cells to start
    # with): 2 materials in FP32 take about 108 bytes per cell, 3 in FP64 273
    assert lib.lr_batch_footprint(512, 512, 2, lr.LR_FP32) / 512 ** 2 < 112
    assert lib.lr_batch_footprint(512, 512, 3, lr.LR_FP64) / 512 ** 2 < 280
    assert lib.lr_batch_footprint(1, 64, 2, lr.LR_FP32) == 0
    assert lib.lr_batch_step(None, None) == lr.LR_EINVAL


def test_noalloc_rejects_bad_arguments_without_device():
    """lr_run_noalloc checks sizes and options before any device call, and
    names the failure in the caller's buffer."""
    from paper_2208_13409_amd import lr
    lib = lr.load()
    o = lr.lr_default_opts()
    eos = (lr.lr_eos * 1)(lr.lr_eos(1.4, 0.0))
    err = ctypes.create_string_buffer(128)
    null = ctypes.c_void_p(0)
    args = [1.0, 10, ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1),
            ctypes.c_void_p(1), 0, None, null, None, None, err, len(err)]
    assert lib.lr_run_noalloc(1, 4, 1, eos, None, ctypes.byref(o), 0.0, *args) == lr.LR_EINVAL
    assert b"invalid grid" in err.value
    o.stages = 1
    assert lib.lr_run_noalloc(4, 4, 1, eos, None, ctypes.byref(o), 0.0, *args) == lr.LR_EINVAL
    assert b"stages" in err.value


def test_eos_arguments_checked_without_device():
    """A stiffened-gas pi must be finite and >= 0, gamma > 1: rejected before
    any device call."""
    from paper_2208_13409_amd import lr
    lib = lr.load()
    o = lr.lr_default_opts()
    h = ctypes.c_void_p()
    for g, pi in ((1.4, -1.0), (1.4, float("inf")), (1.0, 0.0)):
        eos = (lr.lr_eos * 1)(lr.lr_eos(g, pi))
        assert lib.lr_create(8, 8, 1, eos, None, ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL


def test_tile_option_checked_without_device():
    """lr_opts.tile defaults to automatic; a shape outside LR_TILE_* and the
    alternate-direction remap on any shape but 32x8 are rejected before any
    device call."""
    from paper_2208_13409_amd import lr
    lib = lr.load()
    o = lr.lr_default_opts()
    assert o.tile == lr.LR_TILE_AUTO
    eos = (lr.lr_eos * 1)(lr.lr_eos(1.4, 0.0))
    h = ctypes.c_void_p()
    for tile in (-2, lr.LR_NTILE):
        o.tile = tile
        assert lib.lr_create(8, 8, 1, eos, None, ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    o.remap = lr.LR_REMAP_AD
    for tile in (lr.LR_TILE_16x16, lr.LR_TILE_32x16, lr.LR_TILE_32x12):
        o.tile = tile
        assert lib.lr_create(8, 8, 1, eos, None, ctypes.byref(o), ctypes.byref(h)) == lr.LR_EINVAL
    assert lr.TILE_SHAPES[lr.LR_TILE_32x12] == (32, 12) and len(lr.TILE_SHAPES) == lr.LR_NTILE
