"""The C ABI library: it loads, exports every symbol include/oed.h declares, and
rejects invalid arguments on the host before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oed.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^OED_API\s+[\w\s\*]+?\b(oed_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2604_08812_amd import library
    return library()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("oed_create", "oed_greedy", "oed_destroy", "oed_last_error", "oed_force", "oed_reset",
                 "oed_scores", "oed_schur_block", "oed_picks", "oed_get_profile"):
        assert name in syms


def test_every_declared_symbol_is_exported(lib):
    from paper_2604_08812_amd import EXPORTED
    syms = declared_symbols()
    for name in syms:
        assert hasattr(lib, name), name
    assert sorted(EXPORTED) == syms


def test_host_side_argument_validation(lib):
    from paper_2604_08812_amd.oed import oed_options
    opt = oed_options()
    lib.oed_options_init(ctypes.byref(opt))
    assert opt.struct_size == ctypes.sizeof(oed_options) and opt.precision == 0
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    E_ARG = 1
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 0.0, None, ctypes.byref(opt)) == E_ARG
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, float("nan"), None, ctypes.byref(opt)) == E_ARG
    assert lib.oed_create(ctypes.byref(h), fake, 0, 63, 4, 16, 1.0, None, ctypes.byref(opt)) == E_ARG
    assert lib.oed_create(ctypes.byref(h), fake, 7, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == E_ARG
    assert lib.oed_create(ctypes.byref(h), None, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == E_ARG
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 0, 16, 1.0, None, ctypes.byref(opt)) == E_ARG
    bad = oed_options()
    lib.oed_options_init(ctypes.byref(bad))
    bad.precision = 9
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(bad)) == E_ARG
    bad.precision = 2  # BF16 split product, held block columns: N_t <= 1024 (as every precision)
    bad.delay = 2
    assert lib.oed_create(ctypes.byref(h), fake, 0, 2 * 1040, 2, 1040, 1.0, None, ctypes.byref(bad)) == 6
    assert "N_t <= 1024" in lib.oed_last_error(None).decode()
    bad = oed_options()
    lib.oed_options_init(ctypes.byref(bad))
    bad.method = 5
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(bad)) == E_ARG
    bad.method = 1
    bad.max_budget = 5     # > N_s
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(bad)) == E_ARG
    bad.max_budget = 0     # left-looking serves N_t <= 1024
    assert lib.oed_create(ctypes.byref(h), fake, 0, 2 * 1025, 2, 1025, 1.0, None, ctypes.byref(bad)) == 6
    bad = oed_options()
    lib.oed_options_init(ctypes.byref(bad))
    hn = (ctypes.c_double * 4)(0.0, float("nan"), 1.0, 2.0)   # non-finite per-sensor noise term
    bad.noise_half_logdet = ctypes.cast(hn, ctypes.POINTER(ctypes.c_double))
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(bad)) == E_ARG
    bad = oed_options()
    lib.oed_options_init(ctypes.byref(bad))
    bad.delay = 13
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(bad)) == E_ARG
    bad = oed_options()
    lib.oed_options_init(ctypes.byref(bad))
    bad.struct_size = 4
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(bad)) == E_ARG
    cand = (ctypes.c_int32 * 2)(1, 9)
    bad = oed_options()
    lib.oed_options_init(ctypes.byref(bad))
    bad.candidates = ctypes.cast(cand, ctypes.POINTER(ctypes.c_int32))
    bad.n_candidates = 2
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(bad)) == E_ARG
    assert not h.value
    assert lib.oed_greedy(None, 1, None, None, None) == E_ARG
    assert lib.oed_destroy(None) == 0
    assert lib.oed_status_string(2) == b"OED_E_NOT_SPD"
    # NULL handle: the text of the thread's last failed oed_create
    assert lib.oed_last_error(None) == b"candidate out of range or repeated"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2604_08812_amd.oed as b
    monkeypatch.setattr(b, "_lib", None)
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        b.library()


def test_batch_host_side_validation(lib):
    from paper_2604_08812_amd.oed import oed_instance
    b = ctypes.c_void_p()
    fake = 0x1000  # never dereferenced: validation fails before any device call
    ok = oed_instance(fake, 0, 8, 16, 4, 128, 1.0)
    bad_budget = oed_instance(fake, 0, 8, 16, 9, 128, 1.0)
    big_nt = oed_instance(fake, 0, 2, 160, 1, 320, 1.0)
    bad_sigma = oed_instance(fake, 0, 8, 16, 4, 128, -1.0)
    for inst, code in ((bad_budget, 1), (bad_sigma, 1), (big_nt, 6)):
        arr = (oed_instance * 2)(ok, inst)
        assert lib.oed_batch_create(ctypes.byref(b), arr, 2, 1, None, 0) == code
    arr = (oed_instance * 1)(ok)
    assert lib.oed_batch_create(ctypes.byref(b), arr, 0, 1, None, 0) == 1
    assert lib.oed_batch_create(ctypes.byref(b), arr, 1, 9, None, 0) == 1   # no such precision
    assert not b.value
    assert lib.oed_batch_destroy(None) == 0


def test_eval_host_side_validation(lib):
    e = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails before any device call
    E_ARG, E_UNSUPPORTED = 1, 6
    #            K     dtype ld   N_s N_t sigma2 B  batch prec stream flags
    good = [fake, 0, 128, 8, 16, 1.0, 4, 2, 1, None, 0]
    for pos, val, code in ((0, None, E_ARG), (1, 5, E_ARG), (2, 127, E_ARG), (3, 0, E_ARG), (5, 0.0, E_ARG),
                           (5, float("inf"), E_ARG), (6, 0, E_ARG), (6, 9, E_ARG), (7, -1, E_ARG), (8, 7, E_ARG),
                           (10, 0x10, E_ARG), (10, 0x20, E_ARG), (10, 13 << 8, E_ARG)):
        args = list(good)
        args[pos] = val
        assert lib.oed_eval_create(ctypes.byref(e), *args) == code, (pos, val)
        assert not e.value
    big = [fake, 0, 2 * 160, 2, 160, 1.0, 1, 1, 1, None, 0]
    assert lib.oed_eval_create(ctypes.byref(e), *big) == E_UNSUPPORTED
    assert lib.oed_eval_create(None, *good) == E_ARG
    assert lib.oed_eval_destroy(None) == 0
    assert lib.oed_eval_run(None, None, 0, None, None) == E_ARG
    assert lib.oed_eval_stats(None, None, None, None, None) == E_ARG
    assert lib.oed_eval_last_error(None) == b"null evaluator"


def test_deferred_pack_host_side_validation(lib):
    from paper_2604_08812_amd.oed import OED_FLAG_AUTOTUNE, OED_FLAG_DEFER_PACK, oed_options
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced
    opt = oed_options()
    lib.oed_options_init(ctypes.byref(opt))
    opt.flags = OED_FLAG_DEFER_PACK
    # deferred packing takes no K, and cannot autotune (nothing packed to time on)
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == 1
    opt.flags = OED_FLAG_DEFER_PACK | OED_FLAG_AUTOTUNE
    assert lib.oed_create(ctypes.byref(h), None, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == 1
    opt.flags = OED_FLAG_DEFER_PACK
    assert lib.oed_create(ctypes.byref(h), None, 0, 64, 4, 16, 0.0, None, ctypes.byref(opt)) == 1
    assert not h.value
    assert lib.oed_pack_rows(None, fake, 0, 64, 0, 1) == 1


def test_options_layout_and_create_errors_without_a_gpu(lib):
    """The options struct the binding builds has the C size; a device-memory limit below what the
    handle needs is OED_E_OOM before any HIP call, with the bytes in oed_last_error(NULL); bad tile
    orders, negative limits and hook steps are OED_E_ARG with a message."""
    from paper_2604_08812_amd.oed import oed_options
    opt = oed_options()
    lib.oed_options_init(ctypes.byref(opt))
    assert opt.struct_size == ctypes.sizeof(oed_options)
    assert opt.tile_order == 0 and opt.max_device_bytes == 0 and opt.debug_fail_step == 0 and not opt.tune_cache
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails before any HIP call
    opt.max_device_bytes = 1000
    # 4 sensors x 16, FP64: R alone is 10 blocks of 16^2 doubles = 20,480 bytes
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == 3
    msg = lib.oed_last_error(None).decode()
    assert "max_device_bytes = 1000" in msg and "needs" in msg and not h.value
    opt.max_device_bytes = -1
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == 1
    opt.max_device_bytes = 0
    opt.tile_order = 9
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == 1
    assert "tile order" in lib.oed_last_error(None).decode()
    opt.tile_order = 0
    opt.debug_fail_step = -2
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == 1
    opt.debug_fail_step = 0
    opt.tile_size = 64
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == 1
    opt.tile_size = 256      # 256 x 256 downdate tiles: the BF16 split product only
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == 6
    opt.precision = 2        # ... and for N_t <= 128 only
    assert lib.oed_create(ctypes.byref(h), fake, 0, 4 * 160, 4, 160, 1.0, None, ctypes.byref(opt)) == 6
    assert "N_t <= 128" in lib.oed_last_error(None).decode()
    opt.precision = 0
    opt.tile_size = 0
    opt.reserved[0] = 1
    assert lib.oed_create(ctypes.byref(h), fake, 0, 64, 4, 16, 1.0, None, ctypes.byref(opt)) == 1
    assert "reserved" in lib.oed_last_error(None).decode()
