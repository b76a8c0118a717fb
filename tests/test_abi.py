"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2407_11290_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w \*]*?\b(tt_\w+)\s*\(", text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    # the Python binding declares exactly the header's functions
    assert set(names) == set(_lib.SIGNATURES)


def test_options_defaults():
    from paper_2407_11290_amd.api import default_options
    o = default_options()
    assert o.r_max == 64 and o.n_samples == 16384 and o.precision == _lib.PREC_AUTO
    assert list(o.grid)[:4] == [1, 1, 1, 1] and o.lookahead == 2 and o.seed == 0 and o.verify == -1


def test_struct_sizes_match_the_header():
    # tt_options: u64 + 4 i32 + 16 i32 + 4 i32 + pointer + 3 i32 (+ pad to 8)
    assert C.sizeof(_lib.Options) == 8 + 4 * 4 + 4 * 16 + 4 * 4 + 8 + 3 * 4 + 4
    assert C.sizeof(_lib.Stats) == 3 * 8 + 4 * 4 + 4 * 17 + 4 + 3 * 8 + 8 * 16 + 8 + 4 * 8 + 8 + 2 * 4 + 2 * 4


@pytest.mark.parametrize("args,code", [
    ((1, [4], 1e-6, 1), _lib.EINVAL),                 # d < 2
    ((3, [4, 0, 4], 1e-6, 1), _lib.EINVAL),           # empty mode
    ((3, [4, 4, 4], -1.0, 1), _lib.EINVAL),           # eps < 0
    ((3, [4, 4, 4], 1e-6, 99), _lib.EFN),             # unknown function
    ((5, [4] * 5, 1e-6, 2), _lib.EFN),                # Maxwellian needs d = 6
])
def test_create_rejects_bad_arguments(args, code):
    lib = _lib.load()
    d, n, eps, fn = args
    arr = (C.c_int32 * len(n))(*n)
    h = lib.tt_cross_create(d, arr, eps, fn, None, 0)
    assert not h
    assert _lib.last_error()


def test_create_and_options_validation_without_gpu():
    from paper_2407_11290_amd.api import TTCross
    t = TTCross([8, 8, 8], 1e-8, _lib.FN_HILBERT)
    with pytest.raises(_lib.TTError):
        TTCross([8, 8, 8], 1e-8, _lib.FN_HILBERT, r_max=65)
    with pytest.raises(_lib.TTError) as e:
        t.ranks()
    assert e.value.code == _lib.ESTATE
    t.close()


def test_run_fails_loudly_without_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2407_11290_amd.api import TTCross
    t = TTCross([8, 8, 8], 1e-8, _lib.FN_HILBERT)
    with pytest.raises(_lib.TTError) as e:
        t.run()
    assert e.value.code == _lib.EDEVICE


def test_batch_rejects_bad_arguments_before_any_device_work():
    from paper_2407_11290_amd.api import TTCross, batch_run
    a = TTCross([8, 8, 8], 1e-8, _lib.FN_HILBERT)
    b = TTCross([8, 8], 1e-8, _lib.FN_HILBERT)
    with pytest.raises(_lib.TTError) as e:
        batch_run([a, b, a])
    assert e.value.code == _lib.EINVAL and "handle 2 appears twice" in _lib.last_error()
    L = _lib.load()
    assert L.tt_batch_run(None, 3, None) == _lib.EINVAL
    assert L.tt_batch_run(None, 0, None) == _lib.OK
    a.close()
    b.close()


def test_batch_statuses_without_gpu():
    """tt_batch_statuses reads host state only: each handle's status as
    tt_cross_get_stats reports it, and EINVAL for bad arrays."""
    import ctypes as C
    from paper_2407_11290_amd.api import TTCross
    a = TTCross([8, 8, 8], 1e-8, _lib.FN_HILBERT)
    b = TTCross([8, 8], 1e-8, _lib.FN_HILBERT)
    L = _lib.load()
    arr = (C.c_void_p * 2)(a.h, b.h)
    st = (C.c_int32 * 2)(7, 7)
    assert L.tt_batch_statuses(arr, 2, st) == _lib.OK
    assert list(st) == [a.stats()["status"], b.stats()["status"]]
    assert L.tt_batch_statuses(None, 2, st) == _lib.EINVAL
    assert L.tt_batch_statuses(arr, 2, None) == _lib.EINVAL
    assert L.tt_batch_statuses(arr, -1, st) == _lib.EINVAL
    assert L.tt_batch_statuses(None, 0, None) == _lib.OK
    assert L.tt_batch_statuses((C.c_void_p * 2)(a.h, None), 2, st) == _lib.EINVAL
    a.close()
    b.close()


def test_tile_options_and_tuner_arguments_without_gpu():
    """Tile shapes outside what the search kernel supports are refused when
    set; the tuners check their arguments before any device work."""
    from paper_2407_11290_amd.api import TTCross, tile_table, tile_table_clear
    for bad in ({"tile_cols": 128}, {"tile_cols": -1}, {"tile_rows": 257}):
        with pytest.raises(_lib.TTError) as e:
            TTCross([8, 8, 8], 1e-8, _lib.FN_HILBERT, **bad)
        assert e.value.code == _lib.EINVAL
    t = TTCross([8, 8, 8], 1e-8, _lib.FN_HILBERT, tile_rows=256, tile_cols=64)
    with pytest.raises(_lib.TTError) as e:
        t.tiles()
    assert e.value.code == _lib.ESTATE
    L = _lib.load()
    assert L.tt_autotune(None, 3, None, None, None) == _lib.EINVAL
    assert L.tt_autotune(t.h, 0, None, None, None) == _lib.EINVAL
    assert L.tt_batch_autotune(None, 2, 1, 1, None) == _lib.EINVAL
    assert L.tt_batch_autotune(None, 0, 1, 1, None) == 0
    arr = (C.c_void_p * 1)(t.h)
    assert L.tt_batch_autotune(arr, 1, 1, 0, None) == _lib.EINVAL
    tile_table_clear()
    assert tile_table() == [] and L.tt_tile_table(None, 0) == 0
    t.close()


def test_server_refuses_rook_pivoting_without_gpu():
    """Served solves use greedy pivoting; the check comes before device work."""
    from paper_2407_11290_amd.api import default_options
    o = default_options()
    o.pivot_mode = _lib.PIVOT_ROOK
    s = _lib.load().tt_server_create(1 << 30, 4, C.byref(o))
    assert not s and "rook" in _lib.last_error()


def test_rank_caps_arguments_without_gpu():
    from paper_2407_11290_amd.api import TTCross
    t = TTCross([8, 8, 8, 8], 1e-8, _lib.FN_HILBERT)
    t.set_rank_caps([3, 0, 64])
    t.set_rank_caps(None)
    for bad in ([3, -1, 2], [3, 65, 2]):
        with pytest.raises(_lib.TTError) as e:
            t.set_rank_caps(bad)
        assert e.value.code == _lib.EINVAL
    assert _lib.load().tt_cross_set_rank_caps(None, None) == _lib.EINVAL
    t.close()


def test_workload_lists_are_seeded_and_shaped_as_specified():
    from paper_2407_11290_amd.workloads import FN_BIMAXWELL, FN_HILBERT, batch_mix, served_trace
    a, b = batch_mix(), batch_mix()
    assert len(a) == 512 and [p.n for p in a] == [p.n for p in b] and [p.params for p in a] == [p.params for p in b]
    for i, p in enumerate(a):
        assert 3 <= p.d <= 6 and len(set(p.n)) == 1 and p.n[0] in (16, 32, 64, 128)
        assert p.seed == i and p.eps == 1e-6
        if i % 2 == 0:
            assert p.fn_id == FN_HILBERT and 0.0 <= p.params[0] <= 4.0
        else:
            assert p.fn_id == FN_BIMAXWELL and len(p.params) == 11
            for m in range(2):
                rho, ux, uy, uz, T = p.params[5 * m: 5 * m + 5]
                assert 0.5 <= rho <= 2.0 and 0.5 <= T <= 2.0 and all(-2 <= x <= 2 for x in (ux, uy, uz))
    t = served_trace(count=200)
    arr = [p.arrival_s for p in t]
    assert all(x < y for x, y in zip(arr, arr[1:]))
    assert {p.eps for p in t} <= {1e-4, 1e-8} and all(4 <= p.d <= 6 for p in t)


def test_server_stats_struct_and_no_gpu_failure():
    assert C.sizeof(_lib.ServerStats) == 7 * 8
    import torch
    L = _lib.load()
    assert not L.tt_server_create(0, 4, None)                 # no budget
    assert not L.tt_server_create(1 << 30, 0, None)           # no slots
    if not torch.cuda.is_available():
        from paper_2407_11290_amd.api import Server
        with pytest.raises(_lib.TTError):
            Server(1 << 30)


def test_fn_eval_kernel_time_argument_checks():
    # neither call reaches the GPU: a NULL output pointer, and (in a process
    # that has not evaluated anything) no time to report
    lib = _lib.load()
    assert lib.tt_fn_eval_last_kernel_ms(None) == _lib.EINVAL
    ms = C.c_double(-5.0)
    rc = lib.tt_fn_eval_last_kernel_ms(C.byref(ms))
    if rc == _lib.ESTATE:
        assert ms.value == -5.0
    else:
        assert rc == _lib.OK and ms.value > 0.0
