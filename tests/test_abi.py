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
    assert list(o.grid)[:4] == [1, 1, 1, 1] and o.lookahead == 2 and o.seed == 0


def test_struct_sizes_match_the_header():
    # tt_options: u64 + 4 i32 + 16 i32 + 3 i32 (+pad) + pointer
    assert C.sizeof(_lib.Options) == 8 + 4 * 4 + 4 * 16 + 4 * 4 + 8
    assert C.sizeof(_lib.Stats) == 3 * 8 + 4 * 4 + 4 * 17 + 4 + 3 * 8 + 8 * 16 + 8 + 4 * 8


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
