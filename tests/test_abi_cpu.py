"""C-ABI contract checks that need no GPU: the library loads, exports every
declared symbol, and rejects bad arguments on the host before any device work."""
import ctypes as C
import os

import pytest

from paper_2101_03155_amd import ace

LIB = ace.LIB_PATH
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libace.so not built")


def test_exports_every_declared_symbol():
    lib = ace.load()
    names = ace.declared_functions()
    assert {"ace_localize", "ace_pairlist", "ace_build", "ace_apply"} <= set(names)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert b"gfx950" in lib.ace_version()


@pytest.fixture
def ctx():
    lib = ace.load()
    h = C.c_void_p()
    assert lib.ace_create(C.byref(h), None) == 0
    yield lib, h
    lib.ace_destroy(h)


def _grid(n, L=10.0):
    return ace.Grid.cubic(n, L).c()


def test_argument_validation(ctx):
    lib, h = ctx
    g = _grid(24)
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    # norb out of range
    assert lib.ace_build(h, C.byref(g), 0, fake, fake, 1, 0, 0.1, 0, fake, None, None, None, None) == -1
    assert b"norb" in lib.ace_last_error(h)
    assert lib.ace_build(h, C.byref(g), 513, fake, fake, 1, 0, 0.1, 0, fake, None, None, None, None) == -1
    # unsupported grid sizes and shapes
    g7 = _grid(7)
    assert lib.ace_build(h, C.byref(g7), 4, fake, fake, 1, 0, 0.1, 0, fake, None, None, None, None) == -7
    gn = ace.Grid((24, 24, 48), (10.0, 10.0, 20.0)).c()
    assert lib.ace_localize(h, C.byref(gn), 4, fake, fake, fake, None) == -7
    # npairs beyond norb(norb+1)/2, bad kernel, bad precision, erfc without omega
    assert lib.ace_build(h, C.byref(g), 4, fake, fake, 11, 0, 0.1, 0, fake, None, None, None, None) == -1
    assert lib.ace_build(h, C.byref(g), 4, fake, fake, 3, 7, 0.1, 0, fake, None, None, None, None) == -1
    assert lib.ace_build(h, C.byref(g), 4, fake, fake, 3, 0, 0.1, 5, fake, None, None, None, None) == -1
    assert lib.ace_build(h, C.byref(g), 4, fake, fake, 3, 1, 0.0, 0, fake, None, None, None, None) == -1
    # NULL outputs
    assert lib.ace_build(h, C.byref(g), 4, fake, fake, 3, 0, 0.1, 0, None, None, None, None, None) == -1
    n = C.c_int64()
    assert lib.ace_pairlist(h, C.byref(g), 4, fake, 1e-3, -1, fake, None, C.byref(n)) == -1
    assert lib.ace_apply(h, C.byref(g), 4, fake, 0, fake, fake) == -1
    # localization on given columns: NULL arguments and bad grids fail before any device call
    assert lib.ace_localize_pivots(h, C.byref(g), 4, fake, None, fake, None) == -1
    assert lib.ace_localize_pivots(h, C.byref(g), 4, None, fake, fake, None) == -1
    assert lib.ace_localize_pivots(h, C.byref(g), 0, fake, fake, fake, None) == -1
    assert lib.ace_localize_pivots(h, C.byref(g7), 4, fake, fake, fake, None) == -7
    # fused application: energy output required, nvec >= 1
    assert lib.ace_apply_energy(h, C.byref(g), 4, fake, 1, fake, fake, None) == -1
    assert lib.ace_apply_energy(h, C.byref(g), 4, fake, 0, fake, fake, fake) == -1
    # exact exchange: norb, NULL W, bad kernel, precision, erfc without omega, grid
    assert lib.ace_exact_exchange(h, C.byref(g), 0, fake, 0, 0.1, 0, fake, None, None) == -1
    assert lib.ace_exact_exchange(h, C.byref(g), 4, fake, 0, 0.1, 0, None, None, None) == -1
    assert lib.ace_exact_exchange(h, C.byref(g), 4, fake, 7, 0.1, 0, fake, None, None) == -1
    assert lib.ace_exact_exchange(h, C.byref(g), 4, fake, 0, 0.1, 5, fake, None, None) == -1
    assert lib.ace_exact_exchange(h, C.byref(g), 4, fake, 1, 0.0, 0, fake, None, None) == -1
    assert lib.ace_exact_exchange(h, C.byref(g7), 4, fake, 0, 0.1, 0, fake, None, None) == -7
    # non-positive box
    gb = ace.Grid.cubic(24, -1.0).c()
    assert lib.ace_apply(h, C.byref(gb), 4, fake, 1, fake, fake) == -1
    # tuner shape validation
    assert lib.ace_set_pair_shape(h, 0, 7, 1, 8) == -1
    assert lib.ace_set_pair_shape(h, 0, 96, 1, 0) == -1
    assert lib.ace_set_pair_shape(h, 0, 96, 0, 16) == 0
    f, m = C.c_int(), C.c_int()
    assert lib.ace_get_pair_shape(h, 0, 96, C.byref(f), C.byref(m)) == 0
    assert (f.value, m.value) == (0, 16)
    # real-to-complex path: fits FP64 up to 120^3, not 160^3 (half-spectrum plane beyond LDS)
    assert lib.ace_set_pair_shape(h, 0, 96, 2, 16) == 0
    assert lib.ace_get_pair_shape(h, 0, 96, C.byref(f), C.byref(m)) == 0 and f.value == 2
    assert lib.ace_set_pair_shape(h, 0, 160, 2, 16) == 0
    assert lib.ace_get_pair_shape(h, 0, 160, C.byref(f), C.byref(m)) == 0 and f.value == 0
    assert lib.ace_set_pair_shape(h, 1, 160, 2, 16) == 0
    assert lib.ace_get_pair_shape(h, 1, 160, C.byref(f), C.byref(m)) == 0 and f.value == 2
    assert lib.ace_set_pair_shape(h, 0, 96, 3, 16) == 0
    assert lib.ace_get_pair_shape(h, 0, 96, C.byref(f), C.byref(m)) == 0 and f.value == 3
    assert lib.ace_set_pair_shape(h, 0, 96, 4, 16) == -1
    assert lib.ace_set_pair_shape(h, 0, 96, -1, 16) == -1
    # feature stride must be >= 1 and divide the grid size
    assert lib.ace_pair_features(h, C.byref(g), 4, fake, None, 10, fake, 0) == -1
    assert lib.ace_pair_features(h, C.byref(g), 4, fake, None, 10, fake, 5) == -1
    assert lib.ace_profile_read(h, 99, None, None, None, 0) == -1
    assert lib.ace_profile_classes(h, 1 << 20) == -1
    # batched: argument checks before any device work
    arr = (ace.ace_system * 2)()
    for a in arr:
        a.grid = ace.Grid.cubic(24, 8.0).c()
        a.norb, a.kernel, a.omega, a.npairs = 4, 0, 0.1, 3
        a.phi, a.pairs, a.xi = 0x1000, 0x1000, 0x1000
    assert lib.ace_build_batched(h, 0, arr, 1, 0) == -1
    assert lib.ace_build_batched(h, 2, arr, 3, 0) == -1
    assert lib.ace_build_batched(h, 2, arr, 1, 9) == -1
    arr[1].grid = ace.Grid.cubic(120, 8.0).c()
    assert lib.ace_build_batched(h, 2, arr, 1, 0) == -7
    assert b"system 1" in lib.ace_last_error(h)
    arr[1].grid = ace.Grid.cubic(24, 8.0).c()
    arr[0].npairs = 11
    assert lib.ace_build_batched(h, 2, arr, 1, 0) == -1
    assert lib.ace_set_batched_shape(h, 12, 0, 4, 2) == -1
    assert lib.ace_set_batched_shape(h, 8, 1, 4, 1) == -1
    assert lib.ace_set_batched_shape(h, 8, 1, 4, 0) == 0
    assert lib.ace_set_batched_shape(h, 16, 0, 8, 2) == 0
    assert lib.ace_set_batched_shape(h, 16, 0, 8, 3) == 0
    assert lib.ace_set_batched_shape(h, 16, 0, 8, 4) == -1


def test_binding_refuses_without_gpu():
    import torch

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        ace.Context()
