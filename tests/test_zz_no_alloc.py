"""The allocation-free application (ace_apply_energy_noalloc) against
ace_apply_energy: two calls in a row on the shared fixed scratch, the second
with a smaller input, each element by element."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(rng, norb, nvec, n):
    xi = torch.as_tensor(rng.normal(size=(norb, n, n, n)), device="cuda")
    x = torch.as_tensor(rng.normal(size=(nvec, n, n, n)), device="cuda")
    return xi, x


def _noalloc(ctx, lib, xi, x, grid):
    """Through the C ABI directly: caller-owned outputs, no library allocation."""
    y = torch.empty_like(x)
    ex = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx._sync_stream()
    g = grid.c()
    rc = ctx.lib.ace_apply_energy_noalloc(ctx.h, C.byref(g), xi.shape[0], xi.data_ptr(), x.shape[0], x.data_ptr(),
                                          y.data_ptr(), ex.data_ptr())
    assert rc == 0, ctx.lib.ace_last_error(ctx.h).decode()
    return y, ex


def test_noalloc_matches_apply_energy_two_calls(lib):
    from paper_2101_03155_amd import Grid
    ctx = lib.Context()
    rng = np.random.default_rng(77)
    # first call larger (several 128-wide tiles, ragged tails), second smaller
    for norb, nvec, n in ((300, 257, 24), (37, 5, 16)):
        print(f"[gpu-case] noalloc norb={norb} nvec={nvec} N={n}", flush=True)
        grid = Grid.cubic(n, 0.4 * n)
        xi, x = _case(rng, norb, nvec, n)
        y_ref, e_ref = ctx.apply_energy(xi, x, grid)
        y, e = _noalloc(ctx, lib, xi, x, grid)
        torch.cuda.synchronize()
        yr, yn = y_ref.cpu().numpy(), y.cpu().numpy()
        err = np.abs(yn - yr).max() / np.abs(yr).max()
        de = abs(e.item() - e_ref.item()) / abs(e_ref.item())
        print(f"  max elementwise err {err:.2e}, energy rel err {de:.2e}", flush=True)
        assert err <= 1e-13 and de <= 1e-13


def test_noalloc_full_size_and_limits(lib):
    from paper_2101_03155_amd import AceError, Grid
    ctx = lib.Context()
    rng = np.random.default_rng(5)
    grid = Grid.cubic(96, 18.6)
    xi, x = _case(rng, 128, 128, 96)
    y_ref, e_ref = ctx.apply_energy(xi, x, grid)
    y = torch.empty_like(x)
    ex = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.apply_energy_noalloc(xi, x, grid, y, ex)
    err = (y - y_ref).abs().max().item() / y_ref.abs().max().item()
    assert err <= 1e-13 and abs(ex.item() - e_ref.item()) <= 1e-13 * abs(e_ref.item())
    # beyond the fixed scratch: a clear error, nothing launched
    big = torch.empty(513, 8, 8, 8, dtype=torch.float64, device="cuda")
    with pytest.raises(AceError) as ei:
        ctx.apply_energy_noalloc(xi[:, :8, :8, :8].contiguous(), big, Grid.cubic(8, 4.0), torch.empty_like(big), ex)
    assert ei.value.status == "ACE_E_ARG" and "nvec" in str(ei.value)
