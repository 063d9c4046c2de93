"""Thin Python binding of libace (ctypes).

Marshals torch tensors (device memory, the current HIP stream) into the C ABI
declared in include/ace.h; every step of the computation runs in the library's
HIP kernels.  There is no fallback: if libace.so is missing or no GPU is
present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libace.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ace.h")

ACE_OK = 0
STATUS = {0: "ACE_OK", -1: "ACE_E_ARG", -2: "ACE_E_HIP", -3: "ACE_E_NOMEM", -4: "ACE_E_NOT_PD",
          -5: "ACE_E_CAPACITY", -6: "ACE_E_NONFINITE", -7: "ACE_E_UNSUPPORTED"}
KERNELS = {"bare": 0, "coulomb": 0, "erfc": 1}
PRECISIONS = {"fp64": 0, "fp32": 1}
PAIR_PATHS = {"split": 0, "fused": 1, "r2c": 2, "owner": 3}
PAIR_PATH_NAMES = {v: k for k, v in PAIR_PATHS.items()}

# profile classes (see include/ace.h)
KC_FWD_XY, KC_CONV_Z, KC_INV_XY = 0, 1, 2
KC_FWD_X, KC_FWD_Y, KC_INV_Y, KC_INV_X = 3, 4, 5, 6
KC_GEMM_NT, KC_GEMM_TN, KC_QRCP = 7, 8, 9
ST_LOCALIZE, ST_PAIRLIST, ST_PAIRS, ST_TAIL, ST_BUILD = 10, 11, 12, 13, 14


class AceError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class ace_grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3)]


class ace_system(C.Structure):
    _fields_ = [("grid", ace_grid), ("norb", C.c_int32), ("kernel", C.c_int32), ("omega", C.c_double),
                ("phi", C.c_void_p), ("pairs", C.c_void_p), ("npairs", C.c_int64), ("xi", C.c_void_p),
                ("M", C.c_void_p), ("ex", C.c_void_p), ("status", C.c_int32), ("fail_column", C.c_int32)]


BATCHED_MODES = {"graph": 0, "persistent": 1, "eager": 2}

MLP_NPARAM = 4609
MLP_NMODEL = 4631


class ace_step_info(C.Structure):
    _fields_ = [("reused_columns", C.c_int32), ("gram_cond", C.c_double), ("pairs_added", C.c_int64),
                ("pairs_removed", C.c_int64)]


class ace_screen_spec(C.Structure):
    _fields_ = [("mode", C.c_int32), ("rho_cut", C.c_double), ("ex_budget", C.c_double), ("model", C.c_void_p),
                ("ood_tol", C.c_double), ("stride", C.c_int32)]


class ace_mlp_hparams(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("batch", C.c_int32), ("epochs", C.c_int32), ("step0", C.c_int32), ("seed", C.c_uint64)]


@dataclass(frozen=True)
class Grid:
    """Cubic-or-orthorhombic periodic grid: n points and box edge L (bohr) per axis."""

    n: Sequence[int]
    L: Sequence[float]

    @staticmethod
    def cubic(n: int, L: float) -> "Grid":
        return Grid((n, n, n), (L, L, L))

    @property
    def size(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def dV(self) -> float:
        return float(self.L[0]) * float(self.L[1]) * float(self.L[2]) / self.size

    def c(self) -> ace_grid:
        g = ace_grid()
        for d in range(3):
            g.n[d] = int(self.n[d])
            g.L[d] = float(self.L[d])
        return g


_lib = None


def load(path: str = LIB_PATH):
    """Load libace.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it first (python -m paper_2101_03155_amd.build)")
    lib = C.CDLL(path)
    P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
    GP = C.POINTER(ace_grid)
    sig = {
        "ace_version": ([], C.c_char_p),
        "ace_create": ([C.POINTER(P), P], I),
        "ace_destroy": ([P], I),
        "ace_last_error": ([P], C.c_char_p),
        "ace_set_stream": ([P, P], I),
        "ace_localize": ([P, GP, I, P, P, P, P], I),
        "ace_pairlist": ([P, GP, I, P, D, I64, P, P, C.POINTER(I64)], I),
        "ace_localize_step": ([P, GP, I, P, P, D, P, P, C.POINTER(ace_step_info)], I),
        "ace_pairlist_step": ([P, GP, I, P, D, P, I64, I64, P, P, C.POINTER(I64), C.POINTER(ace_step_info)], I),
        "ace_build": ([P, GP, I, P, P, I64, I, D, I, P, P, P, P, P], I),
        "ace_apply": ([P, GP, I, P, I, P, P], I),
        "ace_localize_pivots": ([P, GP, I, P, P, P, P], I),
        "ace_apply_energy": ([P, GP, I, P, I, P, P, P], I),
        "ace_apply_energy_noalloc": ([P, GP, I, P, I, P, P, P], I),
        "ace_exact_exchange": ([P, GP, I, P, I, D, I, P, P, P], I),
        "ace_build_kpoints": ([P, GP, I, I, C.POINTER(D), P, P, I64, I, D, P, P, P, P], I),
        "ace_pairlist_kpoints": ([P, GP, I, P, D, I64, P, P, C.POINTER(I64)], I),
        "ace_profile_enable": ([P, I], I),
        "ace_profile_read": ([P, I, C.POINTER(I64), C.POINTER(D), C.POINTER(D), I], I),
        "ace_profile_classes": ([P, C.c_uint], I),
        "ace_set_pair_shape": ([P, I, I, I, I], I),
        "ace_release_workspace": ([P], I),
        "ace_get_pair_shape": ([P, I, I, C.POINTER(I), C.POINTER(I)], I),
        "ace_build_batched": ([P, I, C.POINTER(ace_system), I, I], I),
        "ace_set_batched_shape": ([P, I, I, I, I], I),
        "ace_pair_features": ([P, GP, I, P, P, I64, P, I], I),
        "ace_pair_energies": ([P, GP, I, P, P, I64, I, D, I, P], I),
        "ace_mlp_init": ([P, P, C.c_uint64], I),
        "ace_mlp_fit_norm": ([P, P, P, P, I64], I),
        "ace_mlp_forward": ([P, P, P, I64, I, P], I),
        "ace_mlp_grad": ([P, P, P, P, I64, P, P], I),
        "ace_mlp_train": ([P, P, P, P, P, P, I64, C.POINTER(ace_mlp_hparams), P], I),
        "ace_screen_learned": ([P, GP, I, P, P, D, D, D, I64, P, C.POINTER(I64), C.POINTER(I), I], I),
        "ace_pairlist_device": ([P, GP, I, P, D, I64, P, P, P], I),
        "ace_screen": ([P, GP, I, P, C.POINTER(ace_screen_spec), I64, P, P, C.POINTER(I64), C.POINTER(I)], I),
        "ace_screener_train": ([P, P, P, I64, C.POINTER(ace_mlp_hparams), P], I),
        "ace_screener_predict": ([P, P, P, I64, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def declared_functions(header: str = HEADER):
    """Names of the functions declared in include/ace.h."""
    txt = open(header).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ace_[a-z_]+)\s*\(", txt)))


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _require(t, dtype, name):
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """An ace_ctx bound to a torch stream (default: the current stream)."""

    def __init__(self, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libace needs a GPU; none is visible")
        self.lib = load()
        self._stream = stream
        h = C.c_void_p()
        s = (stream or torch.cuda.current_stream()).cuda_stream
        rc = self.lib.ace_create(C.byref(h), C.c_void_p(s))
        if rc != ACE_OK:
            raise AceError(rc, "ace_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.ace_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        import torch

        s = (self._stream or torch.cuda.current_stream()).cuda_stream
        self.lib.ace_set_stream(self.h, C.c_void_p(s))

    def _check(self, rc):
        if rc != ACE_OK:
            raise AceError(rc, self.lib.ace_last_error(self.h).decode())

    # ------------------------------------------------------------ API
    def localize(self, psi, grid: Grid):
        """SCDM localization: returns (phi, pivots[int32], U)."""
        import torch

        _require(psi, torch.float64, "psi")
        norb = psi.shape[0]
        phi = torch.empty_like(psi)
        piv = torch.empty(norb, dtype=torch.int32, device=psi.device)
        U = torch.empty(norb, norb, dtype=torch.float64, device=psi.device)
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_localize(self.h, C.byref(g), norb, _ptr(psi), _ptr(phi), _ptr(piv), _ptr(U)))
        return phi, piv, U

    def localize_pivots(self, psi, pivots, grid: Grid):
        """Loewdin step on given columns (e.g. the previous MD step's): returns (phi, U)."""
        import torch

        _require(psi, torch.float64, "psi")
        _require(pivots, torch.int32, "pivots")
        norb = psi.shape[0]
        phi = torch.empty_like(psi)
        U = torch.empty(norb, norb, dtype=torch.float64, device=psi.device)
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_localize_pivots(self.h, C.byref(g), norb, _ptr(psi), _ptr(pivots), _ptr(phi),
                                                 _ptr(U)))
        return phi, U

    def localize_step(self, psi, pivots, grid: Grid, cond_max: float):
        """Next MD step: keep the previous columns (Loewdin only) when their
        diagonal ratio (max R_kk / min R_kk)^2 is <= cond_max, else fresh SCDM.
        Returns (phi, pivots used [new tensor], U, info dict)."""
        import torch

        _require(psi, torch.float64, "psi")
        _require(pivots, torch.int32, "pivots")
        norb = psi.shape[0]
        piv = pivots.clone()
        phi = torch.empty_like(psi)
        U = torch.empty(norb, norb, dtype=torch.float64, device=psi.device)
        info = ace_step_info()
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_localize_step(self.h, C.byref(g), norb, _ptr(psi), _ptr(piv), float(cond_max),
                                               _ptr(phi), _ptr(U), C.byref(info)))
        return phi, piv, U, {"reused_columns": bool(info.reused_columns), "gram_cond": info.gram_cond}

    def pairlist_step(self, phi, grid: Grid, rho_cut: float, prev_pairs):
        """Re-screen against the previous step's list: (pairs, overlap, info)
        with info = pairs_added / pairs_removed relative to prev_pairs."""
        import torch

        _require(phi, torch.float64, "phi")
        _require(prev_pairs, torch.int32, "prev_pairs")
        norb = phi.shape[0]
        cap = norb * (norb + 1) // 2
        pairs = torch.empty(cap, 2, dtype=torch.int32, device=phi.device)
        ov = torch.empty(cap, dtype=torch.float64, device=phi.device)
        n = C.c_int64()
        info = ace_step_info()
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_pairlist_step(self.h, C.byref(g), norb, _ptr(phi), float(rho_cut), _ptr(prev_pairs),
                                               prev_pairs.shape[0], cap, _ptr(pairs), _ptr(ov), C.byref(n),
                                               C.byref(info)))
        return pairs[: n.value], ov[: n.value], {"pairs_added": info.pairs_added, "pairs_removed": info.pairs_removed}

    def pairlist(self, phi, grid: Grid, rho_cut: float, capacity: Optional[int] = None):
        """Screened pair list: returns (pairs[int32, n x 2], overlap[n])."""
        import torch

        _require(phi, torch.float64, "phi")
        norb = phi.shape[0]
        cap = norb * (norb + 1) // 2 if capacity is None else int(capacity)
        pairs = torch.empty(max(cap, 1), 2, dtype=torch.int32, device=phi.device)
        ov = torch.empty(max(cap, 1), dtype=torch.float64, device=phi.device)
        n = C.c_int64()
        self._sync_stream()
        g = grid.c()
        rc = self.lib.ace_pairlist(self.h, C.byref(g), norb, _ptr(phi), float(rho_cut), cap, _ptr(pairs), _ptr(ov),
                                   C.byref(n))
        if rc == -5:
            raise AceError(rc, self.lib.ace_last_error(self.h).decode() + f" (required {n.value})")
        self._check(rc)
        return pairs[: n.value], ov[: n.value]

    def build(self, phi, pairs, grid: Grid, kernel: str = "erfc", omega: float = 0.106, precision: str = "fp64",
              want_M: bool = True, want_W: bool = False, want_energies: bool = False, out=None):
        """ACE build over a pair list: returns dict(xi, M, W, ex, e)."""
        import torch

        _require(phi, torch.float64, "phi")
        _require(pairs, torch.int32, "pairs")
        norb = phi.shape[0]
        npairs = pairs.shape[0]
        dev = phi.device
        o = out or {}
        xi = o.get("xi")
        if xi is None:
            xi = torch.empty_like(phi)
        M = o.get("M") if want_M else None
        if want_M and M is None:
            M = torch.empty(norb, norb, dtype=torch.float64, device=dev)
        W = torch.empty_like(phi) if want_W else None
        ex = o.get("ex")
        if ex is None:
            ex = torch.empty(1, dtype=torch.float64, device=dev)
        e = torch.empty(npairs, dtype=torch.float64, device=dev) if want_energies else None
        self._sync_stream()
        g = grid.c()
        rc = self.lib.ace_build(self.h, C.byref(g), norb, _ptr(phi), _ptr(pairs), npairs, KERNELS[kernel],
                                float(omega), PRECISIONS[precision], _ptr(xi), _ptr(M), _ptr(W), _ptr(ex), _ptr(e))
        self._check(rc)
        return dict(xi=xi, M=M, W=W, ex=ex, e=e)

    def apply(self, xi, x, grid: Grid):
        """y = V_ACE x."""
        import torch

        _require(xi, torch.float64, "xi")
        _require(x, torch.float64, "x")
        y = torch.empty_like(x)
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_apply(self.h, C.byref(g), xi.shape[0], _ptr(xi), x.shape[0], _ptr(x), _ptr(y)))
        return y

    def apply_energy(self, xi, x, grid: Grid, out=None):
        """(y, ex): y = V_ACE x and ex = sum_a <x_a|V_ACE x_a> (device scalar), one pass."""
        import torch

        _require(xi, torch.float64, "xi")
        _require(x, torch.float64, "x")
        o = out or {}
        y = o.get("y")
        if y is None:
            y = torch.empty_like(x)
        ex = o.get("ex")
        if ex is None:
            ex = torch.empty(1, dtype=torch.float64, device=x.device)
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_apply_energy(self.h, C.byref(g), xi.shape[0], _ptr(xi), x.shape[0], _ptr(x),
                                              _ptr(y), _ptr(ex)))
        return y, ex

    def apply_energy_noalloc(self, xi, x, grid: Grid, y, ex):
        """apply_energy into caller-owned y and ex; the library allocates
        nothing (its scratch is a fixed per-device array)."""
        import torch

        _require(xi, torch.float64, "xi")
        _require(x, torch.float64, "x")
        _require(y, torch.float64, "y")
        _require(ex, torch.float64, "ex")
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_apply_energy_noalloc(self.h, C.byref(g), xi.shape[0], _ptr(xi), x.shape[0],
                                                      _ptr(x), _ptr(y), _ptr(ex)))
        return y, ex

    def exact_exchange(self, psi, grid: Grid, kernel: str = "erfc", omega: float = 0.106, precision: str = "fp64",
                       want_M: bool = True, out=None):
        """Exact V_X on every orbital over all pairs: returns dict(W, M, ex)."""
        import torch

        _require(psi, torch.float64, "psi")
        norb = psi.shape[0]
        o = out or {}
        W = o.get("W")
        if W is None:
            W = torch.empty_like(psi)
        M = torch.empty(norb, norb, dtype=torch.float64, device=psi.device) if want_M else None
        ex = o.get("ex")
        if ex is None:
            ex = torch.empty(1, dtype=torch.float64, device=psi.device)
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_exact_exchange(self.h, C.byref(g), norb, _ptr(psi), KERNELS[kernel], float(omega),
                                                PRECISIONS[precision], _ptr(W), _ptr(M), _ptr(ex)))
        return dict(W=W, M=M, ex=ex)

    # ------------------------------------------------------------ complex orbitals, k-points
    def build_kpoints(self, u, kvec, norb: int, pairs, grid: Grid, kernel: str = "erfc", omega: float = 0.106,
                      want_M: bool = True, want_W: bool = False):
        """ACE build of Bloch orbitals: u complex128 [nk * norb, ...grid] (cell-periodic
        parts), kvec [nk][3] (bohr^-1, host sequence).  Returns dict(xi, M, W, ex)."""
        import torch

        _require(u, torch.complex128, "u")
        _require(pairs, torch.int32, "pairs")
        nk = len(kvec)
        kv = (C.c_double * (3 * nk))(*[float(x) for k in kvec for x in k])
        xi = torch.empty_like(u)
        M = torch.empty(nk, norb, norb, dtype=torch.complex128, device=u.device) if want_M else None
        W = torch.empty_like(u) if want_W else None
        ex = torch.empty(1, dtype=torch.float64, device=u.device)
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_build_kpoints(self.h, C.byref(g), norb, nk, kv, _ptr(u), _ptr(pairs), pairs.shape[0],
                                               KERNELS[kernel], float(omega), _ptr(xi), _ptr(M), _ptr(W), _ptr(ex)))
        return dict(xi=xi, M=M, W=W, ex=ex)

    def pairlist_kpoints(self, u, grid: Grid, rho_cut: float):
        """Screened pairs of Bloch orbitals: (pairs[int32, n x 2], overlap[n])."""
        import torch

        _require(u, torch.complex128, "u")
        ntot = u.shape[0]
        cap = ntot * (ntot + 1) // 2
        pairs = torch.empty(cap, 2, dtype=torch.int32, device=u.device)
        ov = torch.empty(cap, dtype=torch.float64, device=u.device)
        n = C.c_int64()
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_pairlist_kpoints(self.h, C.byref(g), ntot, _ptr(u), float(rho_cut), cap, _ptr(pairs),
                                                  _ptr(ov), C.byref(n)))
        return pairs[: n.value], ov[: n.value]

    # ------------------------------------------------------------ timing / tuning
    def profile(self, enable: bool):
        self._check(self.lib.ace_profile_enable(self.h, 1 if enable else 0))

    def profile_classes(self, classes=None):
        """Bracket only the given timing classes (None: all of them)."""
        mask = (1 << 15) - 1 if classes is None else sum(1 << c for c in classes)
        self._check(self.lib.ace_profile_classes(self.h, mask))

    def profile_read(self, cls: int, reset: bool = True):
        """(launches, total milliseconds, total algorithmic units) of a timing class."""
        n = C.c_int64()
        ms = C.c_double()
        u = C.c_double()
        self._check(self.lib.ace_profile_read(self.h, cls, C.byref(n), C.byref(ms), C.byref(u), 1 if reset else 0))
        return n.value, ms.value, u.value

    def release_workspace(self):
        """Free the device workspaces the context has grown."""
        self._check(self.lib.ace_release_workspace(self.h))

    def set_pair_shape(self, precision: str, n: int, path, max_packs: int):
        """path: "split" (or False/0), "fused" (True/1), "r2c" (2) or "owner" (3);
        a path that does not fit the grid size falls back to the split passes."""
        code = PAIR_PATHS[path] if isinstance(path, str) else int(path)
        self._check(self.lib.ace_set_pair_shape(self.h, PRECISIONS[precision], n, code, max_packs))

    def get_pair_shape(self, precision: str, n: int):
        """(path name, max_packs) in effect for this precision and grid size."""
        f = C.c_int()
        m = C.c_int()
        self._check(self.lib.ace_get_pair_shape(self.h, PRECISIONS[precision], n, C.byref(f), C.byref(m)))
        return PAIR_PATH_NAMES[f.value], m.value

    def build_batched(self, systems, precision: str = "fp32", mode: str = "graph", want_M: bool = True,
                      raise_on_not_pd: bool = True):
        """Batched ACE builds.  systems: list of dict(phi, pairs, grid, kernel, omega).

        Returns a list of dict(xi, M, ex, status, fail_column) in input order."""
        import torch

        n = len(systems)
        arr = (ace_system * n)()
        outs = []
        for q, sy in enumerate(systems):
            phi, pairs, grid = sy["phi"], sy["pairs"], sy["grid"]
            _require(phi, torch.float64, f"systems[{q}].phi")
            _require(pairs, torch.int32, f"systems[{q}].pairs")
            norb = phi.shape[0]
            # outputs may be passed in (same buffers => a captured graph is replayed)
            o = dict(xi=sy["xi"] if sy.get("xi") is not None else torch.empty_like(phi),
                     M=(sy["M"] if sy.get("M") is not None else
                        torch.empty(norb, norb, dtype=torch.float64, device=phi.device)) if want_M else None,
                     ex=sy["ex"] if sy.get("ex") is not None else torch.empty(1, dtype=torch.float64,
                                                                               device=phi.device))
            outs.append(o)
            a = arr[q]
            a.grid = grid.c()
            a.norb = norb
            a.kernel = KERNELS[sy.get("kernel", "erfc")]
            a.omega = float(sy.get("omega", 0.106))
            a.phi = phi.data_ptr()
            a.pairs = pairs.data_ptr()
            a.npairs = pairs.shape[0]
            a.xi = o["xi"].data_ptr()
            a.M = _ptr(o["M"])
            a.ex = o["ex"].data_ptr()
        self._sync_stream()
        self._keep = systems  # inputs stay alive for the duration of the call
        rc = self.lib.ace_build_batched(self.h, n, arr, PRECISIONS[precision], BATCHED_MODES[mode])
        for q in range(n):
            outs[q]["status"] = STATUS.get(arr[q].status, arr[q].status)
            outs[q]["fail_column"] = arr[q].fail_column
        if rc == -4 and not raise_on_not_pd:
            return outs
        self._check(rc)
        return outs

    def set_batched_shape(self, txv: int, plan_variant: int, blocks_per_cu: int, layout: str = "owner"):
        """layout: "owner" (all half spectra resident, W formed once per
        row), "r2c" (half spectra, three phases per round) or "split" (five
        passes per round)."""
        code = {"split": 0, "r2c": 2, "owner": 3}[layout]
        self._check(self.lib.ace_set_batched_shape(self.h, txv, plan_variant, blocks_per_cu, code))

    # ------------------------------------------------------------ learned screener
    def pair_features(self, phi, grid: Grid, pairs=None, stride: int = 1):
        """float32 [npairs][5] features (every pair i <= j when pairs is None);
        stride > 1 evaluates the two overlap integrals on the grid subsampled
        by that stride per axis."""
        import torch

        _require(phi, torch.float64, "phi")
        norb = phi.shape[0]
        n = norb * (norb + 1) // 2 if pairs is None else pairs.shape[0]
        if pairs is not None:
            _require(pairs, torch.int32, "pairs")
        f = torch.empty(n, 5, dtype=torch.float32, device=phi.device)
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_pair_features(self.h, C.byref(g), norb, _ptr(phi), _ptr(pairs), n, _ptr(f),
                                               int(stride)))
        return f

    def pair_energies(self, phi, pairs, grid: Grid, kernel: str = "erfc", omega: float = 0.106,
                      precision: str = "fp64"):
        import torch

        _require(phi, torch.float64, "phi")
        _require(pairs, torch.int32, "pairs")
        e = torch.empty(pairs.shape[0], dtype=torch.float64, device=phi.device)
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_pair_energies(self.h, C.byref(g), phi.shape[0], _ptr(phi), _ptr(pairs),
                                               pairs.shape[0], KERNELS[kernel], float(omega), PRECISIONS[precision],
                                               _ptr(e)))
        return e

    def mlp_init(self, seed: int = 0):
        import torch

        m = torch.empty(MLP_NMODEL, dtype=torch.float32, device="cuda")
        self._sync_stream()
        self._check(self.lib.ace_mlp_init(self.h, _ptr(m), C.c_uint64(seed)))
        return m

    def mlp_fit_norm(self, model, x, t):
        self._sync_stream()
        self._check(self.lib.ace_mlp_fit_norm(self.h, _ptr(model), _ptr(x), _ptr(t), x.shape[0]))

    def mlp_forward(self, model, x, clamp: bool = False):
        import torch

        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        self._sync_stream()
        self._check(self.lib.ace_mlp_forward(self.h, _ptr(model), _ptr(x), x.shape[0], 1 if clamp else 0, _ptr(y)))
        return y

    def mlp_grad(self, model, x, t):
        import torch

        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        self._sync_stream()
        self._check(self.lib.ace_mlp_grad(self.h, _ptr(model), _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss)))
        return g, loss

    def mlp_train(self, model, adam_m, adam_v, x, t, lr=1e-3, batch=4096, epochs=10, seed=0, step0=0,
                  beta1=0.9, beta2=0.999, eps=1e-8):
        import torch

        hp = ace_mlp_hparams(lr, beta1, beta2, eps, batch, epochs, step0, seed)
        curve = torch.empty(epochs, dtype=torch.float32, device=x.device)
        self._sync_stream()
        self._check(self.lib.ace_mlp_train(self.h, _ptr(model), _ptr(adam_m), _ptr(adam_v), _ptr(x), _ptr(t),
                                           x.shape[0], C.byref(hp), _ptr(curve)))
        return curve

    def pairlist_device(self, phi, grid: Grid, rho_cut: float, capacity: Optional[int] = None):
        """Screening with the count left on the device and no host wait:
        returns (pairs buffer [capacity, 2], overlap buffer, npairs device int64 [1])."""
        import torch

        _require(phi, torch.float64, "phi")
        norb = phi.shape[0]
        cap = norb * (norb + 1) // 2 if capacity is None else int(capacity)
        pairs = torch.empty(max(cap, 1), 2, dtype=torch.int32, device=phi.device)
        ov = torch.empty(max(cap, 1), dtype=torch.float64, device=phi.device)
        n = torch.empty(1, dtype=torch.int64, device=phi.device)
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_pairlist_device(self.h, C.byref(g), norb, _ptr(phi), float(rho_cut), cap, _ptr(pairs),
                                                 _ptr(ov), _ptr(n)))
        return pairs, ov, n

    def screen(self, phi, grid: Grid, rho_cut: float = 1e-3, model=None, budget: float = 0.0, ood_tol: float = 0.05,
               stride: int = 1):
        """One call for both rules: the overlap rule (model None) or the learned
        rule with the overlap rule as fallback.  Returns (pairs, used_fallback)."""
        import torch

        _require(phi, torch.float64, "phi")
        norb = phi.shape[0]
        cap = norb * (norb + 1) // 2
        pairs = torch.empty(cap, 2, dtype=torch.int32, device=phi.device)
        sc = ace_screen_spec(0 if model is None else 1, float(rho_cut), float(budget), _ptr(model), float(ood_tol),
                             int(stride))
        n = C.c_int64()
        fb = C.c_int()
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_screen(self.h, C.byref(g), norb, _ptr(phi), C.byref(sc), cap, _ptr(pairs), None,
                                        C.byref(n), C.byref(fb)))
        return pairs[: n.value], bool(fb.value)

    def screener_train(self, state, x, t, lr=1e-3, batch=4096, epochs=10, seed=0, step0=0, beta1=0.9, beta2=0.999,
                       eps=1e-8):
        """Adam training on one state array (model, then the two Adam moments)."""
        hp = ace_mlp_hparams(lr, beta1, beta2, eps, batch, epochs, step0, seed)
        self._sync_stream()
        self._check(self.lib.ace_screener_train(self.h, _ptr(x), _ptr(t), x.shape[0], C.byref(hp), _ptr(state)))

    def screener_predict(self, state, x):
        import torch

        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        self._sync_stream()
        self._check(self.lib.ace_screener_predict(self.h, _ptr(state), _ptr(x), x.shape[0], _ptr(y)))
        return y

    def screen_learned(self, phi, grid: Grid, model, budget: float, rho_cut_fallback: float = 1e-3,
                       ood_tol: float = 0.05, stride: int = 1):
        """Learned pair list: returns (pairs[int32, n x 2], used_fallback)."""
        import torch

        _require(phi, torch.float64, "phi")
        norb = phi.shape[0]
        cap = norb * (norb + 1) // 2
        pairs = torch.empty(cap, 2, dtype=torch.int32, device=phi.device)
        n = C.c_int64()
        fb = C.c_int()
        self._sync_stream()
        g = grid.c()
        self._check(self.lib.ace_screen_learned(self.h, C.byref(g), norb, _ptr(phi), _ptr(model), float(budget),
                                                float(rho_cut_fallback), float(ood_tol), cap, _ptr(pairs),
                                                C.byref(n), C.byref(fb), int(stride)))
        return pairs[: n.value], bool(fb.value)

