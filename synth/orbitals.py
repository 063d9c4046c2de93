"""Water-like synthetic occupied-orbital sets on a periodic real-space grid.

The paper benchmarks bulk water: 32 molecules in a 9.85 Angstrom cubic cell
(about 29.9 A^3 per molecule) with four doubly occupied valence orbitals per
molecule (Sec. "Computational details", benchmark subsection).  The paper's
orbitals come from a plane-wave DFT code that is not available here, so every
input is drawn synthetically with the same box sizes, orbital counts and
locality:

* each "molecule" carries four normalized periodic Gaussians
  exp(-|r - c|^2 / (2 sigma^2)), summed over the 27 nearest periodic images,
  whose centres sit ``offset`` bohr from the molecular centre along seeded
  random unit directions;
* molecular centres are uniform in the box (tiny configurations) or on a
  jittered simple lattice (bulk-like configurations);
* the Gaussians are mixed by a seeded Haar-random orthogonal matrix, so the
  resulting canonical orbitals are delocalized, and then Loewdin-orthonormalized
  on the grid, so that sum_r psi_i(r) psi_j(r) dV = delta_ij.

Random draws happen in a fixed order from ``numpy.random.default_rng(seed)``:
centres, jitter, directions, mixing matrix (and, for the batched systems, the
Coulomb-kernel choice).  Consecutive steps of an MD-like trajectory
(``md_step``) move every Gaussian centre along a fixed seeded direction and
keep the mixing matrix, so the orbitals of step t + 1 are a small
displacement of those of step t.

Grid layout: ``psi[orb, z, y, x]`` (x fastest), FP64, bohr^-3/2.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

BOHR_PER_ANGSTROM = 1.8897261246
VOLUME_PER_MOLECULE_A3 = 29.9
ORBITALS_PER_MOLECULE = 4

#: lattice shapes tried in order; the first with capacity >= n_mol is used
_LATTICES = [(2, 2, 2), (4, 2, 2), (4, 4, 2), (4, 4, 4), (8, 4, 4)]


@dataclass(frozen=True)
class SystemSpec:
    """Recipe for one synthetic system (all lengths in bohr)."""

    n_mol: int
    L: float
    N: int
    sigma: float = 1.0
    offset: float = 0.8
    placement: str = "lattice"  # "lattice" or "uniform"
    jitter: float = 0.5
    seed: int = 0
    kernel: str = "erfc"  # "bare" or "erfc"
    omega: float = 0.106
    lattice: Optional[tuple] = None
    #: MD-like trajectory: at step t every Gaussian centre has moved by
    #: t * md_disp bohr along its own seeded unit direction (drawn from a
    #: generator of its own, so step 0 is the plain system)
    md_step: int = 0
    md_disp: float = 0.05

    @property
    def norb(self) -> int:
        return ORBITALS_PER_MOLECULE * self.n_mol

    @property
    def n_grid(self) -> int:
        return self.N ** 3

    @property
    def dV(self) -> float:
        return (self.L / self.N) ** 3

    def replace(self, **kw) -> "SystemSpec":
        return dataclasses.replace(self, **kw)


@dataclass
class OrbitalSet:
    spec: SystemSpec
    psi: object  # numpy array (norb, N, N, N) or torch tensor on a device
    mol_centres: np.ndarray  # (n_mol, 3)
    gauss_centres: np.ndarray  # (norb, 3), wrapped into [0, L)
    mixing: np.ndarray  # (norb, norb) Haar orthogonal matrix Q
    cond_S: float  # condition number of the Gaussian overlap matrix
    kernel: str = "erfc"
    extra: dict = field(default_factory=dict)


def box_length_for(n_mol: int) -> float:
    """Cubic box edge (bohr) at 29.9 A^3 per molecule."""
    return (n_mol * VOLUME_PER_MOLECULE_A3) ** (1.0 / 3.0) * BOHR_PER_ANGSTROM


def lattice_dims(n_mol: int) -> tuple:
    for lat in _LATTICES:
        if lat[0] * lat[1] * lat[2] >= n_mol:
            return lat
    raise ValueError(f"no lattice holds {n_mol} molecules")


def _smooth_235(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def batched_grid_for(L: float) -> int:
    """Smallest N in {48, 64, 80, 96} with spacing L/N <= 0.25 bohr."""
    for n in (48, 64, 80, 96):
        if L / n <= 0.25:
            return n
    return 96


def training_grid_for(L: float) -> int:
    """Smallest even 2,3,5-smooth N with L/N <= 0.196 bohr."""
    n = int(np.ceil(L / 0.196))
    while n % 2 or not _smooth_235(n):
        n += 1
    return n


CONFIGS = {
    # tiny: 2 molecules at uniform positions, bare Coulomb
    "c1": SystemSpec(n_mol=2, L=8.0, N=24, sigma=0.9, offset=0.8, placement="uniform",
                     seed=1001, kernel="bare"),
    # 32 waters: 128 orbitals on 96^3, erfc-screened kernel
    "c2": SystemSpec(n_mol=32, L=18.6, N=96, sigma=1.0, offset=0.8, placement="lattice",
                     jitter=0.5, seed=2001, kernel="erfc", omega=0.106),
    # 64 waters: 256 orbitals on 120^3
    "c3": SystemSpec(n_mol=64, L=23.4, N=120, sigma=1.0, offset=0.8, placement="lattice",
                     jitter=0.5, seed=3001, kernel="erfc", omega=0.106),
    # 128 waters: 512 orbitals on 160^3
    "c5": SystemSpec(n_mol=128, L=29.6, N=160, sigma=1.0, offset=0.8, placement="lattice",
                     jitter=0.5, seed=5001, kernel="erfc", omega=0.106),
}


def config_spec(name: str) -> SystemSpec:
    return CONFIGS[name]


def batched_specs(n_systems: int = 16, master_seed: int = 4000) -> List[SystemSpec]:
    """Uneven batch: n_mol ~ U{8..64}; box from density; grid from spacing."""
    rng = np.random.default_rng(master_seed)
    sizes = rng.integers(8, 65, size=n_systems)
    kinds = rng.random(n_systems)
    out = []
    for k, (n_mol, u) in enumerate(zip(sizes, kinds)):
        L = box_length_for(int(n_mol))
        out.append(SystemSpec(n_mol=int(n_mol), L=L, N=batched_grid_for(L), sigma=1.0,
                              offset=0.8, placement="lattice", jitter=0.5,
                              seed=master_seed + 1 + k,
                              kernel="bare" if u < 0.5 else "erfc", omega=0.106))
    return out


def training_specs(n_configs: int = 200, first_seed: int = 6000,
                   min_mol: int = 32, max_mol: int = 64, kernel: str = "erfc") -> List[SystemSpec]:
    """Training configurations for the learned pair screener (32-64 molecules)."""
    out = []
    for k in range(n_configs):
        seed = first_seed + k
        n_mol = int(np.random.default_rng(seed + 1_000_000).integers(min_mol, max_mol + 1))
        L = box_length_for(n_mol)
        out.append(SystemSpec(n_mol=n_mol, L=L, N=training_grid_for(L), sigma=1.0,
                              offset=0.8, placement="lattice", jitter=0.5, seed=seed,
                              kernel=kernel, omega=0.106))
    return out


def batched_like_specs(n_configs: int, first_seed: int, kernel: str = "erfc",
                       min_mol: int = 8, max_mol: int = 64) -> List[SystemSpec]:
    """Held-out systems drawn like the batched workload (8-64 molecules, box
    from the density, grid spacing <= 0.25 bohr), one kernel: calibration
    systems for a screener that will serve such batches."""
    out = []
    for k in range(n_configs):
        seed = first_seed + k
        n_mol = int(np.random.default_rng(seed + 2_000_000).integers(min_mol, max_mol + 1))
        L = box_length_for(n_mol)
        out.append(SystemSpec(n_mol=n_mol, L=L, N=batched_grid_for(L), sigma=1.0,
                              offset=0.8, placement="lattice", jitter=0.5, seed=seed,
                              kernel=kernel, omega=0.106))
    return out


def _haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    z = rng.normal(size=(n, n))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))[None, :]


def _draw_geometry(spec: SystemSpec, rng: np.random.Generator):
    L = spec.L
    if spec.placement == "uniform":
        centres = rng.uniform(0.0, L, size=(spec.n_mol, 3))
    elif spec.placement == "lattice":
        lat = spec.lattice or lattice_dims(spec.n_mol)
        cap = lat[0] * lat[1] * lat[2]
        order = rng.permutation(cap)[: spec.n_mol]
        ia, rem = np.divmod(order, lat[1] * lat[2])
        ib, ic = np.divmod(rem, lat[2])
        cell = np.array([L / lat[0], L / lat[1], L / lat[2]])
        centres = (np.stack([ia, ib, ic], axis=1) + 0.5) * cell[None, :]
        centres = centres + rng.normal(0.0, spec.jitter, size=(spec.n_mol, 3))
    else:
        raise ValueError(spec.placement)
    gc = np.empty((spec.n_mol, ORBITALS_PER_MOLECULE, 3))
    for m in range(spec.n_mol):
        while True:
            d = rng.normal(size=(ORBITALS_PER_MOLECULE, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            pts = centres[m][None, :] + spec.offset * d
            dist = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
            iu = np.triu_indices(ORBITALS_PER_MOLECULE, 1)
            if dist[iu].min() >= 0.5:
                break
        gc[m] = pts
    gauss_centres = np.mod(gc.reshape(-1, 3), L)
    return np.mod(centres, L), gauss_centres


def _factors_1d(spec: SystemSpec, centres: np.ndarray) -> np.ndarray:
    """Per-Gaussian, per-axis periodic profiles s[a, d, x] (27-image sum)."""
    L, N, s = spec.L, spec.N, spec.sigma
    x = np.arange(N) * (L / N)
    out = np.zeros((centres.shape[0], 3, N))
    for n in (-1, 0, 1):
        diff = x[None, None, :] - centres[:, :, None] - n * L
        out += np.exp(-(diff * diff) / (2.0 * s * s))
    return out


def make_orbitals(spec: SystemSpec, device=None) -> OrbitalSet:
    """Draw one orbital set.  ``device`` (a torch device) assembles psi there.

    The final assembly psi = C^T G^T (C = Q (Q^T S Q)^-1/2) is a dense product;
    on a GPU device it runs in torch FP64, elsewhere in NumPy FP64.  Either way the
    seeded draws and the small matrices are identical.
    """
    rng = np.random.default_rng(spec.seed)
    mol_centres, gauss_centres = _draw_geometry(spec, rng)
    if spec.md_step:
        d = np.random.default_rng([spec.seed, 7919]).normal(size=gauss_centres.shape)
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        gauss_centres = np.mod(gauss_centres + (spec.md_step * spec.md_disp) * d, spec.L)
    q = _haar_orthogonal(rng, spec.norb)
    kernel = spec.kernel
    if spec.kernel == "mixed":
        kernel = "bare" if rng.random() < 0.5 else "erfc"

    f = _factors_1d(spec, gauss_centres)  # (norb, 3, N)
    dV = spec.dV
    # normalize each Gaussian on the grid: dV * prod_d sum_x f_d(x)^2 = 1
    norm2 = dV * np.prod(np.einsum("adx,adx->ad", f, f), axis=1)
    scale = 1.0 / np.sqrt(norm2)
    # overlap of the normalized Gaussians on the grid (the grid sum factorizes)
    ov = np.einsum("adx,bdx->abd", f, f)
    S = dV * np.prod(ov, axis=2) * scale[:, None] * scale[None, :]
    evals_S = np.linalg.eigvalsh(S)
    cond_S = float(evals_S[-1] / evals_S[0])
    T = q.T @ S @ q
    w, V = np.linalg.eigh(T)
    C = q @ (V @ np.diag(w ** -0.5) @ V.T)  # (norb_gauss, norb_orb)
    Cs = C * scale[:, None]
    N = spec.N

    if device is None or str(device) == "cpu":
        gt = (f[:, 2, :, None, None] * f[:, 1, None, :, None]) * f[:, 0, None, None, :]
        psi = (Cs.T @ gt.reshape(spec.norb, -1)).reshape(spec.norb, N, N, N)
    else:
        import torch

        ft = torch.as_tensor(f, dtype=torch.float64, device=device)
        gt = (ft[:, 2, :, None, None] * ft[:, 1, None, :, None]) * ft[:, 0, None, None, :]
        ct = torch.as_tensor(np.ascontiguousarray(Cs.T), dtype=torch.float64, device=device)
        psi = (ct @ gt.reshape(spec.norb, -1)).reshape(spec.norb, N, N, N)
        del gt
    return OrbitalSet(spec=spec, psi=psi, mol_centres=mol_centres,
                      gauss_centres=gauss_centres, mixing=q, cond_S=cond_S, kernel=kernel)


def smooth_test_vectors(spec: SystemSpec, n: int = 16, seed: int = 7) -> np.ndarray:
    """Seeded smooth test functions (sums of 3 broad periodic Gaussians), unit norm."""
    rng = np.random.default_rng(seed)
    N, L = spec.N, spec.L
    x = np.arange(N) * (L / N)
    out = np.zeros((n, N, N, N))
    for k in range(n):
        for _ in range(3):
            c = rng.uniform(0, L, size=3)
            s = rng.uniform(1.2, 2.5)
            amp = rng.normal()
            prof = np.zeros((3, N))
            for m in (-1, 0, 1):
                prof += np.exp(-((x[None, :] - c[:, None] - m * L) ** 2) / (2 * s * s))
            out[k] += amp * prof[2][:, None, None] * prof[1][None, :, None] * prof[0][None, None, :]
        out[k] /= np.sqrt(np.sum(out[k] ** 2) * spec.dV)
    return out


def disjoint_gaussians(spec: SystemSpec, centres: Sequence) -> np.ndarray:
    """Normalized, non-overlapping-by-construction Gaussians at given centres
    (for special-case tests; orthonormality holds only up to their tails)."""
    c = np.mod(np.asarray(centres, dtype=float), spec.L)
    f = _factors_1d(spec, c)
    g = (f[:, 2, :, None, None] * f[:, 1, None, :, None]) * f[:, 0, None, None, :]
    g /= np.sqrt((g * g).sum(axis=(1, 2, 3)) * spec.dV)[:, None, None, None]
    return g


def _haar_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def make_bloch_orbitals(spec: SystemSpec, kfrac: Sequence, mix: bool = True) -> tuple:
    """Complex Bloch orbitals on a k-point sampling, by their cell-periodic parts.

    The molecules and Gaussians are drawn as by make_orbitals.  For each
    k-point k = 2 pi kfrac / L each Gaussian g becomes the Bloch sum
    sum_R exp(i k.R) g(r - R) over the 27 nearest images, whose cell-periodic
    part is exp(-i k.r) times it; the norb sums of each k-point are mixed by a
    seeded Haar-random unitary matrix (mix=True; the draw happens either way)
    and Loewdin-orthonormalized on the grid.  Unmixed, the orbitals stay
    localized, as localized orbitals are for the screening criterion.
    Returns (u complex [n_k * norb][N][N][N], a = q * norb + m;
    kvec [n_k][3] in bohr^-1)."""
    rng = np.random.default_rng(spec.seed)
    _, gauss_centres = _draw_geometry(spec, rng)
    L, N, s = spec.L, spec.N, spec.sigma
    x = np.arange(N) * (L / N)
    kf = np.asarray(kfrac, dtype=np.float64).reshape(-1, 3)
    kvec = 2.0 * np.pi * kf / L
    out = np.empty((len(kf) * spec.norb, N, N, N), dtype=np.complex128)
    for q, k in enumerate(kvec):
        prof = np.zeros((spec.norb, 3, N), dtype=np.complex128)
        for n in (-1, 0, 1):
            diff = x[None, None, :] - gauss_centres[:, :, None] - n * L
            prof += np.exp(1j * k[None, :, None] * n * L) * np.exp(-(diff * diff) / (2.0 * s * s))
        prof *= np.exp(-1j * k[None, :, None] * x[None, None, :])
        ov = np.einsum("adx,bdx->abd", np.conj(prof), prof)
        S = spec.dV * np.prod(ov, axis=2)
        U = _haar_unitary(rng, spec.norb)
        if not mix:
            U = np.eye(spec.norb)
        w, V = np.linalg.eigh(U.conj().T @ S @ U)
        C = U @ (V @ np.diag(w ** -0.5) @ V.conj().T)
        g = (prof[:, 2, :, None, None] * prof[:, 1, None, :, None]) * prof[:, 0, None, None, :]
        out[q * spec.norb:(q + 1) * spec.norb] = (C.T @ g.reshape(spec.norb, -1)).reshape(spec.norb, N, N, N)
    return out, kvec
