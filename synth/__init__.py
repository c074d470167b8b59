"""Seeded synthetic inputs for the ISDF-SMW dielectric inverse.

This module is shared by the CPU oracle, the tests and the benchmark.  It
draws inputs only: orbitals, band energies, interpolation points and the
plane-wave (Miller index) list.  It holds none of the method's arithmetic
(no pair products, no fitting, no Coulomb kernel, no inversion).

The paper's test systems (Si8 .. Si64, (SrTiO3)8, C60 from KSSOLV, Table S1)
are not available, so these stand in for them with the same ratios:
Nr / Ne between 100 and 1000 (abstract) and N_mu = k_mu sqrt(Nv Nc) with
k_mu of order ten (ISDF section).

Recipe:
  * grid: n^3 points in a cubic box of side L = 10.26 (Nv/8)^(1/3) Bohr
    (the Si conventional cell at constant density); grid index
    k = i0 + n*(i1 + n*i2), i0 fastest (x).
  * low-pass set S: integer frequency vectors m in [-n/2, n/2)^3 with
    |m|^2 <= s_cut, s_cut the smallest value giving |S| >= 2 (Nv + Nc).
  * complex orbitals: complex Gaussian coefficients on S, orthonormalised by
    QR in coefficient space, mapped to the grid by the unitary inverse DFT;
    the columns are orthonormal in the plain grid inner product.
  * real orbitals: real Gaussian noise on the grid, low-pass filtered to S,
    real part, thin QR.
  * energies: eps_v ~ U[-20, -5] eV, eps_c ~ U[1, 30] eV, each sorted
    ascending, converted to Hartree.
  * draw order from numpy.random.default_rng(seed): orbital noise, eps_v,
    eps_c, point-selection sketch.
  * interpolation points: column-pivoted QR of a random sketch of the pair
    products (the paper names QRCP as one choice of points); the index list
    is an input shared by both sides, so pivot ties never affect parity.
  * plane waves: Miller vectors m in [-n/2, n/2)^3 sorted by
    (|m|^2, m_x, m_y, m_z) ascending; the first NG are kept.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg

HARTREE_EV = 27.211386245988

# name -> (n, nv, nc, nmu, ng, complex, seed)
CONFIGS = {
    # Static, plain FP64: 12^3 grid, real orbitals, 8/24 states, 96 points, 256 PWs.
    "cfg0": dict(n=12, nv=8, nc=24, nmu=96, ng=256, complex=False, seed=0),
    # Static: 48^3 grid, complex orbitals, 64/256 states, 640 points, 4096 PWs.
    "cfg1": dict(n=48, nv=64, nc=256, nmu=640, ng=4096, complex=True, seed=1),
    # Static, solid-like: 64^3 grid, 256/1024 states, 2048 points, 8192 PWs.
    "cfg2": dict(n=64, nv=256, nc=1024, nmu=2048, ng=8192, complex=True, seed=2),
    # Small cases for parity tests (several tiles plus ragged tails).
    "mid": dict(n=20, nv=12, nc=36, nmu=150, ng=500, complex=True, seed=5),
    "mid_real": dict(n=16, nv=10, nc=22, nmu=110, ng=300, complex=False, seed=6),
    "tiny": dict(n=8, nv=3, nc=5, nmu=12, ng=40, complex=True, seed=7),
    # 16-aligned state counts with ragged points and grid: interior tiles plus both edge strips.
    "tiles": dict(n=22, nv=16, nc=48, nmu=200, ng=600, complex=True, seed=10),
    # Full tiles everywhere (points and plane waves multiples of 128): the interior fast paths.
    "kmaj": dict(n=20, nv=16, nc=48, nmu=256, ng=512, complex=True, seed=11),
    # Both state counts multiples of 32 (even numbers of K tiles in both pair ranges) on a
    # 28^3 grid: the pair kernel's path that stages each range's first K tile ahead, with
    # 686 interior tiles, so most workgroups walk several and refill across tiles.
    "kmaj_even": dict(n=28, nv=32, nc=64, nmu=256, ng=512, complex=True, seed=15),
    # Points a multiple of 128 and Nc a multiple of 32: the single-precision core on the
    # k-major engine (one occupied state per split).
    "core32": dict(n=20, nv=12, nc=64, nmu=256, ng=400, complex=True, seed=13),
    # 2048 plane waves on full tiles: 272 Hermitian output tiles, so the output
    # product's last round is cut along K (split tail).
    "tail": dict(n=20, nv=16, nc=48, nmu=256, ng=2048, complex=True, seed=14),
    # Uneven systems batched with the 48^3 one (Nc = 4 Nv, N_mu = 10 Nv, NG = 32 Nv).
    **{f"batch{i}": dict(n=n, nv=nv, nc=4 * nv, nmu=10 * nv, ng=32 * nv, complex=True, seed=30 + i)
       for i, (n, nv) in enumerate(zip((24, 25, 27, 28, 30, 32, 36, 40), (16, 20, 24, 28, 32, 40, 44, 48)))},
    # 32-aligned state counts on a 14^3 grid: the self-energy pair sets (occupied x all,
    # all x all) run the single-precision pair kernel's interior path with even K ranges.
    "sig_even": dict(n=14, nv=32, nc=32, nmu=192, ng=400, complex=True, seed=16),
    # 3000 plane waves on a 20^3 grid: 17 or more x-frequencies, so the warp-specialised DFT
    # runs three matrix-core waves per slab group, spread unevenly over the SIMDs.
    "pipe3": dict(n=20, nv=12, nc=36, nmu=150, ng=3000, complex=True, seed=17),
    # Odd 33^3 grid above 32 points per axis (every grid vector in the Gram: two DFT x/y chunks).
    "wide": dict(n=33, nv=6, nc=18, nmu=60, ng=300, complex=True, seed=12),
    # Full rank: N_mu = Nv * Nc, where ISDF is exact.
    "fullrank": dict(n=12, nv=4, nc=6, nmu=24, ng=200, complex=True, seed=8),
    "fullrank_real": dict(n=12, nv=4, nc=6, nmu=24, ng=200, complex=False, seed=9),
}


def box_length(nv: int) -> float:
    """Cubic box side in Bohr: the Si cell (10.26 Bohr, 8 occupied states) at constant density."""
    return 10.26 * (nv / 8.0) ** (1.0 / 3.0)


def freq_grid(n: int) -> np.ndarray:
    """Signed integer frequencies in [-n/2, n/2) in numpy FFT order."""
    return np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)


def lowpass_cut(n: int, nstates: int) -> int:
    """Smallest s with #{m : |m|^2 <= s} >= 2 * nstates (all m in [-n/2, n/2)^3)."""
    f = freq_grid(n)
    m2 = (f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2).ravel()
    vals, counts = np.unique(m2, return_counts=True)
    cum = np.cumsum(counts)
    idx = int(np.searchsorted(cum, 2 * nstates))
    if idx >= len(vals):
        raise ValueError("grid too small for the requested number of states")
    return int(vals[idx])


def miller_list(n: int, ng: int) -> np.ndarray:
    """First ng Miller vectors in [-n/2, n/2)^3 ordered by (|m|^2, m_x, m_y, m_z); int32 (ng, 3)."""
    f = np.arange(-(n // 2), n - n // 2, dtype=np.int64)
    mx, my, mz = np.meshgrid(f, f, f, indexing="ij")
    mx, my, mz = mx.ravel(), my.ravel(), mz.ravel()
    m2 = mx * mx + my * my + mz * mz
    order = np.lexsort((mz, my, mx, m2))
    if ng > order.size:
        raise ValueError("ng exceeds the number of grid frequencies")
    sel = order[:ng]
    return np.stack([mx[sel], my[sel], mz[sel]], axis=1).astype(np.int32)


@dataclasses.dataclass
class Inputs:
    name: str
    n: int
    nv: int
    nc: int
    nmu: int
    ng: int
    is_complex: bool
    L: float
    psi_t: np.ndarray      # (N, Nr): psi_t[n, k] = psi_n(r_k); column-major Nr x N
    energies: np.ndarray   # (N,) Hartree; first nv occupied
    mu_idx: np.ndarray     # (nmu,) int32, sorted, distinct
    miller: np.ndarray     # (ng, 3) int32
    omegas: np.ndarray     # imaginary frequencies (Hartree); empty = static
    seed: int

    @property
    def nr(self) -> int:
        return self.n ** 3

    @property
    def cell(self) -> np.ndarray:
        return np.eye(3) * self.L

    @property
    def v_scale(self) -> float:
        """Grid-independent Coulomb prefactor Nr / Omega_cell for unit-norm grid orbitals."""
        return self.nr / self.L ** 3


def _orbitals(rng, n, nstates, is_complex):
    nr = n ** 3
    s_cut = lowpass_cut(n, nstates)
    f = freq_grid(n)
    m2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2  # [z, y, x]
    mask = m2 <= s_cut
    if is_complex:
        ns = int(mask.sum())
        coef = (rng.standard_normal((ns, nstates)) + 1j * rng.standard_normal((ns, nstates))) / math.sqrt(2.0)
        q, _ = np.linalg.qr(coef)
        spec = np.zeros((nstates, n, n, n), dtype=np.complex128)
        spec[:, mask] = q.T
        psi = np.fft.ifftn(spec, axes=(1, 2, 3), norm="ortho").reshape(nstates, nr)
        del spec
        return np.ascontiguousarray(psi), s_cut
    noise = rng.standard_normal((nstates, n, n, n))
    spec = np.fft.fftn(noise, axes=(1, 2, 3))
    spec[:, ~mask] = 0.0
    g = np.fft.ifftn(spec, axes=(1, 2, 3)).real.reshape(nstates, nr)
    q, _ = np.linalg.qr(g.T)
    return np.ascontiguousarray(q.T), s_cut


def _energies(rng, nv, nc):
    ev = np.sort(rng.uniform(-20.0, -5.0, nv))
    ec = np.sort(rng.uniform(1.0, 30.0, nc))
    return np.concatenate([ev, ec]) / HARTREE_EV


def select_points(rng, psi_t, nv, nmu, is_complex):
    """Interpolation points of the valence-conduction pair set (occupied x empty states)."""
    nstates = psi_t.shape[0]
    return select_pair_points(rng, psi_t, np.arange(nv), np.arange(nv, nstates), nmu, is_complex)


def select_pair_points(rng, psi_t, a_rows, b_rows, nmu, is_complex):
    """Interpolation points by column-pivoted QR of a random sketch of the pair products
    conj(psi_a) psi_b, a in a_rows, b in b_rows.

    The sketch column t is conj(sum_a psi_a g_at) * (sum_b psi_b h_bt), i.e. the pair
    products contracted with Gaussian weights; it is evaluated on a random candidate
    subset of the grid when the grid is large.  Returns sorted distinct int32 indices.
    """
    nr = psi_t.shape[1]
    na, nb = len(a_rows), len(b_rows)
    p = nmu + min(nmu, 64)
    if nr <= 20000:
        cand = np.arange(nr)
    else:
        cand = np.sort(rng.choice(nr, size=min(nr, 4 * nmu), replace=False))
    pa = psi_t[a_rows][:, cand].T
    pb = psi_t[b_rows][:, cand].T
    if is_complex:
        g = rng.standard_normal((na, p)) + 1j * rng.standard_normal((na, p))
        h = rng.standard_normal((nb, p)) + 1j * rng.standard_normal((nb, p))
    else:
        g = rng.standard_normal((na, p))
        h = rng.standard_normal((nb, p))
    sk = np.conj(pa @ g) * (pb @ h)
    _, _, piv = scipy.linalg.qr(sk.T, mode="economic", pivoting=True)
    mu = np.sort(cand[piv[:nmu]]).astype(np.int32)
    return mu


def sigma_point_counts(inp) -> tuple[int, int]:
    """Point counts of the two self-energy pair sets at the valence-conduction set's ratio
    k_mu = N_mu / sqrt(Nv Nc): N_mu^vn = k_mu sqrt(Nv N) and N_mu^nn = k_mu N (N = Nv + Nc),
    each at most Nr and below the pair set's rank (N (N + 1) / 2 distinct products for
    real orbitals)."""
    ns = inp.nv + inp.nc
    k = inp.nmu / math.sqrt(inp.nv * inp.nc)
    nvn = int(round(k * math.sqrt(inp.nv * ns)))
    nnn = int(round(k * ns))
    nnn_rank = ns * (ns + 1) // 2 if not inp.is_complex else ns * ns
    return min(nvn, inp.nr, inp.nv * ns), min(nnn, inp.nr, nnn_rank)


def sigma_points(inp, nmu_vn: int | None = None, nmu_nn: int | None = None):
    """Interpolation points of the occupied x all (vn) and all x all (nn) pair sets that
    the self-energy fits use (Algorithm 3's P_vn and P_nn), from their own seeded
    stream (seed + 1000), so the dielectric inputs stay as drawn."""
    dvn, dnn = sigma_point_counts(inp)
    nvn = dvn if nmu_vn is None else nmu_vn
    nnn = dnn if nmu_nn is None else nmu_nn
    rng = np.random.default_rng(inp.seed + 1000)
    ns = inp.nv + inp.nc
    allr = np.arange(ns)
    mu_vn = select_pair_points(rng, inp.psi_t, np.arange(inp.nv), allr, nvn, inp.is_complex)
    mu_nn = select_pair_points(rng, inp.psi_t, allr, allr, nnn, inp.is_complex)
    return mu_vn, mu_nn


def make_inputs(name: str = "cfg0", *, nmu: int | None = None, n_omega: int = 0,
                seed: int | None = None, **overrides) -> Inputs:
    c = dict(CONFIGS[name])
    c.update(overrides)
    if nmu is not None:
        c["nmu"] = nmu
    if seed is not None:
        c["seed"] = seed
    rng = np.random.default_rng(c["seed"])
    n, nv, nc = c["n"], c["nv"], c["nc"]
    psi_t, _ = _orbitals(rng, n, nv + nc, c["complex"])
    energies = _energies(rng, nv, nc)
    mu = select_points(rng, psi_t, nv, c["nmu"], c["complex"])
    miller = miller_list(n, c["ng"])
    if n_omega > 0:
        # log-spaced imaginary frequencies in [0.01, 100] eV
        omegas = np.logspace(-2.0, 2.0, n_omega) / HARTREE_EV
    else:
        omegas = np.zeros(0)
    return Inputs(name=name, n=n, nv=nv, nc=nc, nmu=c["nmu"], ng=c["ng"],
                  is_complex=bool(c["complex"]), L=box_length(nv), psi_t=psi_t,
                  energies=energies, mu_idx=mu, miller=miller, omegas=omegas,
                  seed=int(c["seed"]))


def loss_weight(ng: int, seed: int = 4) -> np.ndarray:
    """Seeded Hermitian weight W (NG x NG) of the scalar loss Re tr(W eps~^{-1}):
    W = (X + X^H) / 2 with X ~ CN(0, 1) / sqrt(NG), values exactly representable
    in complex64, returned as complex128."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((ng, ng)) + 1j * rng.standard_normal((ng, ng))) / np.sqrt(2.0 * ng)
    w = ((x + x.conj().T) / 2).astype(np.complex64)
    w = (w + w.conj().T) / 2   # exact Hermitian after the rounding (halving is exact)
    return w.astype(np.complex128)
