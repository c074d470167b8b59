"""Plain FP64 CPU oracle for the static / imaginary-frequency dielectric inverse.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the GPU library (no kernels, tables or helpers); the only
common dependency is the seeded input generator ``synth``.

Notation (paper, Sec. 2 "matrix forms" and Sec. "Interpolative separable
density fitting"):
  * psi_t[n, k] = psi_n(r_k) on the real-space grid, unit-norm grid columns;
    states 0..nv-1 occupied (v), nv..N-1 unoccupied (c).
  * M_vc(k; (i, j)) = conj(psi_i(r_k)) psi_j(r_k), pair index (i, j) i-major.
  * Omega = diag(eps_i - eps_j) < 0 (eq. Omega).
  * chi0 = f M_vc Omega^{-1} M_vc^H with f = 2 (eq. matrices; time-reversal
    merging of the two pole terms).
  * ISDF: M_vc ~ P C with C(mu; (i, j)) = conj(psi_i(r_mu)) psi_j(r_mu)
    (eq. ISDF, eq. MatrixExpressionISDF); P is written Theta here.
  * Symmetrised dielectric matrix in the plane-wave basis
    eps~ = I - V^{1/2} chi0 V^{1/2}, V(G) = v_scale 4 pi / |G|^2, V(0) = 0
    (the Hermitian form used in the error analysis of the supplement).
  * Imaginary frequency i*omega: the two pole terms of eq. Hedin_fourier at
    omega -> i*omega, eta -> 0 merge into the weight
    Delta / (Delta^2 + omega^2), Delta = eps_i - eps_j; at omega = 0 this is
    1 / Delta, the static Omega^{-1}.

Readings where the paper is silent:
  * quadrature weights are dropped as in the paper (Sec. 2), the grid DFT is
    unitary, and v_scale = Nr / Omega_cell restores the grid-independent
    physical screening for unit-norm grid orbitals;
  * Theta is the least-squares fit min ||M_vc - Theta C||_F, so
    Theta (C C^H) = M_vc C^H (the paper cites Hu et al. for the fit).

Every function below states the definition it implements.  Pins that tie
each one to something other than itself live in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

PAIR_FACTOR = 2.0


# ----------------------------------------------------------------------------
# Definitions on the grid
# ----------------------------------------------------------------------------
def pair_products(psi_t: np.ndarray, nv: int) -> np.ndarray:
    """Rows of M_vc^T: out[(i, j), k] = conj(psi_i(r_k)) psi_j(r_k), i in v, j in c.

    The pair-function matrix defined beside eq. Omega (Sec. 2).
    """
    pv = psi_t[:nv]
    pc = psi_t[nv:]
    nc = pc.shape[0]
    out = np.empty((nv * nc, psi_t.shape[1]), dtype=np.result_type(psi_t, np.complex128))
    for i in range(nv):
        out[i * nc:(i + 1) * nc] = np.conj(pv[i])[None, :] * pc
    return out


def gvectors_cart(miller: np.ndarray, cell: np.ndarray) -> np.ndarray:
    """Cartesian G = 2 pi B^T m with B = inv(cell)^T rows; cell rows are lattice vectors."""
    recip = 2.0 * np.pi * np.linalg.inv(np.asarray(cell, dtype=np.float64)).T
    return np.asarray(miller, dtype=np.float64) @ recip


def coulomb_diag(miller: np.ndarray, cell: np.ndarray, v_scale: float) -> np.ndarray:
    """V(G) = v_scale * 4 pi / |G|^2 on the plane-wave list, with V(G = 0) = 0."""
    g = gvectors_cart(miller, cell)
    g2 = np.einsum("gi,gi->g", g, g)
    v = np.zeros(len(g2))
    nz = g2 > 0
    v[nz] = v_scale * 4.0 * np.pi / g2[nz]
    return v


def dft_rows(x: np.ndarray, n: int, miller: np.ndarray) -> np.ndarray:
    """Unitary 3-D DFT of each row, sampled on the Miller list.

    out[b, g] = Nr^{-1/2} sum_k x[b, k] exp(-2 pi i m_g . (i0, i1, i2)_k / n),
    k = i0 + n (i1 + n i2).
    """
    b = x.shape[0]
    cube = x.reshape(b, n, n, n)  # [b, i2, i1, i0]
    f = np.fft.fftn(cube, axes=(1, 2, 3), norm="ortho")
    m = np.mod(np.asarray(miller, dtype=np.int64), n)
    return f[:, m[:, 2], m[:, 1], m[:, 0]]


def pair_weights(energies: np.ndarray, nv: int, omega: float = 0.0) -> np.ndarray:
    """w[i, j] = Delta / (Delta^2 + omega^2), Delta = eps_i - eps_j (i in v, j in c).

    omega = 0 gives 1 / (eps_i - eps_j), the diagonal of Omega^{-1} (eq. Omega).
    """
    d = energies[:nv, None] - energies[None, nv:]
    return d / (d * d + omega * omega)


def chi0_exact_pw(psi_t, energies, nv, n, miller, f=PAIR_FACTOR, omega=0.0):
    """chi0 in the plane-wave basis from all pair products (eq. matrices).

    chi0(G, G') = f sum_{i in v, j in c} (F m_ij)(G) w_ij conj((F m_ij)(G')),
    accumulated one occupied state at a time.
    """
    ng = len(miller)
    w = pair_weights(energies, nv, omega)
    chi = np.zeros((ng, ng), dtype=np.complex128)
    pc = psi_t[nv:]
    for i in range(nv):
        r = dft_rows(np.conj(psi_t[i])[None, :] * pc, n, miller)  # (Nc, NG)
        chi += f * (r.T * w[i][None, :]) @ np.conj(r)
    return chi


def eps_tilde(chi0: np.ndarray, v: np.ndarray) -> np.ndarray:
    """eps~ = I - V^{1/2} chi0 V^{1/2} (symmetrised dielectric matrix)."""
    s = np.sqrt(v)
    return np.eye(len(v)) - s[:, None] * chi0 * s[None, :]


def invert_lu(a: np.ndarray) -> np.ndarray:
    """Dense inverse by LU (LAPACK getrf/getri through scipy)."""
    return scipy.linalg.inv(a)


def eps_inv_exact(inp, f=PAIR_FACTOR, omega=0.0, v_scale=None):
    """eps~^{-1} with chi0 built from every valence-conduction pair, then dense LU."""
    vs = inp.v_scale if v_scale is None else v_scale
    v = coulomb_diag(inp.miller, inp.cell, vs)
    chi = chi0_exact_pw(inp.psi_t, inp.energies, inp.nv, inp.n, inp.miller, f, omega)
    return invert_lu(eps_tilde(chi, v))


# ----------------------------------------------------------------------------
# ISDF (eq. ISDF, eq. MatrixExpressionISDF)
# ----------------------------------------------------------------------------
def isdf_coefficients(psi_t, nv, mu_idx) -> np.ndarray:
    """C(mu; (i, j)) = conj(psi_i(r_mu)) psi_j(r_mu), shape (N_mu, Nv Nc)."""
    pts = psi_t[:, mu_idx]                       # (N, N_mu)
    pv, pc = pts[:nv], pts[nv:]
    c = np.conj(pv)[:, None, :] * pc[None, :, :]  # (Nv, Nc, N_mu)
    return c.reshape(-1, len(mu_idx)).T.astype(np.complex128)


def isdf_rhs(psi_t, nv, mu_idx) -> np.ndarray:
    """Z = M_vc C^H in factored form, shape (Nr, N_mu).

    (M_vc C^H)(k, mu) = sum_{i, j} conj(psi_i(r_k)) psi_j(r_k) psi_i(r_mu) conj(psi_j(r_mu))
                      = conj(sum_i psi_i(r_k) conj(psi_i(r_mu))) * sum_j psi_j(r_k) conj(psi_j(r_mu)),
    i.e. the Hadamard product of two orbital Gram blocks, the identity the paper
    uses to reduce its self-energy sums (eq. Hadamard).
    """
    pv, pc = psi_t[:nv], psi_t[nv:]
    gv = pv.T @ np.conj(pv[:, mu_idx])   # (Nr, N_mu)
    gc = pc.T @ np.conj(pc[:, mu_idx])
    return np.conj(gv) * gc


def isdf_fit(psi_t, nv, mu_idx) -> np.ndarray:
    """Theta = argmin ||M_vc - Theta C||_F = (M_vc C^H) (C C^H)^{-1}, shape (Nr, N_mu).

    C C^H is formed by a plain product of the explicit C; the solve is LU.
    """
    c = isdf_coefficients(psi_t, nv, mu_idx)
    s = c @ np.conj(c.T)
    z = isdf_rhs(psi_t, nv, mu_idx)
    # Theta S = Z  <=>  S Theta^H = Z^H  (S Hermitian)
    th_h = scipy.linalg.solve(s, np.conj(z.T), assume_a="gen")
    return np.conj(th_h.T)


def isdf_fit_bruteforce(psi_t, nv, mu_idx) -> np.ndarray:
    """Theta from numpy least squares on the explicit pair-function matrix (small sizes only)."""
    m = pair_products(psi_t, nv).T               # (Nr, Nv Nc)
    c = isdf_coefficients(psi_t, nv, mu_idx)     # (N_mu, Nv Nc)
    # Theta C = M  <=>  C^T Theta^T = M^T
    sol, *_ = np.linalg.lstsq(c.T, m.T, rcond=None)
    return sol.T


def core_matrix(psi_t, energies, nv, mu_idx, f=PAIR_FACTOR, omega=0.0) -> np.ndarray:
    """f C diag(w) C^H, the N_mu x N_mu core (eq. COmegaCstar with the factor f).

    The paper writes the SMW core as (1/2)(C Omega^{-1} C^H)^{-1}; with f = 2,
    (f C Omega^{-1} C^H)^{-1} is the same matrix.
    """
    c = isdf_coefficients(psi_t, nv, mu_idx)
    w = pair_weights(energies, nv, omega).ravel()
    return f * (c * w[None, :]) @ np.conj(c.T)


def theta_pw(theta: np.ndarray, n: int, miller: np.ndarray) -> np.ndarray:
    """Theta_G = (F Theta) on the plane-wave list, shape (NG, N_mu)."""
    return dft_rows(np.ascontiguousarray(theta.T), n, miller).T


def coulomb_factor(inp, v_scale=None) -> np.ndarray:
    vs = inp.v_scale if v_scale is None else v_scale
    return coulomb_diag(inp.miller, inp.cell, vs)


def isdf_stages(inp, f=PAIR_FACTOR, omega=0.0, v_scale=None) -> dict:
    """Stage outputs of the ISDF route: Theta, Theta_G, U = V^{1/2} Theta_G, core M."""
    theta = isdf_fit(inp.psi_t, inp.nv, inp.mu_idx)
    tg = theta_pw(theta, inp.n, inp.miller)
    v = coulomb_factor(inp, v_scale)
    u = np.sqrt(v)[:, None] * tg
    m = core_matrix(inp.psi_t, inp.energies, inp.nv, inp.mu_idx, f, omega)
    return dict(theta=theta, theta_g=tg, v=v, u=u, m=m)


def eps_inv_isdf(inp, f=PAIR_FACTOR, omega=0.0, v_scale=None, stages=None):
    """eps~^{-1} for the ISDF pair products M_vc ~ Theta C: dense eps~, then LU.

    chi0 = f (Theta C) Omega^{-1} (Theta C)^H = Theta M Theta^H; in the plane-wave
    basis eps~ = I - U M U^H with U = V^{1/2} Theta_G.  No SMW here: the
    definition is inverted directly.
    """
    st = stages if stages is not None else isdf_stages(inp, f, omega, v_scale)
    u, m = st["u"], st["m"]
    eps = np.eye(u.shape[0]) - u @ m @ np.conj(u.T)
    return invert_lu(eps)


def eps_inv_smw(u: np.ndarray, m: np.ndarray) -> np.ndarray:
    """SMW form (eq. epsilon_with_SMW, symmetrised): I + U (M^{-1} - U^H U)^{-1} U^H.

    Explicit inverses exactly as the formula reads; used for pins only.
    """
    k = np.linalg.inv(np.linalg.inv(m) - np.conj(u.T) @ u)
    return np.eye(u.shape[0]) + u @ k @ np.conj(u.T)


# ----------------------------------------------------------------------------
# Full-grid Coulomb Gram (the paper's P^H V P over the whole real-space grid)
# ----------------------------------------------------------------------------
def grid_miller(n: int) -> np.ndarray:
    """Every Miller vector of the n^3 grid, components in [-n/2, n/2)."""
    r = np.arange(-(n // 2), n - n // 2)
    mz, my, mx = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1).astype(np.int32)


def full_grid_list(miller: np.ndarray, n: int) -> np.ndarray:
    """The plane-wave list followed by every other grid vector."""
    allm = grid_miller(n)
    key = lambda m: (m[:, 0] % n) + n * ((m[:, 1] % n) + n * (m[:, 2] % n))
    rest = allm[~np.isin(key(allm), key(np.asarray(miller)))]
    return np.concatenate([np.asarray(miller, dtype=np.int32), rest])


def eps_inv_exact_full(inp, f=PAIR_FACTOR, omega=0.0, v_scale=None):
    """NG block of the inverse of eps~ over the whole grid, chi0 from every pair.

    Dense over all Nr plane waves: small grids only.
    """
    vs = inp.v_scale if v_scale is None else v_scale
    full = full_grid_list(inp.miller, inp.n)
    v = coulomb_diag(full, inp.cell, vs)
    chi = chi0_exact_pw(inp.psi_t, inp.energies, inp.nv, inp.n, full, f, omega)
    return invert_lu(eps_tilde(chi, v))[:inp.ng, :inp.ng]


def u_full(inp, stages, v_scale=None) -> np.ndarray:
    """U = V^{1/2} F Theta on the whole grid, rows in full_grid_list order (Nr, N_mu)."""
    vs = inp.v_scale if v_scale is None else v_scale
    full = full_grid_list(inp.miller, inp.n)
    return np.sqrt(coulomb_diag(full, inp.cell, vs))[:, None] * theta_pw(stages["theta"], inp.n, full)


def eps_inv_smw_full(inp, f=PAIR_FACTOR, omega=0.0, v_scale=None, stages=None):
    """NG block of the SMW form with the Gram U^H U summed over the whole grid.

    I + U_NG (M^{-1} - U^H U)^{-1} U_NG^H (eq. epsilon_with_SMW, symmetrised),
    U over every grid vector, explicit inverses as the formula reads.
    """
    st = stages if stages is not None else isdf_stages(inp, f, omega, v_scale)
    u = u_full(inp, st, v_scale)
    k = np.linalg.inv(np.linalg.inv(st["m"]) - np.conj(u.T) @ u)
    un = u[:inp.ng]
    return np.eye(inp.ng) + un @ k @ np.conj(un.T)


def eps_inv_isdf_full(inp, f=PAIR_FACTOR, omega=0.0, v_scale=None, stages=None, tol=1e-12):
    """NG block of the inverse of eps~ = I - U M U^H over the whole grid (ISDF pairs).

    U = V^{1/2} F Theta on every grid vector.  Plane waves where every column of U
    is below tol (relative) lie outside the pair products' Fourier support; there
    eps~ is the identity to that tolerance, so the dense LU runs on the support
    plus the output list.
    """
    st = stages if stages is not None else isdf_stages(inp, f, omega, v_scale)
    u = u_full(inp, st, v_scale)
    norms = np.linalg.norm(u, axis=1)
    keep = norms > tol * norms.max()
    keep[:inp.ng] = True
    uk = u[keep]
    eps = np.eye(uk.shape[0]) - uk @ st["m"] @ np.conj(uk.T)
    return invert_lu(eps)[:inp.ng, :inp.ng]


# ----------------------------------------------------------------------------
# Sampled evaluations for full-size checks
# ----------------------------------------------------------------------------
def isdf_gram(psi_t, nv, mu_idx) -> np.ndarray:
    """S = C C^H from the explicit coefficients."""
    c = isdf_coefficients(psi_t, nv, mu_idx)
    return c @ np.conj(c.T)


def theta_rows(psi_t, nv, mu_idx, rows, s=None) -> np.ndarray:
    """Theta at selected grid rows: Z(rows, :) S^{-1}."""
    if s is None:
        s = isdf_gram(psi_t, nv, mu_idx)
    pv, pc = psi_t[:nv], psi_t[nv:]
    gv = pv[:, rows].T @ np.conj(pv[:, mu_idx])
    gc = pc[:, rows].T @ np.conj(pc[:, mu_idx])
    z = np.conj(gv) * gc
    return np.conj(scipy.linalg.solve(s, np.conj(z.T), assume_a="gen").T)


def core_entries(psi_t, energies, nv, mu_idx, pairs, f=PAIR_FACTOR, omega=0.0) -> np.ndarray:
    """Selected entries M(mu, nu) = f sum_{i,j} C(mu,ij) w_ij conj(C(nu,ij)) (eq. COmegaCstar)."""
    w = pair_weights(energies, nv, omega)
    out = np.empty(len(pairs), dtype=np.complex128)
    for t, (a, b) in enumerate(pairs):
        ra, rb = mu_idx[a], mu_idx[b]
        ca = np.conj(psi_t[:nv, ra])[:, None] * psi_t[nv:, ra][None, :]
        cb = np.conj(psi_t[:nv, rb])[:, None] * psi_t[nv:, rb][None, :]
        out[t] = f * np.sum(ca * w * np.conj(cb))
    return out


# ----------------------------------------------------------------------------
# The same definitions evaluated with bounded memory (full-size references)
# ----------------------------------------------------------------------------
def state_coefficients(psi_t, nv, mu_idx, i) -> np.ndarray:
    """The block of C for one occupied state i: C_i(mu, j) = conj(psi_i(r_mu)) psi_j(r_mu), (N_mu, Nc)."""
    pts = psi_t[:, mu_idx]
    return (np.conj(pts[i])[:, None] * pts[nv:].T).astype(np.complex128)


def isdf_gram_by_state(psi_t, nv, mu_idx) -> np.ndarray:
    """S = C C^H summed over the occupied index: S = sum_i C_i C_i^H (C never held whole)."""
    nmu = len(mu_idx)
    s = np.zeros((nmu, nmu), dtype=np.complex128)
    for i in range(nv):
        ci = state_coefficients(psi_t, nv, mu_idx, i)
        s += ci @ np.conj(ci.T)
    return s


def core_matrix_by_state(psi_t, energies, nv, mu_idx, f=PAIR_FACTOR, omega=0.0) -> np.ndarray:
    """f C diag(w) C^H summed over the occupied index: f sum_i C_i diag(w_i) C_i^H (eq. COmegaCstar)."""
    nmu = len(mu_idx)
    w = pair_weights(energies, nv, omega)
    m = np.zeros((nmu, nmu), dtype=np.complex128)
    for i in range(nv):
        ci = state_coefficients(psi_t, nv, mu_idx, i)
        m += f * (ci * w[i][None, :]) @ np.conj(ci.T)
    return m


def isdf_stages_chunked(inp, f=PAIR_FACTOR, omega=0.0, v_scale=None, chunk=16384, mu_chunk=128) -> dict:
    """isdf_stages with bounded memory: S and M summed over the occupied index,
    Theta = Z S^{-1} (eq. MatrixExpressionISDF, least squares) formed by blocks of
    grid rows, and Theta_G = F Theta by blocks of columns.  Theta itself (Nr x N_mu)
    is the only full-size array held."""
    psi_t, nv, mu = inp.psi_t, inp.nv, inp.mu_idx
    nr, nmu = psi_t.shape[1], len(mu)
    s = isdf_gram_by_state(psi_t, nv, mu)
    lu = scipy.linalg.lu_factor(s)
    pv, pc = psi_t[:nv], psi_t[nv:]
    av, ac = np.conj(pv[:, mu]), np.conj(pc[:, mu])
    theta = np.empty((nr, nmu), dtype=np.complex128)
    for r0 in range(0, nr, chunk):
        r1 = min(nr, r0 + chunk)
        z = np.conj(pv[:, r0:r1].T @ av) * (pc[:, r0:r1].T @ ac)     # Z rows (isdf_rhs)
        # Theta S = Z  <=>  S Theta^H = Z^H
        theta[r0:r1] = np.conj(scipy.linalg.lu_solve(lu, np.conj(z.T)).T)
    tg = np.empty((len(inp.miller), nmu), dtype=np.complex128)
    for c0 in range(0, nmu, mu_chunk):
        c1 = min(nmu, c0 + mu_chunk)
        tg[:, c0:c1] = theta_pw(theta[:, c0:c1], inp.n, inp.miller)
    v = coulomb_factor(inp, v_scale)
    u = np.sqrt(v)[:, None] * tg
    m = core_matrix_by_state(psi_t, inp.energies, nv, mu, f, omega)
    return dict(theta=theta, theta_g=tg, v=v, u=u, m=m, s=s)
