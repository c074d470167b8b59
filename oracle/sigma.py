"""Plain FP64 CPU oracle for the static COHSEX self-energy diagonals.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the GPU library.

What is computed (paper, Sec. 2, eq. selfenergySum in matrix form beside
eq. matrices; Algorithm 3, steps 2 and 4-7): for every band n,

    Sigma_SEX_X(n) = - sum_{i in v}   m_in^H (W - V) m_in
    Sigma_X(n)     = - sum_{i in v}   m_in^H  V      m_in
    Sigma_COH(n)   = 1/2 sum_{n' in all} m_n'n^H (W - V) m_n'n

with the pair function m_in(r) = conj(psi_i(r)) psi_n(r) and W - V = (eps^{-1} - I) V.
Readings (the same as for the dielectric inverse):
  * symmetrised form: (eps^{-1} - I) V = V^{1/2} (eps~^{-1} - I) V^{1/2}, so with
    u = V^{1/2} F m on the plane-wave list, m^H (W - V) m = u^H (eps~^{-1} - I) u and
    m^H V m = u^H u;
  * the plane-wave list is the one eps~^{-1} is built on (the NG-truncated Coulomb
    operator), for the bare exchange term too;
  * Algorithm 3 replaces every pair function by its ISDF fit: m_in ~ Theta_vn c_in
    with c_in(mu) = conj(psi_i(r_mu)) psi_n(r_mu) on the vn points, and
    m_n'n ~ Theta_nn c_n'n on the nn points, each Theta the least-squares fit of
    its own pair set (as for the valence-conduction set);
  * the three diagonals are real (each term is a Hermitian form); step 7 of
    Algorithm 3 keeps the real part.

Two modes:
  * ``sigma_exact``: the pair functions themselves (no ISDF), given eps~^{-1};
  * ``sigma_isdf``: the ISDF-fitted pair functions of both sets, given eps~^{-1}.
Neither uses the Hadamard identity (eq. Hadamard) or the low-rank form of
W_vn / W_nn of Algorithm 3; those are what the GPU path computes, and the pins
check that they agree with these plain sums.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .dielectric import coulomb_diag, dft_rows


def pair_set_coefficients(psi_t, a_rows, b_rows, mu_idx) -> np.ndarray:
    """C(mu; (a, b)) = conj(psi_a(r_mu)) psi_b(r_mu), pair index a-major, shape (N_mu, |a| |b|)."""
    pts = psi_t[:, mu_idx]
    pa, pb = pts[a_rows], pts[b_rows]
    c = np.conj(pa)[:, None, :] * pb[None, :, :]
    return c.reshape(-1, len(mu_idx)).T.astype(np.complex128)


def pair_set_functions(psi_t, a_rows, b_rows) -> np.ndarray:
    """Rows m_ab(r) = conj(psi_a(r)) psi_b(r), pair index a-major, shape (|a| |b|, Nr)."""
    pa, pb = psi_t[a_rows], psi_t[b_rows]
    out = np.empty((len(a_rows) * len(b_rows), psi_t.shape[1]), dtype=np.complex128)
    for t, a in enumerate(range(len(a_rows))):
        out[t * len(b_rows):(t + 1) * len(b_rows)] = np.conj(pa[a])[None, :] * pb
    return out


def pair_set_fit(psi_t, a_rows, b_rows, mu_idx) -> np.ndarray:
    """Theta = argmin ||M - Theta C||_F for the pair set (a, b): Theta (C C^H) = M C^H.

    M C^H is formed from the explicit pair functions and coefficients; the solve is LU.
    """
    c = pair_set_coefficients(psi_t, a_rows, b_rows, mu_idx)
    m = pair_set_functions(psi_t, a_rows, b_rows)             # (pairs, Nr) = M^T
    s = c @ np.conj(c.T)
    z = m.T @ np.conj(c.T)                                    # M C^H, (Nr, N_mu)
    th_h = scipy.linalg.solve(s, np.conj(z.T), assume_a="gen")
    return np.conj(th_h.T)


def _sigma_terms(u_vn: np.ndarray, u_nn: np.ndarray, nv: int, ns: int, eps_inv: np.ndarray) -> np.ndarray:
    """The three diagonals from the plane-wave coefficients of the pair functions.

    u_vn: (NG, nv * ns) columns u_in, pair index i-major (i in v, n in all);
    u_nn: (NG, ns * ns) columns u_n'n, pair index n'-major.
    Returns (3, ns): Sigma_SEX_X, Sigma_X, Sigma_COH.
    """
    d = eps_inv - np.eye(eps_inv.shape[0])
    out = np.zeros((3, ns))
    for i in range(nv):
        for n in range(ns):
            u = u_vn[:, i * ns + n]
            out[0, n] -= np.real(np.vdot(u, d @ u))
            out[1, n] -= np.real(np.vdot(u, u))
    for a in range(ns):
        for n in range(ns):
            u = u_nn[:, a * ns + n]
            out[2, n] += 0.5 * np.real(np.vdot(u, d @ u))
    return out


def sigma_exact(inp, eps_inv, v_scale=None) -> np.ndarray:
    """(3, N) diagonals from the pair functions themselves, given eps~^{-1} on the list."""
    vs = inp.v_scale if v_scale is None else v_scale
    ns = inp.nv + inp.nc
    v = coulomb_diag(inp.miller, inp.cell, vs)
    sv = np.sqrt(v)[:, None]
    allr, occ = np.arange(ns), np.arange(inp.nv)
    u_vn = sv * dft_rows(pair_set_functions(inp.psi_t, occ, allr), inp.n, inp.miller).T
    u_nn = sv * dft_rows(pair_set_functions(inp.psi_t, allr, allr), inp.n, inp.miller).T
    return _sigma_terms(u_vn, u_nn, inp.nv, ns, eps_inv)


def sigma_isdf(inp, mu_vn, mu_nn, eps_inv, v_scale=None) -> np.ndarray:
    """(3, N) diagonals from the ISDF-fitted pair functions of the vn and nn sets."""
    vs = inp.v_scale if v_scale is None else v_scale
    ns = inp.nv + inp.nc
    v = coulomb_diag(inp.miller, inp.cell, vs)
    sv = np.sqrt(v)[:, None]
    allr, occ = np.arange(ns), np.arange(inp.nv)
    u_sets = []
    for a_rows, mu in ((occ, mu_vn), (allr, mu_nn)):
        theta = pair_set_fit(inp.psi_t, a_rows, allr, mu)                        # (Nr, N_mu)
        c = pair_set_coefficients(inp.psi_t, a_rows, allr, mu)                  # (N_mu, pairs)
        tg = dft_rows(np.ascontiguousarray(theta.T), inp.n, inp.miller).T       # (NG, N_mu)
        u_sets.append(sv * (tg @ c))                                            # fitted pairs, (NG, pairs)
    return _sigma_terms(u_sets[0], u_sets[1], inp.nv, ns, eps_inv)


# ----------------------------------------------------------------------------
# Plane-wave orbitals: every quantity in closed form
# ----------------------------------------------------------------------------
def plane_wave_sigma(kvecs, nv, n, miller, cell, v_scale, energies, f=2.0) -> np.ndarray:
    """Closed form for orbitals psi_n(r) = exp(2 pi i k_n . x / n) / sqrt(Nr) (distinct k_n).

    Every pair function is one plane wave, F m_ab = delta(G, k_b - k_a) / sqrt(Nr), so chi0
    is diagonal on the list: chi0(G) = f / Nr sum_{i in v, j in c, k_j - k_i = G} 1 / (e_i - e_j),
    eps~^{-1}(G) = 1 / (1 - V(G) chi0(G)), and each self-energy term is a sum of
    V(G) (eps~^{-1}(G) - 1) / Nr or V(G) / Nr over the pairs whose difference G is on the list.
    Returns (3, N) and the diagonal of eps~^{-1} on the list.
    """
    kvecs = np.asarray(kvecs, dtype=np.int64)
    nr = n ** 3
    ns = len(kvecs)
    key = {tuple(np.mod(m, n)): g for g, m in enumerate(np.asarray(miller, dtype=np.int64))}
    v = coulomb_diag(miller, cell, v_scale)
    chi = np.zeros(len(miller))
    for i in range(nv):
        for j in range(nv, ns):
            g = key.get(tuple(np.mod(kvecs[j] - kvecs[i], n)))
            if g is not None:
                chi[g] += f / nr / (energies[i] - energies[j])
    einv = 1.0 / (1.0 - v * chi)
    out = np.zeros((3, ns))
    for b in range(ns):
        for a in range(ns):
            g = key.get(tuple(np.mod(kvecs[b] - kvecs[a], n)))
            if g is None:
                continue
            if a < nv:
                out[0, b] -= v[g] * (einv[g] - 1.0) / nr
                out[1, b] -= v[g] / nr
            out[2, b] += 0.5 * v[g] * (einv[g] - 1.0) / nr
    return out, einv
