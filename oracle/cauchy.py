"""Cauchy-integral form of the ISDF core (Algorithm 2) on the CPU, FP64.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the GPU library.

The core M = f C Omega^{-1} C^H (eq. COmegaCstar, static) is rewritten with the
residue theorem: for i occupied and j empty,
    1 / (eps_i - eps_j) = -1/(2 pi i) * contour integral of d lambda / ((lambda - eps_i)(lambda - eps_j))
over a closed contour around the empty-state energies that leaves the occupied
ones outside (eq. coeffchi0).  Summed over the pairs, M = -f/(2 pi i) * contour
integral of J(lambda), with the Hadamard product (eq. defJlambda)
    J(lambda)(mu, nu) = [sum_i conj(psi_i(r_mu)) psi_i(r_nu) / (lambda - eps_i)]
                      * [sum_j psi_j(r_mu) conj(psi_j(r_nu)) / (lambda - eps_j)].
For complex orbitals J(conj(lambda)) = J(lambda)^H, so for a contour symmetric
about the real axis the closed integral is A - A^H with A the integral over
the upper half (counterclockwise), and
    M = -f / (2 pi i) (A - A^H)
(for real orbitals this is the elementwise imaginary part of the paper's form).

Contour (Sec. "Cauchy integral representation", following the elliptic map the
paper takes from Lu and Thicke): with q = eps_{v+1} - eps_v (gap) and
Q = eps_{last} - eps_v, r = (sqrt(Q/q) - 1) / (sqrt(Q/q) + 1), R = K(r) and
L = K'(r) / 2, the segment t in [-R + iL, R + iL] is mapped to the upper half of
the contour by
    z(t) = sqrt(qQ) (1/r + sn(t, r)) / (1/r - sn(t, r)) + eps_v,
    dz/dt = 2 sqrt(qQ) (1/r) cn(t) dn(t) / (1/r - sn(t))^2,
and is walked from left to right, i.e. clockwise; the midpoint rule in t is
used.  Readings (the printed algorithm is garbled in places): the prefactor and
the Jacobian are re-derived as above, and L uses an infinite upper limit in its
integral (the printed limit 1/r gives a different height), i.e. L = K'/2.

The quadrature error falls like exp(-pi^2 N / (2 log(Q/q) + 6)) with N nodes
(eq. rel_err_Cauchy); ``nodes_for_tolerance`` inverts that bound, and
``core_cauchy_adaptive`` doubles N until two successive results agree to the
requested relative tolerance.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ellipj, ellipk

from .dielectric import PAIR_FACTOR


def jacobi_sn_cn_dn(x: np.ndarray, y: np.ndarray, m: float):
    """sn, cn, dn at the complex argument x + i y for parameter m = k^2.

    Addition theorem with the imaginary transformation (Abramowitz and Stegun
    16.21.1-3): real-argument values at (x, m) and (y, 1 - m)."""
    s, c, d, _ = ellipj(x, m)
    s1, c1, d1, _ = ellipj(y, 1.0 - m)
    den = c1 ** 2 + m * s ** 2 * s1 ** 2
    sn = (s * d1 + 1j * c * d * s1 * c1) / den
    cn = (c * c1 - 1j * s * d * s1 * d1) / den
    dn = (d * c1 * d1 - 1j * m * s * c * s1) / den
    return sn, cn, dn


def contour_nodes(q: float, Q: float, n: int):
    """Nodes z_k (relative to eps_v) and weights dz/dt * (2R / n) of the midpoint
    rule on the upper half of the contour, in the order of increasing t."""
    r = (np.sqrt(Q / q) - 1.0) / (np.sqrt(Q / q) + 1.0)
    m = r * r
    big_r, big_l = ellipk(m), 0.5 * ellipk(1.0 - m)
    x = -big_r + 2.0 * big_r * (np.arange(n) + 0.5) / n
    sn, cn, dn = jacobi_sn_cn_dn(x, np.full(n, big_l), m)
    s = np.sqrt(q * Q)
    z = s * (1.0 / r + sn) / (1.0 / r - sn)
    dz = 2.0 * s / r * cn * dn / (1.0 / r - sn) ** 2
    return z, dz * (2.0 * big_r / n)


def gap_and_width(energies: np.ndarray, nv: int):
    """(eps_v, q, Q) of the contour: the top occupied energy, the gap and the span."""
    e = np.asarray(energies, dtype=np.float64)
    return e[nv - 1], e[nv] - e[nv - 1], e[-1] - e[nv - 1]


def nodes_for_tolerance(q: float, Q: float, tol: float) -> int:
    """Smallest N with exp(-pi^2 N / (2 log(Q/q) + 6)) <= tol (eq. rel_err_Cauchy)."""
    return int(np.ceil((2.0 * np.log(Q / q) + 6.0) * np.log(1.0 / tol) / np.pi ** 2))


def core_cauchy(psi_t, energies, nv, mu_idx, n_nodes, f=PAIR_FACTOR) -> np.ndarray:
    """M = f C Omega^{-1} C^H (static) by the contour integral with n_nodes nodes."""
    ev, q, big_q = gap_and_width(energies, nv)
    z, w = contour_nodes(q, big_q, n_nodes)
    lam = z + ev
    pv = np.asarray(psi_t)[:nv][:, mu_idx]      # (Nv, N_mu): psi_i(r_mu)
    pc = np.asarray(psi_t)[nv:][:, mu_idx]      # (Nc, N_mu)
    e = np.asarray(energies, dtype=np.float64)
    a = np.zeros((len(mu_idx), len(mu_idx)), dtype=np.complex128)
    for k in range(n_nodes):
        av = np.conj(pv).T @ (pv / (lam[k] - e[:nv])[:, None])            # sum_i conj(psi_i(mu)) psi_i(nu) / (lam - eps_i)
        ac = pc.T @ (np.conj(pc) / (lam[k] - e[nv:])[:, None])            # sum_j psi_j(mu) conj(psi_j(nu)) / (lam - eps_j)
        a -= w[k] * (av * ac)                                             # counterclockwise upper half
    return -f / (2j * np.pi) * (a - np.conj(a.T))


def core_cauchy_adaptive(psi_t, energies, nv, mu_idx, tol, f=PAIR_FACTOR, n0=8, n_max=1024):
    """Algorithm 2's adaptive rule: double N until successive results agree to tol
    (relative Frobenius); returns (M, N)."""
    n = n0
    prev = core_cauchy(psi_t, energies, nv, mu_idx, n, f)
    while n < n_max:
        n *= 2
        cur = core_cauchy(psi_t, energies, nv, mu_idx, n, f)
        if np.linalg.norm(cur - prev) <= tol * np.linalg.norm(cur):
            return cur, n
        prev = cur
    return prev, n
