"""Pins of the COHSEX self-energy oracle (oracle/sigma.py) to closed forms,
brute force and the mathematics, not to itself.

Plausible mistakes and the pin that catches them:
  pair function conjugated on the wrong orbital, wrong sum range (v vs all),
  dropped 1/2 on COH, wrong sign of a term
      -> plane-wave orbitals (every term in closed form), sign invariants
  wrong DFT sign or Coulomb placement
      -> plane-wave closed form, real-space brute force with an explicit DFT matrix
  wrong least-squares fit of a pair set
      -> full-rank ISDF equals the exact pair functions; the fit against numpy lstsq
  the route the GPU takes (eq. Hadamard on the points, W_vn / W_nn of Algorithm 3 in
  the low-rank form with K) differs from the plain sums
      -> the low-rank Hadamard route equals sigma_isdf
"""
import numpy as np
import pytest

import oracle
import oracle.sigma as osig
import synth


def dft_matrix(n, miller):
    """Explicit unitary DFT rows exp(-2 pi i m . (i0, i1, i2) / n) / sqrt(Nr), from the definition."""
    k = np.arange(n ** 3)
    i0, i1, i2 = k % n, (k // n) % n, k // (n * n)
    ph = (np.outer(miller[:, 0], i0) + np.outer(miller[:, 1], i1) + np.outer(miller[:, 2], i2))
    return np.exp(-2j * np.pi * ph / n) / np.sqrt(n ** 3)


def plane_wave_inputs(n=8, nv=3, nc=5, ng=100, seed=21):
    """Orbitals exp(2 pi i k . x / n) / sqrt(Nr) with distinct small k, a gap in the energies."""
    rng = np.random.default_rng(seed)
    ks = synth.miller_list(n, 27)[1:]                       # |k|^2 <= 2, G = 0 left out
    kv = ks[rng.choice(len(ks), nv + nc, replace=False)]
    k = np.arange(n ** 3)
    x = np.stack([k % n, (k // n) % n, k // (n * n)], axis=1)
    psi = np.exp(2j * np.pi * (kv @ x.T) / n) / np.sqrt(n ** 3)
    e = np.concatenate([np.sort(rng.uniform(-20, -5, nv)), np.sort(rng.uniform(1, 30, nc))]) / synth.HARTREE_EV
    inp = synth.Inputs(name="pw", n=n, nv=nv, nc=nc, nmu=nv * nc, ng=ng, is_complex=True,
                       L=synth.box_length(nv), psi_t=np.ascontiguousarray(psi), energies=e,
                       mu_idx=np.arange(nv * nc, dtype=np.int32), miller=synth.miller_list(n, ng),
                       omegas=np.zeros(0), seed=seed)
    return inp, kv


@pytest.fixture(scope="module")
def tiny():
    return synth.make_inputs("tiny")


@pytest.fixture(scope="module")
def cfg0():
    return synth.make_inputs("cfg0")


def test_plane_wave_closed_form():
    """Plane-wave orbitals: chi0 and eps~ are diagonal, and each of the three terms is a
    sum of V(G)(eps~^-1(G) - 1)/Nr or V(G)/Nr over the pair differences on the list."""
    inp, kv = plane_wave_inputs()
    einv = oracle.eps_inv_exact(inp)
    got = osig.sigma_exact(inp, einv)
    ref, ediag = osig.plane_wave_sigma(kv, inp.nv, inp.n, inp.miller, inp.cell, inp.v_scale, inp.energies)
    assert np.abs(np.diag(einv) - ediag).max() < 1e-12
    assert np.abs(einv - np.diag(np.diag(einv))).max() < 1e-12
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(ref[0]).max() > 0 and np.abs(ref[2]).max() > 0   # the screening terms are not empty


def test_real_space_bruteforce(tiny):
    """The three terms from the real-space matrices of eq. selfenergySum:
    V_rs = F^H V F and (W - V)_rs = F^H V^{1/2} (eps~^-1 - I) V^{1/2} F with an explicit
    DFT matrix F on the list, and the pair functions psi_n conj(psi_i) on the grid."""
    inp = tiny
    einv = oracle.eps_inv_isdf(inp)
    f = dft_matrix(inp.n, inp.miller)
    sv = np.sqrt(oracle.coulomb_diag(inp.miller, inp.cell, inp.v_scale))
    v_rs = np.conj(f.T) @ (sv[:, None] ** 2 * f)
    wv_rs = np.conj(f.T) @ (sv[:, None] * (einv - np.eye(inp.ng)) * sv[None, :]) @ f
    ns = inp.nv + inp.nc
    p = inp.psi_t
    ref = np.zeros((3, ns))
    for n in range(ns):
        for i in range(ns):
            m = p[n] * np.conj(p[i])
            if i < inp.nv:
                ref[0, n] -= np.real(np.conj(m) @ wv_rs @ m)
                ref[1, n] -= np.real(np.conj(m) @ v_rs @ m)
            ref[2, n] += 0.5 * np.real(np.conj(m) @ wv_rs @ m)
    got = osig.sigma_exact(inp, einv)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["fullrank", "fullrank_real"])
def test_fullrank_isdf_equals_exact(name):
    """With as many points as independent pair functions in each set, the ISDF fits are
    exact, so sigma_isdf equals sigma_exact."""
    inp = synth.make_inputs(name)
    ns = inp.nv + inp.nc
    # independent pair functions: every pair for complex orbitals; for real ones the
    # products are symmetric, so the occupied x occupied pairs of the vn set and every
    # swapped pair of the nn set repeat
    nvn = inp.nv * ns if inp.is_complex else inp.nv * ns - inp.nv * (inp.nv - 1) // 2
    nnn = ns * ns if inp.is_complex else ns * (ns + 1) // 2
    mu_vn, mu_nn = synth.sigma_points(inp, nvn, nnn)
    einv = oracle.eps_inv_isdf(inp)
    got = osig.sigma_isdf(inp, mu_vn, mu_nn, einv)
    ref = osig.sigma_exact(inp, einv)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


def test_pair_set_fit_matches_lstsq(tiny):
    """The normal-equation fit of a pair set equals numpy least squares on the explicit pairs."""
    mu_vn, _ = synth.sigma_points(tiny)
    ns = tiny.nv + tiny.nc
    a, b = np.arange(tiny.nv), np.arange(ns)
    th = osig.pair_set_fit(tiny.psi_t, a, b, mu_vn)
    c = osig.pair_set_coefficients(tiny.psi_t, a, b, mu_vn)
    m = osig.pair_set_functions(tiny.psi_t, a, b)
    sol, *_ = np.linalg.lstsq(c.T, m, rcond=None)
    assert np.abs(th - sol.T).max() <= 1e-9 * np.abs(sol).max()


def test_signs(cfg0):
    """V is positive semidefinite and eps~^-1 - I negative semidefinite (static), so
    Sigma_X <= 0, Sigma_SEX_X >= 0 and Sigma_COH <= 0 for every band, in both modes."""
    einv = oracle.eps_inv_isdf(cfg0)
    mu_vn, mu_nn = synth.sigma_points(cfg0)
    for s in (osig.sigma_exact(cfg0, einv), osig.sigma_isdf(cfg0, mu_vn, mu_nn, einv)):
        assert (s[0] >= 0).all() and (s[1] <= 0).all() and (s[2] <= 0).all()
        assert np.abs(s[1]).min() > 0


def test_phase_invariance(tiny):
    """psi_n -> exp(i theta_n) psi_n leaves every diagonal unchanged (exact and ISDF)."""
    rng = np.random.default_rng(3)
    einv = oracle.eps_inv_isdf(tiny)
    mu_vn, mu_nn = synth.sigma_points(tiny)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, tiny.nv + tiny.nc))
    t2 = synth.Inputs(**{**tiny.__dict__, "psi_t": tiny.psi_t * ph[:, None]})
    for f in (lambda i: osig.sigma_exact(i, einv), lambda i: osig.sigma_isdf(i, mu_vn, mu_nn, einv)):
        a, b = f(tiny), f(t2)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_isdf_error_falls_with_points(cfg0):
    """The ISDF self-energies approach the exact ones as both point sets grow."""
    einv = oracle.eps_inv_isdf(cfg0)
    ref = osig.sigma_exact(cfg0, einv)
    errs = []
    for scale in (0.5, 1.0, 2.0):
        dvn, dnn = synth.sigma_point_counts(cfg0)
        mu_vn, mu_nn = synth.sigma_points(cfg0, int(dvn * scale), int(dnn * scale))
        errs.append(np.abs(osig.sigma_isdf(cfg0, mu_vn, mu_nn, einv) - ref).max())
    assert errs[0] > errs[1] > errs[2]


def low_rank_hadamard_route(inp, mu_vn, mu_nn):
    """What the GPU path computes (Algorithm 3 steps 2-6 in the X formulation):
    X_s = V^{1/2} F Z_s (Z_s = M_s C_s^H), S_s = C_s C_s^H, A_s = X_s^H X,
    H = X^H X - S M^{-1} S, W_s = -S_s^{-1} A_s H^{-1} A_s^H S_s^{-1},
    V_vn = S_vn^{-1} X_vn^H X_vn S_vn^{-1}; then eq. Hadamard on the points:
    Sigma = coef diag(Psi_s^H (W_s (.) G) Psi_s), G(mu, nu) = sum_{i in set} psi_i(r_mu) conj(psi_i(r_nu))."""
    ns = inp.nv + inp.nc
    sv = np.sqrt(oracle.coulomb_diag(inp.miller, inp.cell, inp.v_scale))[:, None]
    allr, occ = np.arange(ns), np.arange(inp.nv)

    def xs(a_rows, b_rows, mu):
        c = osig.pair_set_coefficients(inp.psi_t, a_rows, b_rows, mu)
        m = osig.pair_set_functions(inp.psi_t, a_rows, b_rows)
        z = m.T @ np.conj(c.T)
        x = sv * oracle.dft_rows(np.ascontiguousarray(z.T), inp.n, inp.miller).T
        return x, c @ np.conj(c.T)

    x, s = xs(occ, np.arange(inp.nv, ns), inp.mu_idx)
    mm = oracle.core_matrix(inp.psi_t, inp.energies, inp.nv, inp.mu_idx)
    hinv = np.linalg.inv(np.conj(x.T) @ x - s @ np.linalg.inv(mm) @ s)
    out = np.zeros((3, ns))
    for k, (a_rows, mu, rows) in enumerate(((occ, mu_vn, occ), (allr, mu_nn, allr))):
        xk, sk = xs(a_rows, allr, mu)
        ski = np.linalg.inv(sk)
        ak = np.conj(xk.T) @ x
        wk = -ski @ ak @ hinv @ np.conj(ak.T) @ ski
        pts = inp.psi_t[:, mu]                                   # (N, N_mu)
        g = pts[rows].T @ np.conj(pts[rows])                     # sum over the set
        diag = lambda y: np.real(np.einsum("mn,mk,kn->n", np.conj(pts.T), y * g, pts.T))
        if k == 0:
            out[0] = -diag(wk)
            out[1] = -diag(ski @ (np.conj(xk.T) @ xk) @ ski)
        else:
            out[2] = 0.5 * diag(wk)
    return out


@pytest.mark.parametrize("name", ["tiny", "cfg0", "mid_real"])
def test_low_rank_hadamard_route_equals_plain_sums(name):
    inp = synth.make_inputs(name)
    mu_vn, mu_nn = synth.sigma_points(inp)
    einv = oracle.eps_inv_isdf(inp)
    ref = osig.sigma_isdf(inp, mu_vn, mu_nn, einv)
    got = low_rank_hadamard_route(inp, mu_vn, mu_nn)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
