"""Pins that tie the FP64 oracle to the paper and to mathematics, not to itself.

Each test names the fact it checks.  Plausible oracle mistakes and the pin that
catches them:
  dropped or doubled pair factor f, wrong sign of Delta, sqrt(V) misplaced
      -> single-pair Sherman-Morrison closed form, brute-force chi0
  transposed / conjugated operand in chi0 or C
      -> brute-force chi0 (complex), full-rank ISDF == exact
  wrong DFT sign, axis order or Miller indexing
      -> plane-wave delta, brute-force chi0 with an explicit DFT matrix,
         grid-translation phase
  wrong least-squares fit (Hadamard factorisation)
      -> brute-force lstsq on the explicit pair matrix, interpolation property
  wrong Coulomb kernel -> closed form at |m| = 1
"""
import numpy as np
import pytest

import oracle
import synth


def dft_matrix(n, miller):
    """Explicit unitary DFT rows exp(-2 pi i m . (i0, i1, i2) / n) / sqrt(Nr), from the definition."""
    k = np.arange(n ** 3)
    i0, i1, i2 = k % n, (k // n) % n, k // (n * n)
    ph = (np.outer(miller[:, 0], i0) + np.outer(miller[:, 1], i1) + np.outer(miller[:, 2], i2))
    return np.exp(-2j * np.pi * ph / n) / np.sqrt(n ** 3)


@pytest.fixture(scope="module")
def cfg0():
    return synth.make_inputs("cfg0")


@pytest.fixture(scope="module")
def tiny():
    return synth.make_inputs("tiny")


@pytest.fixture(scope="module")
def tiny_real():
    return synth.make_inputs("tiny", complex=False)


# ---------------------------------------------------------------------------
# Textbook identities and closed forms
# ---------------------------------------------------------------------------
def test_smw_formula_textbook():
    """eq. S--M--W on random matrices against numpy's dense inverse."""
    rng = np.random.default_rng(11)
    n, k = 30, 7
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 8 * np.eye(n)
    u = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    v = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    ai = np.linalg.inv(a)
    smw = ai - ai @ u @ np.linalg.inv(np.eye(k) + v.conj().T @ ai @ u) @ v.conj().T @ ai
    ref = np.linalg.inv(a + u @ v.conj().T)
    assert np.abs(smw - ref).max() < 1e-12


def test_coulomb_closed_form(cfg0):
    """V(G) = v_scale 4 pi / |G|^2 with G = 2 pi m / L: at |m| = 1 it is v_scale L^2 / pi; V(0) = 0."""
    v = oracle.coulomb_diag(cfg0.miller, cfg0.cell, 3.5)
    m2 = (cfg0.miller.astype(np.int64) ** 2).sum(1)
    assert v[0] == 0.0 and m2[0] == 0
    one = m2 == 1
    assert one.sum() == 6
    np.testing.assert_allclose(v[one], 3.5 * cfg0.L ** 2 / np.pi, rtol=1e-14)
    nz = m2 > 0
    np.testing.assert_allclose(v[nz] * m2[nz], 3.5 * cfg0.L ** 2 / np.pi, rtol=1e-14)


def test_dft_plane_wave_delta():
    """A grid plane wave exp(+2 pi i m0 . k / n) / sqrt(Nr) transforms to a unit delta at m0."""
    n = 6
    miller = synth.miller_list(n, n ** 3)
    m0 = np.array([2, -1, 3])
    k = np.arange(n ** 3)
    i0, i1, i2 = k % n, (k // n) % n, k // (n * n)
    x = np.exp(2j * np.pi * (m0[0] * i0 + m0[1] * i1 + m0[2] * i2) / n) / np.sqrt(n ** 3)
    y = oracle.dft_rows(x[None, :], n, miller)[0]
    hit = np.all(np.mod(miller - m0, n) == 0, axis=1)
    assert hit.sum() == 1
    np.testing.assert_allclose(y[hit], 1.0, atol=1e-13)
    assert np.abs(y[~hit]).max() < 1e-13


def test_dft_matches_explicit_matrix_and_parseval(tiny):
    n = tiny.n
    miller = synth.miller_list(n, n ** 3)
    x = tiny.psi_t[:4]
    y = oracle.dft_rows(x, n, miller)
    np.testing.assert_allclose(y, x @ dft_matrix(n, miller).T, atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(y, axis=1), np.linalg.norm(x, axis=1), rtol=1e-13)


def test_single_pair_sherman_morrison_closed_form():
    """One occupied and one empty state: eps~ = I + a a^H with a = sqrt(V) sqrt(f/|Delta|) F m,
    so eps~^{-1} = I - a a^H / (1 + a^H a) (rank-one update, Sherman-Morrison)."""
    inp = synth.make_inputs("tiny", nv=1, nc=1, nmu=1)
    psi, e = inp.psi_t, inp.energies
    m = np.conj(psi[0]) * psi[1]
    fm = dft_matrix(inp.n, inp.miller) @ m
    v = oracle.coulomb_diag(inp.miller, inp.cell, inp.v_scale)
    delta = e[0] - e[1]
    assert delta < 0
    a = np.sqrt(v) * np.sqrt(2.0 / abs(delta)) * fm
    ref = np.eye(len(a)) - np.outer(a, a.conj()) / (1.0 + np.vdot(a, a).real)
    got = oracle.eps_inv_exact(inp)
    assert np.abs(got - ref).max() < 1e-13
    assert np.abs(ref - np.eye(len(a))).max() > 1e-4  # non-trivial screening


# ---------------------------------------------------------------------------
# chi0 by brute force from the paper's sums
# ---------------------------------------------------------------------------
def test_chi0_bruteforce_real(tiny_real):
    """Real orbitals: the literal four-orbital sum of eq. Hedin_G0W0 (factor 2, 1/(eps_i - eps_j))
    in real space, taken to plane waves with an explicit DFT matrix."""
    inp = tiny_real
    psi, e, nv = inp.psi_t, inp.energies, inp.nv
    nr = inp.nr
    chi_r = np.zeros((nr, nr))
    for i in range(nv):
        for j in range(nv, len(e)):
            u = psi[i] * np.conj(psi[j])            # psi_i(r) conj(psi_j(r))
            w = np.conj(psi[i]) * psi[j]            # conj(psi_i(r')) psi_j(r')
            chi_r += 2.0 * np.outer(u, w).real / (e[i] - e[j])
    f = dft_matrix(inp.n, inp.miller)
    ref = f @ chi_r @ f.conj().T
    got = oracle.chi0_exact_pw(psi, e, nv, inp.n, inp.miller)
    assert np.abs(got - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_chi0_bruteforce_complex(tiny):
    """Complex orbitals: eq. matrices literally, chi0 = 2 M Omega^{-1} M^H with M columns conj(psi_i) psi_j."""
    inp = tiny
    psi, e, nv = inp.psi_t, inp.energies, inp.nv
    cols, diag = [], []
    for i in range(nv):
        for j in range(nv, len(e)):
            cols.append(np.conj(psi[i]) * psi[j])
            diag.append(e[i] - e[j])
    m = np.array(cols).T
    chi_r = 2.0 * m @ np.diag(1.0 / np.array(diag)) @ m.conj().T
    f = dft_matrix(inp.n, inp.miller)
    ref = f @ chi_r @ f.conj().T
    got = oracle.chi0_exact_pw(psi, e, nv, inp.n, inp.miller)
    assert np.abs(got - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())
    # chi0 is Hermitian negative semidefinite
    assert np.abs(got - got.conj().T).max() < 1e-14
    assert np.linalg.eigvalsh(got).max() < 1e-12


# ---------------------------------------------------------------------------
# ISDF fit and core
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["tiny", "cfg0"])
def test_theta_matches_bruteforce_lstsq(name):
    inp = synth.make_inputs(name)
    th = oracle.isdf_fit(inp.psi_t, inp.nv, inp.mu_idx)
    ref = oracle.isdf_fit_bruteforce(inp.psi_t, inp.nv, inp.mu_idx)
    assert np.abs(th - ref).max() < 1e-11 * np.abs(ref).max()


def test_theta_interpolation_property(cfg0):
    """At the interpolation points the least-squares fit reproduces C exactly: Theta(r_mu, :) = I."""
    th = oracle.isdf_fit(cfg0.psi_t, cfg0.nv, cfg0.mu_idx)
    assert np.abs(th[cfg0.mu_idx] - np.eye(cfg0.nmu)).max() < 1e-11


def test_theta_rows_matches_full_fit(cfg0):
    th = oracle.isdf_fit(cfg0.psi_t, cfg0.nv, cfg0.mu_idx)
    rows = np.array([0, 5, 777, cfg0.nr - 1])
    got = oracle.theta_rows(cfg0.psi_t, cfg0.nv, cfg0.mu_idx, rows)
    assert np.abs(got - th[rows]).max() < 1e-11 * np.abs(th).max()


def test_core_matrix_by_loops(tiny):
    """eq. COmegaCstar entry by entry with Python loops (times f = 2); Hermitian, negative definite."""
    inp = tiny
    psi, e, nv, mu = inp.psi_t, inp.energies, inp.nv, inp.mu_idx
    nmu = len(mu)
    ref = np.zeros((nmu, nmu), dtype=complex)
    for a in range(nmu):
        for b in range(nmu):
            s = 0.0
            for i in range(nv):
                for j in range(nv, len(e)):
                    s += (np.conj(psi[i, mu[a]]) * psi[i, mu[b]] * psi[j, mu[a]] * np.conj(psi[j, mu[b]])
                          / (e[i] - e[j]))
            ref[a, b] = 2.0 * s
    got = oracle.core_matrix(psi, e, nv, mu)
    assert np.abs(got - ref).max() < 1e-14
    assert np.abs(got - got.conj().T).max() < 1e-15
    assert np.linalg.eigvalsh(got).max() < 0
    pairs = [(0, 0), (3, 7), (11, 2)]
    ent = oracle.core_entries(psi, e, nv, mu, pairs)
    np.testing.assert_allclose(ent, [ref[a, b] for a, b in pairs], atol=1e-15)


@pytest.mark.parametrize("name", ["tiny", "cfg0", "mid"])
def test_bounded_memory_forms_equal_plain_definitions(name):
    """The bounded-memory forms used for the full-size references (S and M summed over
    the occupied index, Theta by blocks of grid rows, Theta_G by blocks of columns)
    equal the plain definitions; small blocks force several of each.  The plain
    definitions are themselves pinned by the brute-force tests in this file."""
    inp = synth.make_inputs(name)
    ref = oracle.isdf_stages(inp)
    got = oracle.isdf_stages_chunked(inp, chunk=97, mu_chunk=7)
    for k in ("theta", "theta_g", "u", "m"):
        assert np.abs(got[k] - ref[k]).max() <= 1e-12 * np.abs(ref[k]).max(), k
    s = oracle.isdf_gram(inp.psi_t, inp.nv, inp.mu_idx)
    assert np.abs(got["s"] - s).max() <= 1e-13 * np.abs(s).max()


# ---------------------------------------------------------------------------
# Exact-rank special cases reduce to the dense LU inverse
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["fullrank", "fullrank_real"])
def test_fullrank_isdf_equals_exact(name):
    """With N_mu = Nv Nc the ISDF fit is exact, so the ISDF inverse equals the definition."""
    inp = synth.make_inputs(name)
    assert inp.nmu == inp.nv * inp.nc
    ex = oracle.eps_inv_exact(inp)
    st = oracle.isdf_stages(inp)
    pm = oracle.pair_products(inp.psi_t, inp.nv).T
    c = oracle.isdf_coefficients(inp.psi_t, inp.nv, inp.mu_idx)
    assert np.abs(st["theta"] @ c - pm).max() < 1e-10 * np.abs(pm).max()
    iso = oracle.eps_inv_isdf(inp, stages=st)
    assert np.linalg.norm(iso - ex) / np.linalg.norm(ex) < 1e-10
    smw = oracle.eps_inv_smw(st["u"], st["m"])
    assert np.linalg.norm(smw - ex) / np.linalg.norm(ex) < 1e-10


@pytest.mark.parametrize("name", ["tiny", "cfg0"])
def test_exact_rank_smw_equals_direct_inverse(name):
    """SMW with P = M_vc and C = I (rank Nv Nc, no ISDF) reproduces the dense LU inverse to 1e-10."""
    inp = synth.make_inputs(name)
    pm = oracle.pair_products(inp.psi_t, inp.nv)                    # (NvNc, Nr)
    u = np.sqrt(oracle.coulomb_factor(inp))[:, None] * oracle.dft_rows(pm, inp.n, inp.miller).T
    core = 2.0 * np.diag(oracle.pair_weights(inp.energies, inp.nv).ravel())
    smw = oracle.eps_inv_smw(u, core)
    ex = oracle.eps_inv_exact(inp)
    assert np.linalg.norm(smw - ex) / np.linalg.norm(ex) < 1e-10


# ---------------------------------------------------------------------------
# Invariants of eps~^{-1}
# ---------------------------------------------------------------------------
def _check_invariants(inv, eps=None):
    assert np.abs(inv - inv.conj().T).max() < 1e-13
    ev = np.linalg.eigvalsh((inv + inv.conj().T) / 2)
    assert ev.min() > 0 and ev.max() < 1 + 1e-12       # eps~ = I + X, X >= 0
    e0 = np.zeros(len(inv)); e0[0] = 1.0
    assert np.abs(inv[0] - e0).max() < 1e-14 and np.abs(inv[:, 0] - e0).max() < 1e-14
    if eps is not None:
        assert np.abs(inv @ eps - np.eye(len(inv))).max() < 1e-12


@pytest.mark.parametrize("name", ["cfg0", "mid_real"])
def test_invariants_exact_and_isdf(name):
    inp = synth.make_inputs(name)
    v = oracle.coulomb_factor(inp)
    chi = oracle.chi0_exact_pw(inp.psi_t, inp.energies, inp.nv, inp.n, inp.miller)
    eps = oracle.eps_tilde(chi, v)
    _check_invariants(oracle.invert_lu(eps), eps)
    st = oracle.isdf_stages(inp)
    iso = oracle.eps_inv_isdf(inp, stages=st)
    _check_invariants(iso, np.eye(inp.ng) - st["u"] @ st["m"] @ st["u"].conj().T)


def test_invariance_shift_phase_permutation(tiny):
    inp = tiny
    base = oracle.eps_inv_isdf(inp)
    base_ex = oracle.eps_inv_exact(inp)
    rng = np.random.default_rng(3)
    # energy shift
    sh = synth.Inputs(**{**inp.__dict__, "energies": inp.energies + 0.37})
    assert np.abs(oracle.eps_inv_isdf(sh) - base).max() < 1e-12
    # per-orbital phases
    ph = np.exp(2j * np.pi * rng.random(inp.psi_t.shape[0]))
    pp = synth.Inputs(**{**inp.__dict__, "psi_t": inp.psi_t * ph[:, None]})
    assert np.abs(oracle.eps_inv_isdf(pp) - base).max() < 1e-12
    assert np.abs(oracle.eps_inv_exact(pp) - base_ex).max() < 1e-12
    # permutation within v and within c (with their energies)
    perm = np.concatenate([rng.permutation(inp.nv), inp.nv + rng.permutation(inp.nc)])
    pr = synth.Inputs(**{**inp.__dict__, "psi_t": inp.psi_t[perm], "energies": inp.energies[perm]})
    assert np.abs(oracle.eps_inv_isdf(pr) - base).max() < 1e-12


def test_grid_translation_phase(tiny):
    """psi(r) -> psi(r - t) multiplies eps~^{-1}(G, G') by exp(-2 pi i (m - m') . t / n)."""
    inp = tiny
    n = inp.n
    t = np.array([2, 0, 3])  # (x, y, z) steps
    cube = inp.psi_t.reshape(-1, n, n, n)                        # [state, z, y, x]
    moved = np.roll(cube, shift=(t[2], t[1], t[0]), axis=(1, 2, 3)).reshape(inp.psi_t.shape)
    k = inp.mu_idx
    x, y, z = k % n, (k // n) % n, k // (n * n)
    mu2 = (((x + t[0]) % n) + n * (((y + t[1]) % n) + n * ((z + t[2]) % n))).astype(np.int32)
    tr = synth.Inputs(**{**inp.__dict__, "psi_t": np.ascontiguousarray(moved), "mu_idx": mu2})
    ph = np.exp(-2j * np.pi * (inp.miller @ t) / n)
    expect_ex = ph[:, None] * oracle.eps_inv_exact(inp) * ph.conj()[None, :]
    assert np.abs(oracle.eps_inv_exact(tr) - expect_ex).max() < 1e-12
    expect_is = ph[:, None] * oracle.eps_inv_isdf(inp) * ph.conj()[None, :]
    assert np.abs(oracle.eps_inv_isdf(tr) - expect_is).max() < 1e-12


def test_isdf_error_falls_with_nmu():
    """ISDF error on eps~^{-1} decreases as N_mu grows and vanishes at N_mu = Nv Nc."""
    base = synth.make_inputs("cfg0")
    ex = oracle.eps_inv_exact(base)
    errs = []
    for nmu in (24, 96, 192):
        inp = synth.make_inputs("cfg0", nmu=nmu)
        iso = oracle.eps_inv_isdf(inp)
        errs.append(np.linalg.norm(iso - ex) / np.linalg.norm(ex - np.eye(len(ex))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-10


def test_frequency_limits(tiny):
    """omega = 0 is the static matrix; the screening vanishes as omega grows (eq. Hedin_fourier at i omega)."""
    st0 = oracle.eps_inv_isdf(tiny)
    np.testing.assert_array_equal(oracle.eps_inv_isdf(tiny, omega=0.0), st0)
    prev = np.linalg.norm(st0 - np.eye(tiny.ng))
    for om in (0.1, 1.0, 10.0, 1e4):
        cur = np.linalg.norm(oracle.eps_inv_isdf(tiny, omega=om) - np.eye(tiny.ng))
        assert cur < prev
        prev = cur
    assert prev < 1e-6


def test_pair_weights_two_pole_sum():
    """At i omega the two pole terms 1/(i w + D) + 1/(-i w + D) equal 2 D / (D^2 + w^2)."""
    e = np.array([-0.5, -0.3, 0.2, 0.9])
    for om in (0.0, 0.05, 3.0):
        w = oracle.pair_weights(e, 2, om)
        d = e[:2, None] - e[None, 2:]
        two = 1.0 / (1j * om + d) + 1.0 / (-1j * om + d)
        np.testing.assert_allclose(2 * w, two.real, rtol=1e-14)
        assert np.abs(two.imag).max() < 1e-14


# ---- full-grid Coulomb Gram (the paper's P^H V P over the whole grid) ----------------
def test_full_grid_list_is_a_permutation_of_the_grid():
    inp = synth.make_inputs("tiny")
    full = oracle.full_grid_list(inp.miller, inp.n)
    assert full.shape == (inp.nr, 3)
    assert np.array_equal(full[:inp.ng], inp.miller)
    key = (full[:, 0] % inp.n) + inp.n * ((full[:, 1] % inp.n) + inp.n * (full[:, 2] % inp.n))
    assert np.array_equal(np.sort(key), np.arange(inp.nr))


def test_full_grid_isdf_equals_exact_at_full_rank():
    """N_mu = Nv Nc: the ISDF route over the support (dense LU) equals chi0 from every
    pair over the whole grid (dense LU over all Nr plane waves)."""
    inp = synth.make_inputs("fullrank")
    a = oracle.eps_inv_isdf_full(inp)
    b = oracle.eps_inv_exact_full(inp)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-10


def test_full_grid_support_cut_is_exact():
    """Dropping the plane waves outside the pair products' Fourier support changes
    nothing at the level of the tolerance: compare with the uncut whole grid."""
    inp = synth.make_inputs("tiny")
    st = oracle.isdf_stages(inp)
    a = oracle.eps_inv_isdf_full(inp, stages=st)
    b = oracle.eps_inv_isdf_full(inp, stages=st, tol=0.0)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-12


def test_full_grid_differs_from_truncated():
    """The full-grid Gram is a different (larger) operator than the NG-truncated one:
    the NG blocks differ when NG does not cover the support, and agree when it does."""
    inp = synth.make_inputs("cfg0")
    st = oracle.isdf_stages(inp)
    full = oracle.eps_inv_isdf_full(inp, stages=st)
    trunc = oracle.eps_inv_isdf(inp, stages=st)
    assert np.linalg.norm(full - trunc) / np.linalg.norm(trunc) > 1e-8
    big = synth.make_inputs("tiny", ng=synth.make_inputs("tiny").nr)   # NG = every grid vector
    stb = oracle.isdf_stages(big)
    a = oracle.eps_inv_isdf_full(big, stages=stb)
    b = oracle.eps_inv_isdf(big, stages=stb)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-12


@pytest.mark.parametrize("name", ["tiny", "cfg0"])
def test_full_grid_smw_equals_dense_inverse(name):
    """SMW with the Gram summed over every grid vector equals the dense LU inverse of
    I - U M U^H over the whole grid (support-cut): two routes to the same NG block."""
    inp = synth.make_inputs(name)
    st = oracle.isdf_stages(inp)
    a = oracle.eps_inv_smw_full(inp, stages=st)
    b = oracle.eps_inv_isdf_full(inp, stages=st, tol=0.0)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-10


# ---- oracle gradient of L = Re tr(W eps~^{-1}) (autograd through the dense definition) ----
@pytest.mark.parametrize("name", ["tiny", "cfg0"])
def test_torch_definition_matches_numpy_oracle(name):
    """The torch transcription computes the same eps~^{-1} as the pinned NumPy route."""
    import torch
    from oracle import adjoint as oadj
    inp = synth.make_inputs(name)
    got = oadj.eps_inv_isdf_torch(torch.as_tensor(inp.psi_t.astype(np.complex128)),
                                  torch.as_tensor(inp.energies), inp).numpy()
    ref = oracle.eps_inv_isdf(inp)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("omega", [0.0, 0.05])
def test_oracle_gradient_matches_central_differences(omega):
    """dL/d eps_n and dL/dRe psi + i dL/dIm psi (at interpolation points and at one
    other grid point) against central differences, h = 1e-5: fixes the autograd
    route and the gradient convention independently of each other."""
    from oracle import adjoint as oadj
    inp = synth.make_inputs("tiny")
    w = synth.loss_weight(inp.ng)
    lval, ge, gpsi = oadj.loss_and_grad(inp, w, omega=omega)
    h = 1e-5
    psi0 = inp.psi_t.astype(np.complex128)
    for n in range(inp.nv + inp.nc):
        e1, e2 = inp.energies.copy(), inp.energies.copy()
        e1[n] += h
        e2[n] -= h
        fd = (oadj.loss_value(inp, psi0, e1, w, omega=omega) - oadj.loss_value(inp, psi0, e2, w, omega=omega)) / (2 * h)
        assert abs(fd - ge[n]) <= 1e-6 * max(1.0, abs(fd)), (n, fd, ge[n])
    other = int(np.setdiff1d(np.arange(inp.nr), inp.mu_idx)[3])
    cases = [(0, inp.mu_idx[0]), (inp.nv, inp.mu_idx[5]), (inp.nv + inp.nc - 1, inp.mu_idx[-1]), (1, other)]
    for n, k in cases:
        for step, part in ((h, "re"), (1j * h, "im")):
            p1, p2 = psi0.copy(), psi0.copy()
            p1[n, k] += step
            p2[n, k] -= step
            fd = (oadj.loss_value(inp, p1, inp.energies, w, omega=omega)
                  - oadj.loss_value(inp, p2, inp.energies, w, omega=omega)) / (2 * h)
            g = gpsi[n, k].real if part == "re" else gpsi[n, k].imag
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)), (n, k, part, fd, g)
    assert np.isfinite(lval)


# ---- Cauchy-integral core (Algorithm 2) ----------------------------------------------
def test_contour_quadrature_of_one_pole_pair():
    """Closed form: the contour rule gives 1/(a - b) for a below the top occupied
    energy and b in the empty band, within the cited quadrature bound."""
    from oracle import cauchy as oc
    rng = np.random.default_rng(3)
    for q, big_q in ((0.2, 1.0), (0.3, 25.0), (0.05, 40.0)):
        n = oc.nodes_for_tolerance(q, big_q, 1e-12)
        z, w = oc.contour_nodes(q, big_q, n)
        for _ in range(5):
            a = -rng.uniform(0.0, 3.0 * big_q)
            b = rng.uniform(q, big_q)
            s = -np.sum(w / ((z - a) * (z - b)))                   # counterclockwise upper half
            val = -(s - np.conj(s)) / (2j * np.pi)
            assert abs(val - 1.0 / (a - b)) * abs(a - b) <= 1e-11, (q, big_q, a, b, val)


def test_contour_half_plane_and_ends():
    """The mapped nodes lie in the upper half plane, and the ends of the segment map to
    real points below the gap and above the band (the contour separates them)."""
    from oracle import cauchy as oc
    q, big_q = 0.3, 25.0
    z, _ = oc.contour_nodes(q, big_q, 64)
    assert np.all(z.imag > 0)
    assert z[0].real < q and z[-1].real > big_q


@pytest.mark.parametrize("name", ["tiny", "cfg0", "mid"])
def test_cauchy_core_equals_direct_sum(name):
    """Algorithm 2 with the node count from eq. rel_err_Cauchy at 1e-13 equals the
    direct pair sum of eq. COmegaCstar; the adaptive rule reaches its tolerance."""
    from oracle import cauchy as oc
    inp = synth.make_inputs(name)
    ref = oracle.core_matrix(inp.psi_t, inp.energies, inp.nv, inp.mu_idx)
    _, q, big_q = oc.gap_and_width(inp.energies, inp.nv)
    m = oc.core_cauchy(inp.psi_t, inp.energies, inp.nv, inp.mu_idx, oc.nodes_for_tolerance(q, big_q, 1e-13))
    assert np.linalg.norm(m - ref) / np.linalg.norm(ref) < 1e-11
    assert np.array_equal(m, m.conj().T)
    ma, _ = oc.core_cauchy_adaptive(inp.psi_t, inp.energies, inp.nv, inp.mu_idx, 1e-10)
    assert np.linalg.norm(ma - ref) / np.linalg.norm(ref) < 1e-9


def test_cauchy_error_falls_with_nodes():
    """Geometric convergence in the node count, below the cited bound."""
    from oracle import cauchy as oc
    inp = synth.make_inputs("mid")
    ref = oracle.core_matrix(inp.psi_t, inp.energies, inp.nv, inp.mu_idx)
    _, q, big_q = oc.gap_and_width(inp.energies, inp.nv)
    errs = []
    for n in (4, 6, 8, 10):
        m = oc.core_cauchy(inp.psi_t, inp.energies, inp.nv, inp.mu_idx, n)
        errs.append(np.linalg.norm(m - ref) / np.linalg.norm(ref))
        assert errs[-1] <= np.exp(-np.pi ** 2 * n / (2 * np.log(big_q / q) + 6))
    assert all(b < a for a, b in zip(errs, errs[1:]))
