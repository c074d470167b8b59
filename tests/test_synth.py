"""Seeded input generator: determinism and the recipe's stated properties."""
import numpy as np

import synth


def test_deterministic_and_orthonormal():
    a = synth.make_inputs("mid")
    b = synth.make_inputs("mid")
    np.testing.assert_array_equal(a.psi_t, b.psi_t)
    np.testing.assert_array_equal(a.mu_idx, b.mu_idx)
    g = a.psi_t.conj() @ a.psi_t.T
    assert np.abs(g - np.eye(len(g))).max() < 1e-13


def test_energies_and_points():
    x = synth.make_inputs("cfg0")
    ev, ec = x.energies[: x.nv], x.energies[x.nv:]
    assert np.all(np.diff(ev) >= 0) and np.all(np.diff(ec) >= 0)
    assert ev.max() < ec.min()
    assert ev.min() >= -20 / synth.HARTREE_EV and ec.max() <= 30 / synth.HARTREE_EV
    assert len(np.unique(x.mu_idx)) == x.nmu and x.mu_idx.min() >= 0 and x.mu_idx.max() < x.nr


def test_orbitals_are_band_limited():
    x = synth.make_inputs("tiny")
    n = x.n
    s_cut = synth.lowpass_cut(n, x.nv + x.nc)
    spec = np.fft.fftn(x.psi_t.reshape(-1, n, n, n), axes=(1, 2, 3))
    f = synth.freq_grid(n)
    m2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    assert np.abs(spec[:, m2 > s_cut]).max() < 1e-12


def test_miller_list_order():
    m = synth.miller_list(12, 256)
    assert m.dtype == np.int32 and m.shape == (256, 3)
    assert np.all(m[0] == 0)
    m2 = (m.astype(np.int64) ** 2).sum(1)
    assert np.all(np.diff(m2) >= 0)
    keys = [tuple([int(a)] + list(map(int, r))) for a, r in zip(m2, m)]
    assert keys == sorted(keys)
    assert len({tuple(r) for r in m.tolist()}) == 256
    assert m.min() >= -6 and m.max() < 6
