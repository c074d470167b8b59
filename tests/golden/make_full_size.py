"""Write the stored oracle reference for the 64^3 workload (tests/golden/cfg2_oracle.npz).

    python tests/golden/make_full_size.py        # a few minutes of CPU, ~20 GB of RAM

Calls only the CPU oracle (``oracle``) and the seeded input generator (``synth``);
nothing here touches the GPU library.  The 64^3 workload (256 / 1024 states, 2048
interpolation points, 8192 plane waves, complex orbitals, seed 2) is too large for
the oracle's dense route to run inside a test, so this script runs it once and
keeps what the full-size parity tests compare element by element:

  * eps~^{-1} (isdf mode: dense eps~ = I - U M U^H, LU inverse) at 16 sampled rows,
    with the Frobenius norms of eps~^{-1} and of eps~^{-1} - I over the whole matrix;
  * Theta (the least-squares ISDF fit) at 16 sampled grid rows;
  * U = V^{1/2} F Theta at 16 sampled plane-wave rows;
  * 64 sampled entries of the core M = f C Omega^{-1} C^H;
  * the interpolation points and a fingerprint of the orbitals, so a test can
    confirm that the generator still produces these inputs.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "cfg2_oracle.npz")


def sample_rows(n, count, seed):
    rng = np.random.default_rng(seed)
    fixed = np.array([0, 1, 2, 3, n // 2, n - 1])
    rest = rng.choice(np.setdiff1d(np.arange(n), fixed), size=count - len(fixed), replace=False)
    return np.sort(np.concatenate([fixed, rest])).astype(np.int64)


def main():
    t0 = time.time()
    inp = synth.make_inputs("cfg2")
    print(f"inputs {time.time() - t0:.1f}s", flush=True)
    st = oracle.isdf_stages_chunked(inp)
    print(f"stages {time.time() - t0:.1f}s", flush=True)
    u, m = st["u"], st["m"]
    eps = np.eye(inp.ng) - u @ m @ np.conj(u.T)
    inv = oracle.invert_lu(eps)
    del eps
    print(f"inverse {time.time() - t0:.1f}s", flush=True)
    eye = np.eye(inp.ng)
    rows = sample_rows(inp.ng, 16, 20)
    th_rows = sample_rows(inp.nr, 16, 21)
    u_rows = sample_rows(inp.ng, 16, 22)
    rng = np.random.default_rng(23)
    pairs = rng.integers(0, inp.nmu, size=(64, 2))
    pairs[:8, 1] = pairs[:8, 0]
    np.savez_compressed(
        OUT,
        mu_idx=inp.mu_idx, psi_fingerprint=inp.psi_t[:, :16].copy(), energies=inp.energies,
        rows=rows, eps_rows=inv[rows],
        norm_eps=np.linalg.norm(inv), norm_screen=np.linalg.norm(inv - eye),
        max_screen=np.abs(inv - eye).max(),
        theta_rows_idx=th_rows, theta_rows=st["theta"][th_rows],
        u_rows_idx=u_rows, u_rows=u[u_rows],
        m_pairs=pairs, m_entries=m[pairs[:, 0], pairs[:, 1]])
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e6:.1f} MB) in {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main()
