"""FP64 oracle gradient of L = Re tr(W eps~^{-1}) for the ISDF route.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the GPU library.

The dense ISDF definition of ``dielectric.eps_inv_isdf`` is written out again
in torch CPU operations on complex128, so that torch's automatic
differentiation supplies the derivative of the definition itself:
  * C(mu; (i, j)) = conj(psi_i(r_mu)) psi_j(r_mu) formed explicitly (eq. ISDF);
  * Theta from the least-squares normal equations Theta (C C^H) = M_vc C^H,
    M_vc(k; (i, j)) = conj(psi_i(r_k)) psi_j(r_k) formed explicitly;
  * Theta_G = unitary DFT of Theta on the plane-wave list, U = V^{1/2} Theta_G;
  * core M = f C diag(w) C^H, w_ij = Delta / (Delta^2 + omega^2) (eq. COmegaCstar,
    eq. Hedin_fourier at imaginary frequency);
  * eps~ = I - U M U^H, its dense inverse, and L = Re tr(W eps~^{-1}).
No Sherman-Morrison-Woodbury step and no hand-written adjoint: the derivative
is the one autograd takes of the definition.  Small inputs only (the pair
matrices are Nr x Nv Nc).

Gradient convention (pinned in tests/test_oracle_pins.py by central
differences): for a complex variable z = x + i y the gradient is
dL/dx + i dL/dy; for the energies it is dL/d eps_n.  The gradient with respect
to the orbitals is the total derivative with respect to each grid value
psi_n(r_k); its columns at the interpolation points r_mu are the orbital
samples the points see (through C, S, M and the grid rows of M_vc).
"""
from __future__ import annotations

import numpy as np
import torch

from .dielectric import PAIR_FACTOR, coulomb_diag


def eps_inv_isdf_torch(psi_t: torch.Tensor, energies: torch.Tensor, inp, f=PAIR_FACTOR, omega=0.0,
                       v_scale=None) -> torch.Tensor:
    """eps~^{-1} (NG x NG) by the dense ISDF definition, differentiable in psi_t and energies."""
    nv, n = inp.nv, inp.n
    mu = torch.as_tensor(np.asarray(inp.mu_idx, dtype=np.int64))
    pv, pc = psi_t[:nv], psi_t[nv:]
    nc, nmu = pc.shape[0], len(inp.mu_idx)
    a, b = pv[:, mu], pc[:, mu]                                        # orbitals at the points
    c = (a.conj()[:, None, :] * b[None, :, :]).reshape(nv * nc, nmu).T  # C, (N_mu, Nv Nc), pair i-major
    mvc = (pv.conj()[:, None, :] * pc[None, :, :]).reshape(nv * nc, -1).T  # M_vc, (Nr, Nv Nc)
    s = c @ c.conj().T
    z = mvc @ c.conj().T                                               # M_vc C^H
    theta = torch.linalg.solve(s, z.conj().T).conj().T                 # Theta S = M_vc C^H (S Hermitian)
    cube = theta.T.reshape(nmu, n, n, n)                               # [mu, i2, i1, i0]
    fc = torch.fft.fftn(cube, dim=(1, 2, 3), norm="ortho")
    m = np.mod(np.asarray(inp.miller, dtype=np.int64), n)
    tg = fc[:, m[:, 2], m[:, 1], m[:, 0]].T                            # Theta_G, (NG, N_mu)
    vs = inp.v_scale if v_scale is None else v_scale
    v = torch.as_tensor(coulomb_diag(inp.miller, inp.cell, vs))
    u = torch.sqrt(v)[:, None].to(tg.dtype) * tg
    d = energies[:nv, None] - energies[None, nv:]
    w = (d / (d * d + omega * omega)).reshape(-1)
    core = f * (c * w[None, :].to(c.dtype)) @ c.conj().T
    eps = torch.eye(inp.ng, dtype=u.dtype) - u @ core @ u.conj().T
    return torch.linalg.inv(eps)


def loss(e_inv: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """L = Re tr(W eps~^{-1})."""
    return (w * e_inv.T).sum().real


def loss_and_grad(inp, w: np.ndarray, f=PAIR_FACTOR, omega=0.0, v_scale=None):
    """(L, dL/d energies (N,), dL/d psi (N, Nr) complex) by autograd through the definition."""
    psi = torch.tensor(np.asarray(inp.psi_t, dtype=np.complex128), requires_grad=True)
    e = torch.tensor(np.asarray(inp.energies, dtype=np.float64), requires_grad=True)
    lval = loss(eps_inv_isdf_torch(psi, e, inp, f, omega, v_scale), torch.as_tensor(w))
    lval.backward()
    return float(lval.item()), e.grad.numpy().copy(), psi.grad.numpy().copy()


def loss_value(inp, psi_t: np.ndarray, energies: np.ndarray, w: np.ndarray, f=PAIR_FACTOR, omega=0.0,
               v_scale=None) -> float:
    """L at given orbitals and energies (no gradient), for finite differences."""
    with torch.no_grad():
        e_inv = eps_inv_isdf_torch(torch.as_tensor(np.asarray(psi_t, dtype=np.complex128)),
                                   torch.as_tensor(np.asarray(energies, dtype=np.float64)), inp, f, omega, v_scale)
        return float(loss(e_inv, torch.as_tensor(w)).item())
