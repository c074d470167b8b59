"""GPU checks of the hand-written adjoint (isdf_eps_inv_grad, FP64 and mixed) of
L = Re tr(W eps~^{-1}).

Parity: loss and gradients against the oracle gradient (torch CPU autograd
through the dense ISDF definition, itself pinned by central differences in
test_oracle_pins.py).  Bars: loss <= 1e-10 relative; gradients <= 1e-8
relative Frobenius (FP64 on both sides; the routes differ in summation order
and go through inverses of condition number <= 2e2 here, so agreement to
~1e-12 is expected and 1e-8 leaves four digits of margin).

Consistency at sizes the oracle cannot reach: central differences (h = 1e-5)
of the FP64 GPU forward, including the 64^3 solid-like system.
"""
import numpy as np
import pytest
import torch

import paper_2403_12340_amd as isdf
import synth
from oracle import adjoint as oadj

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def relf(got, ref):
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("name,omega", [("tiny", 0.0), ("tiny", 0.05), ("cfg0", 0.0), ("fullrank", 0.0),
                                        ("mid", 0.02)])
def test_grad_matches_oracle(name, omega):
    inp = synth.make_inputs(name)
    w = synth.loss_weight(inp.ng)
    print(f"[grad] case={name} omega={omega}", flush=True)
    lref, ge_ref, gp_ref = oadj.loss_and_grad(inp, w, omega=omega)
    lval, ge, gp = isdf.eps_inv_grad(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller,
                                     isdf.problem_for(inp, "fp64"), dev(w), omega)
    ge, gp = ge.cpu().numpy(), gp.cpu().numpy()
    gp_ref = gp_ref[:, inp.mu_idx]
    e_l = abs(lval - lref) / max(1.0, abs(lref))
    e_e, e_p = relf(ge, ge_ref), relf(gp, gp_ref)
    print(f"  loss {lval:.6f} rel {e_l:.2e}  d/d eps rel-F {e_e:.2e}  d/d psi(r_mu) rel-F {e_p:.2e}", flush=True)
    assert e_l <= 1e-10, e_l
    assert e_e <= 1e-8, e_e
    assert e_p <= 1e-8, e_p


@pytest.mark.parametrize("name,omega", [("tiny", 0.0), ("cfg0", 0.0), ("mid", 0.02), ("core32", 0.0), ("core32", 0.03)])
def test_grad_mixed_matches_oracle(name, omega):
    """The mixed backward (ISDF_FP32: the contractions over the grid and over the
    points in FP32 on MFMA, everything else FP64) against the FP64 oracle gradient.
    Bar 1e-5 relative Frobenius: those contractions sum up to Nr terms of products
    rounded to FP32 (u = 6e-8, error growing like sqrt(Nr) u ~ 5e-6 at 20^3), and the
    result passes through S^{-1} and the SMW core (cond <= 2e2) only in FP64.  The
    core32 case (256 points, 64 empty states) recomputes M with the single-precision
    core of the forward pass (FP64 flush), as the larger systems do."""
    inp = synth.make_inputs(name)
    w = synth.loss_weight(inp.ng)
    print(f"[grad-mixed] case={name} omega={omega}", flush=True)
    lref, ge_ref, gp_ref = oadj.loss_and_grad(inp, w, omega=omega)
    lval, ge, gp = isdf.eps_inv_grad(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller,
                                     isdf.problem_for(inp, "fp32"), dev(w), omega)
    ge, gp = ge.cpu().numpy(), gp.cpu().numpy()
    gp_ref = gp_ref[:, inp.mu_idx]
    e_l = abs(lval - lref) / max(1.0, abs(lref))
    e_e, e_p = relf(ge, ge_ref), relf(gp, gp_ref)
    print(f"  loss {lval:.6f} rel {e_l:.2e}  d/d eps rel-F {e_e:.2e}  d/d psi(r_mu) rel-F {e_p:.2e}", flush=True)
    assert e_l <= 1e-5 and e_e <= 1e-5 and e_p <= 1e-5, (e_l, e_e, e_p)


def _loss_gpu(inp, prob, psi_t, energies, w_dev, omega, ws):
    e = isdf.eps_inv(psi_t, energies, inp.mu_idx, inp.miller, prob, omegas=[omega] if omega else None,
                     workspace=ws).eps_inv[0]
    return float((w_dev * e.T).sum().real.item())


def _fd_check(inp, prob, omega, samples, energies_idx, tol):
    w = synth.loss_weight(inp.ng)
    w_dev = dev(w)
    psi = dev(inp.psi_t)
    lval, ge, gp = isdf.eps_inv_grad(psi, inp.energies, inp.mu_idx, inp.miller, prob, w_dev, omega)
    ge, gp = ge.cpu().numpy(), gp.cpu().numpy()
    nbytes = isdf.workspace_bytes(prob, inp.nmu, inp.ng, 1 if omega else 0)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    h = 1e-5
    scale_e = np.abs(ge).max()
    for n in energies_idx:
        e1, e2 = inp.energies.copy(), inp.energies.copy()
        e1[n] += h
        e2[n] -= h
        fd = (_loss_gpu(inp, prob, psi, e1, w_dev, omega, ws) - _loss_gpu(inp, prob, psi, e2, w_dev, omega, ws)) / (2 * h)
        print(f"  d/d eps[{n}]: adjoint {ge[n]: .10e}  fd {fd: .10e}", flush=True)
        assert abs(fd - ge[n]) <= tol * scale_e, (n, fd, ge[n])
    scale_p = np.abs(gp).max()
    parts = ("re", "im") if inp.is_complex else ("re",)
    for n, m in samples:
        k = int(inp.mu_idx[m])
        for part in parts:
            p1, p2 = psi.clone(), psi.clone()
            step = h if part == "re" else 1j * h
            p1[n, k] += step
            p2[n, k] -= step
            fd = (_loss_gpu(inp, prob, p1, inp.energies, w_dev, omega, ws)
                  - _loss_gpu(inp, prob, p2, inp.energies, w_dev, omega, ws)) / (2 * h)
            g = gp[n, m].real if part == "re" else gp[n, m].imag
            print(f"  d/d{part} psi[{n}](r_{m}): adjoint {g: .10e}  fd {fd: .10e}", flush=True)
            assert abs(fd - g) <= tol * scale_p, (n, m, part, fd, g)
    return lval


@pytest.mark.parametrize("name,coulomb_sum", [("cfg0", 0), ("tiny", 1), ("wide", 1)])
def test_grad_matches_central_differences(name, coulomb_sum):
    """Backward against the derivative of this library's own FP64 forward (real
    orbitals in cfg0; the whole-grid Gram in tiny and wide, which the oracle gradient
    does not cover; wide's 33 x-frequencies take the plain adjoint y and x stages
    instead of the matrix-core ones).  Tolerance 1e-6 of the largest gradient entry:
    FD truncation O(h^2) and roundoff O(eps / h) stay below that at these sizes."""
    inp = synth.make_inputs(name)
    prob = isdf.problem_for(inp, "fp64", coulomb_sum=coulomb_sum)
    print(f"[grad-fd] case={name} coulomb_sum={coulomb_sum}", flush=True)
    _fd_check(inp, prob, 0.0, [(0, 0), (inp.nv, 3), (inp.nv + inp.nc - 1, inp.nmu - 1)], [0, inp.nv - 1, inp.nv],
              1e-6)


def test_autograd_function():
    """The torch.autograd.Function returns the adjoint's gradients for (energies, psi_mu)."""
    inp = synth.make_inputs("tiny")
    w = dev(synth.loss_weight(inp.ng))
    psi = dev(inp.psi_t)
    prob = isdf.problem_for(inp, "fp64")
    energies = torch.tensor(inp.energies, requires_grad=True)
    psi_mu = psi[:, torch.as_tensor(inp.mu_idx, device="cuda")].clone().requires_grad_(True)
    lval = isdf.eps_inv_loss(energies, psi_mu, psi, w, inp.mu_idx, inp.miller, prob, 0.0)
    lval.backward()
    l2, ge, gp = isdf.eps_inv_grad(psi, inp.energies, inp.mu_idx, inp.miller, prob, w, 0.0)
    assert lval.item() == l2
    assert torch.equal(energies.grad, ge.cpu())
    assert torch.equal(psi_mu.grad, gp)


def test_grad_full_size_64cubed():
    """The adjoint at the 64^3 solid-like size (256 / 1024 states, 2048 points,
    8192 plane waves): central differences of the FP64 forward on sampled
    energies and orbital samples (re and im parts)."""
    inp = synth.make_inputs("cfg2")
    prob = isdf.problem_for(inp, "fp64")
    print("[grad-fd] case=cfg2", flush=True)
    _fd_check(inp, prob, 0.0, [(0, 0), (inp.nv + 5, 100)], [0, inp.nv], 1e-5)


def test_grad_48cubed_chunks_and_mixed():
    """At 48^3 (640 points, Nr = 110592) the adjoint forms its N_mu x Nr intermediates in
    three chunks of points: central differences of the FP64 forward on sampled
    entries, and the mixed backward within 1e-4 (relative Frobenius) of the FP64 one
    (FP32 sums over 1e5 grid terms: sqrt(Nr) u ~ 2e-5)."""
    inp = synth.make_inputs("cfg1")
    prob = isdf.problem_for(inp, "fp64")
    print("[grad-fd] case=cfg1", flush=True)
    _fd_check(inp, prob, 0.0, [(0, 0), (inp.nv + 7, 300), (inp.nv + inp.nc - 1, inp.nmu - 1)], [0, inp.nv], 1e-6)
    w = dev(synth.loss_weight(inp.ng))
    psi = dev(inp.psi_t)
    _, ge64, gp64 = isdf.eps_inv_grad(psi, inp.energies, inp.mu_idx, inp.miller, prob, w, 0.0)
    _, ge32, gp32 = isdf.eps_inv_grad(psi, inp.energies, inp.mu_idx, inp.miller, isdf.problem_for(inp, "fp32"), w, 0.0)
    e_e = relf(ge32.cpu().numpy(), ge64.cpu().numpy())
    e_p = relf(gp32.cpu().numpy(), gp64.cpu().numpy())
    print(f"  mixed vs FP64 adjoint: d/d eps rel-F {e_e:.2e}  d/d psi(r_mu) rel-F {e_p:.2e}", flush=True)
    assert e_e <= 1e-4 and e_p <= 1e-4, (e_e, e_p)
