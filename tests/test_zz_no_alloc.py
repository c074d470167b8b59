"""The allocation-free entry point isdf_eps_inv_noalloc (library-owned per-GPU
scratch array as the workspace) against isdf_eps_inv with a caller workspace and
against the FP64 oracle, on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_12340_amd as isdf
import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-6}
_inputs = {}


def get_inputs(name):
    if name not in _inputs:
        _inputs[name] = synth.make_inputs(name)
    return _inputs[name]


def _check(name, prec, noalloc_out):
    inp = get_inputs(name)
    prob = isdf.problem_for(inp, prec)
    psi = torch.from_numpy(inp.psi_t).to("cuda:0")
    print(f"[noalloc] {name} {prec}: allocation-free call", flush=True)
    got = isdf.eps_inv_noalloc(psi, inp.energies, inp.mu_idx, inp.miller, prob, out=noalloc_out).eps_inv
    torch.cuda.synchronize()
    got = got[0].cpu().numpy()
    print(f"[noalloc] {name} {prec}: workspace call", flush=True)
    ref = isdf.eps_inv(psi, inp.energies, inp.mu_idx, inp.miller, prob).eps_inv[0].cpu().numpy()
    # the same kernels on the same inputs: equal to the workspace entry point's result
    assert np.array_equal(got, ref), f"{name} {prec}: differs from isdf_eps_inv by {np.abs(got - ref).max()}"
    orc = oracle.eps_inv_isdf(inp)
    d = orc - np.eye(inp.ng)
    err = np.abs(got - orc).max() / np.abs(d).max()
    rel_scr = np.linalg.norm(got - orc) / np.linalg.norm(d)
    print(f"[noalloc] {name} {prec}: max-abs / max|eps~^-1 - I| = {err:.2e}, rel-F(eps~^-1 - I) = {rel_scr:.2e}",
          flush=True)
    assert err <= TOL[prec] and rel_scr <= TOL[prec]


@pytest.mark.parametrize("prec,first,second", [("fp64", "mid", "tiny"), ("fp32", "kmaj", "cfg0")])
def test_noalloc_matches_workspace_entry(prec, first, second):
    for name in (first, second):
        inp = get_inputs(name)
        need = isdf.workspace_bytes(isdf.problem_for(inp, prec), inp.nmu, inp.ng, 0)
        assert need <= isdf.binding.SCRATCH_MAX_BYTES
        out = torch.full((1, inp.ng, inp.ng), float("nan"), dtype=torch.complex128, device="cuda:0")
        _check(name, prec, out)


def test_noalloc_rejects_large_problem():
    """A problem whose workspace exceeds the scratch array is refused on the host
    (nothing enqueued) with ISDF_E_WORKSPACE and a message naming the limit."""
    inp = get_inputs("kmaj")
    prob = isdf.problem_for(inp, "fp64")
    assert isdf.workspace_bytes(prob, inp.nmu, inp.ng, 0) > isdf.binding.SCRATCH_MAX_BYTES
    psi = torch.from_numpy(inp.psi_t).to("cuda:0")
    out = torch.zeros((1, inp.ng, inp.ng), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(isdf.IsdfError) as err:
        isdf.eps_inv_noalloc(psi, inp.energies, inp.mu_idx, inp.miller, prob, out=out)
    assert err.value.status == isdf.binding.E_WORKSPACE
    assert "at most" in str(err.value)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
