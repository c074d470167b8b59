"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Every comparison is element by element on the same seeded inputs (check_eps,
check_stage):
  eps~^{-1}: relative Frobenius error and largest entry error (|eps~^{-1}| <= 1)
      <= TOL_EPS, the stated targets (1e-10 for the FP64 path, 1e-6 for the
      mixed paths);
  the screening part eps~^{-1} - I, which is only ~2% of eps~^{-1} in norm on
      these inputs (so the first bar alone would dilute an error there ~50x):
      relative Frobenius error of eps~^{-1} - I, and the largest entry error
      relative to max |eps~^{-1} - I|, both <= TOL_SCREEN.  FP64: the stated
      1e-10.  FP32: 4e-6 (~64 u, u = 2^-24): the screening part is
      -X H^{-1} X^H from single-precision products over N_mu terms (measured
      4e-7 - 8e-7).  BF16x3: 2e-5: the pair products use operands split as
      hi + lo with 8 significant bits each, which represent a value to 2^-16
      relative (hi*lo and lo*hi kept, lo*lo dropped), so the fitted pair
      functions carry ~2^-16 relative error before any cancellation
      (measured 1e-6 - 3e-6);
  stage outputs (Theta, U, M): relative Frobenius error and the largest entry
      error relative to the largest entry, both <= TOL_STAGE: FP32 rounding
      (6e-8) times the conditioning of the least-squares fit (cond(C C^H) up to
      ~1e3 at these sizes); BF16x3 the split's 2^-16 times cond(S) <= 2e2.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_12340_amd as isdf
import synth

pytestmark = pytest.mark.gpu

SMALL = ["tiny", "cfg0", "mid", "mid_real", "fullrank", "tiles", "kmaj", "kmaj_even", "core32", "tail", "wide"]
TOL_EPS = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-6}
TOL_SCREEN = {"fp64": 1e-10, "fp32": 4e-6, "bf16x3": 2e-5}
# bf16x3 stages: effective unit roundoff ~3 * 2^-16 (hi + lo split, lo*lo dropped) times cond(S) <= 2e2 here
TOL_STAGE = {"fp64": 1e-10, "fp32": 1e-4, "bf16x3": 2e-3}
PRECS = ["fp64", "fp32", "bf16x3"]

_inputs = {}
_stages = {}


def get_inputs(name):
    if name not in _inputs:
        _inputs[name] = synth.make_inputs(name)
    return _inputs[name]


def get_stages(name):
    if name not in _stages:
        _stages[name] = oracle.isdf_stages(get_inputs(name))
    return _stages[name]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def relf(got, ref):
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


def eps_errors(got, ref, eye=None):
    """Errors of eps~^{-1} (or of a block of its rows, with the matching rows of I)."""
    if eye is None:
        eye = np.eye(ref.shape[0])
    d = got - ref
    scr = ref - eye
    return dict(rel_fro=float(np.linalg.norm(d) / np.linalg.norm(ref)), max_abs=float(np.abs(d).max()),
                rel_fro_screening=float(np.linalg.norm(d) / np.linalg.norm(scr)),
                max_rel_screening=float(np.abs(d).max() / np.abs(scr).max()))


def check_eps(got, ref, prec, eye=None, tag=""):
    e = eps_errors(got, ref, eye)
    print(f"  {tag}rel-F {e['rel_fro']:.3e}  max-abs {e['max_abs']:.3e}  rel-F(eps^-1 - I) "
          f"{e['rel_fro_screening']:.3e}  max-abs/max|eps^-1 - I| {e['max_rel_screening']:.3e}", flush=True)
    assert e["rel_fro"] <= TOL_EPS[prec], e
    assert e["max_abs"] <= TOL_EPS[prec], e
    assert e["rel_fro_screening"] <= TOL_SCREEN[prec], e
    assert e["max_rel_screening"] <= TOL_SCREEN[prec], e
    return e


def check_stage(got, ref, tol, tag=""):
    err = relf(got, ref)
    mx = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"  {tag}rel-F {err:.3e}  max-abs/max|ref| {mx:.3e}", flush=True)
    assert err <= tol, err
    assert mx <= tol, mx


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", SMALL)
def test_theta(name, prec):
    inp = get_inputs(name)
    print(f"[theta] case={name} prec={prec}", flush=True)
    got = isdf.fit_theta(dev(inp.psi_t), inp.mu_idx, isdf.problem_for(inp, prec)).cpu().numpy().T
    check_stage(got, get_stages(name)["theta"], TOL_STAGE[prec])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", SMALL)
def test_core(name, prec):
    inp = get_inputs(name)
    print(f"[core] case={name} prec={prec}", flush=True)
    got = isdf.core_m(dev(inp.psi_t), inp.energies, inp.mu_idx, isdf.problem_for(inp, prec)).cpu().numpy()
    check_stage(got, get_stages(name)["m"], TOL_STAGE[prec] * 1e-2)
    asym = float(np.abs(got - got.conj().T).max())
    assert asym == 0.0, asym  # lower computed, upper mirrored


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", SMALL)
def test_coulomb_u(name, prec):
    inp = get_inputs(name)
    print(f"[u] case={name} prec={prec}", flush=True)
    got = isdf.coulomb_u(dev(inp.psi_t), inp.mu_idx, inp.miller, isdf.problem_for(inp, prec)).cpu().numpy()
    check_stage(got, get_stages(name)["u"], TOL_STAGE[prec])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", SMALL)
def test_smw_apply(name, prec):
    """Step 4 alone from the oracle's U and M, against the dense-LU inverse."""
    inp = get_inputs(name)
    st = get_stages(name)
    print(f"[smw] case={name} prec={prec}", flush=True)
    res = isdf.smw_apply(dev(st["u"]), dev(st["m"]), isdf.problem_for(inp, prec))
    check_eps(res.eps_inv[0].cpu().numpy(), oracle.eps_inv_isdf(inp, stages=st), prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", SMALL)
def test_eps_inv(name, prec):
    inp = get_inputs(name)
    print(f"[eps_inv] case={name} prec={prec}", flush=True)
    res = isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller, isdf.problem_for(inp, prec))
    got = res.eps_inv[0].cpu().numpy()
    check_eps(got, oracle.eps_inv_isdf(inp, stages=get_stages(name)), prec)
    assert np.array_equal(got, got.conj().T), "not exactly Hermitian"
    e0 = np.zeros(inp.ng); e0[0] = 1.0
    assert np.array_equal(got[0], e0) and np.array_equal(got[:, 0], e0), "G = 0 row/column is not e0"  # V(0) = 0


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["tiny", "cfg0", "mid", "kmaj"])
def test_core_contour_integral(name, prec):
    """core_method 1 (Algorithm 2, 1e-13 quadrature tolerance) against the oracle's
    direct pair sum: the stage (FP64 <= 1e-11; single precision at the core's stage
    bar) and the whole build (the eps~^{-1} bars)."""
    inp = get_inputs(name)
    print(f"[cauchy] case={name} prec={prec}", flush=True)
    prob = isdf.problem_for(inp, prec, core_method=1)
    m = isdf.core_m(dev(inp.psi_t), inp.energies, inp.mu_idx, prob).cpu().numpy()
    ref = get_stages(name)["m"]
    err_m = relf(m, ref)
    got = isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller, prob).eps_inv[0].cpu().numpy()
    print(f"  core rel-F {err_m:.3e}", flush=True)
    assert err_m <= (1e-11 if prec == "fp64" else TOL_STAGE["fp32"] * 1e-2), err_m
    check_stage(m, ref, 1e-11 if prec == "fp64" else TOL_STAGE["fp32"] * 1e-2, "core ")
    assert np.array_equal(m, m.conj().T)
    check_eps(got, oracle.eps_inv_isdf(inp, stages=get_stages(name)), prec)


def test_core_contour_integral_unsupported():
    """The contour core is static and needs host energies: frequencies, plans and the
    adjoint refuse it."""
    inp = get_inputs("tiny")
    prob = isdf.problem_for(inp, "fp64", core_method=1)
    with pytest.raises(isdf.IsdfError) as e1:
        isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller, prob, omegas=[0.1])
    with pytest.raises(isdf.IsdfError) as e2:
        isdf.Plan(prob, inp.mu_idx, inp.miller)
    with pytest.raises(isdf.IsdfError) as e3:
        isdf.core_m(dev(inp.psi_t), inp.energies, inp.mu_idx, prob, omega=0.1)
    assert e1.value.status == e2.value.status == e3.value.status == isdf.binding.E_UNSUPPORTED


def test_fullrank_equals_exact_definition():
    """N_mu = Nv Nc: the GPU ISDF-SMW result equals chi0 from all pairs + dense LU."""
    inp = get_inputs("fullrank")
    res = isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller, isdf.problem_for(inp, "fp64"))
    check_eps(res.eps_inv[0].cpu().numpy(), oracle.eps_inv_exact(inp), "fp64")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["tiny", "cfg0", "fullrank", "wide"])
def test_eps_inv_whole_grid_gram(name, prec):
    """coulomb_sum = 1: the Gram X^H X runs over every grid vector (33^3 in 'wide',
    two DFT chunks per axis); the NG block equals the oracle's SMW with the
    whole-grid Gram."""
    inp = get_inputs(name)
    print(f"[whole-grid] case={name} prec={prec}", flush=True)
    res = isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller,
                       isdf.problem_for(inp, prec, coulomb_sum=1))
    got = res.eps_inv[0].cpu().numpy()
    check_eps(got, oracle.eps_inv_smw_full(inp, stages=get_stages(name)), prec)
    assert np.array_equal(got, got.conj().T)
    if name == "fullrank" and prec == "fp64":   # ISDF exact: chi0 from every pair, whole grid, dense LU
        check_eps(got, oracle.eps_inv_exact_full(inp), "fp64")


def test_plan_whole_grid_frequencies():
    """Plan path with coulomb_sum = 1 and a frequency batch: equals the direct call."""
    inp = synth.make_inputs("wide", n_omega=3)
    prob = isdf.problem_for(inp, "fp32", coulomb_sum=1)
    psi = dev(inp.psi_t)
    direct = isdf.eps_inv(psi, inp.energies, inp.mu_idx, inp.miller, prob, omegas=inp.omegas).eps_inv.cpu()
    plan = isdf.Plan(prob, inp.mu_idx, inp.miller, n_omega=3)
    out = plan.new_output()
    plan.eps_inv_async(psi, dev(inp.energies), out, plan.new_workspace(), omegas=inp.omegas)
    plan.sync()
    assert torch.equal(out.cpu(), direct)
    st = get_stages("wide")
    for k, om in enumerate(inp.omegas):
        stw = dict(st)
        stw["m"] = oracle.core_matrix(inp.psi_t, inp.energies, inp.nv, inp.mu_idx, omega=om)
        check_eps(direct[k].numpy(), oracle.eps_inv_smw_full(inp, stages=stw), "fp32", tag=f"w{k} ")


@pytest.mark.parametrize("prec,refine", [("fp64", 0), ("fp32", 0), ("fp32", 1)])
def test_frequencies(prec, refine):
    """Several imaginary frequencies in one call (the batched-frequency pipeline)."""
    inp = synth.make_inputs("mid", n_omega=4)
    print(f"[freq] prec={prec} refine={refine}", flush=True)
    res = isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller,
                       isdf.problem_for(inp, prec, refine_steps=refine), omegas=inp.omegas)
    got = res.eps_inv.cpu().numpy()
    st = get_stages("mid")
    for k, om in enumerate(inp.omegas):
        stw = dict(st)
        stw["m"] = oracle.core_matrix(inp.psi_t, inp.energies, inp.nv, inp.mu_idx, omega=om)
        check_eps(got[k], oracle.eps_inv_isdf(inp, stages=stw), prec, tag=f"w{k} ")
        assert np.array_equal(got[k], got[k].conj().T)


def test_refinement_reports_residual():
    inp = get_inputs("mid")
    prob = isdf.problem_for(inp, "fp32", refine_steps=2)
    res = isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller, prob)
    rep = res.report
    assert rep.n_refine_reported == 3
    r = [rep.refine_residual[k] for k in range(3)]
    assert all(np.isfinite(r)) and r[-1] < 1e-13
    check_eps(res.eps_inv[0].cpu().numpy(), oracle.eps_inv_isdf(inp, stages=get_stages("mid")), "fp32")


def test_deterministic():
    inp = get_inputs("mid")
    prob = isdf.problem_for(inp, "fp32")
    a = isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller, prob).eps_inv.cpu()
    b = isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller, prob).eps_inv.cpu()
    assert torch.equal(a, b)


def test_side_stream():
    inp = get_inputs("cfg0")
    prob = isdf.problem_for(inp, "fp64")
    psi = dev(inp.psi_t)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        res = isdf.eps_inv(psi, inp.energies, inp.mu_idx, inp.miller, prob)
    torch.cuda.synchronize()
    check_eps(res.eps_inv[0].cpu().numpy(), oracle.eps_inv_isdf(inp, stages=get_stages("cfg0")), "fp64")


def test_error_paths():
    inp = get_inputs("cfg0")
    prob = isdf.problem_for(inp, "fp64")
    psi = dev(inp.psi_t)
    bad_mu = inp.mu_idx.copy(); bad_mu[1] = bad_mu[0]
    with pytest.raises(isdf.IsdfError) as e:
        isdf.eps_inv(psi, inp.energies, bad_mu, inp.miller, prob)
    assert e.value.status == -1
    e2 = inp.energies.copy(); e2[0] = e2[-1] + 1.0
    with pytest.raises(isdf.IsdfError) as e:
        isdf.eps_inv(psi, e2, inp.mu_idx, inp.miller, prob)
    assert e.value.status == -1
    # every orbital vanishes at one interpolation point -> C has a zero row -> S singular
    psi0 = inp.psi_t.copy(); psi0[:, inp.mu_idx[5]] = 0.0
    with pytest.raises(isdf.IsdfError) as e:
        isdf.eps_inv(dev(psi0), inp.energies, inp.mu_idx, inp.miller, prob)
    assert e.value.status == -2
    # the library still works afterwards
    res = isdf.eps_inv(psi, inp.energies, inp.mu_idx, inp.miller, prob)
    check_eps(res.eps_inv[0].cpu().numpy(), oracle.eps_inv_isdf(inp, stages=get_stages("cfg0")), "fp64")


def _plan_case(name, prec, n_omega=0):
    inp = synth.make_inputs(name, n_omega=n_omega) if n_omega else get_inputs(name)
    prob = isdf.problem_for(inp, prec)
    plan = isdf.Plan(prob, inp.mu_idx, inp.miller, n_omega=n_omega)
    return inp, prob, plan


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plan_matches_direct(prec):
    """Enqueue-only plan calls (back to back on one workspace, one sync) give the
    direct call's result bit for bit."""
    inp, prob, plan = _plan_case("mid", prec)
    print(f"[plan] case=mid prec={prec}", flush=True)
    psi = dev(inp.psi_t)
    direct = isdf.eps_inv(psi, inp.energies, inp.mu_idx, inp.miller, prob).eps_inv.cpu()
    e = dev(inp.energies)
    ws = plan.new_workspace()
    outs = [plan.new_output() for _ in range(3)]
    for o in outs:
        plan.eps_inv_async(psi, e, o, ws)
    rep = plan.sync()
    assert rep.min_pivot > 0
    for o in outs:
        assert torch.equal(o.cpu(), direct)


def test_plan_stage_timing():
    """Stage timing on a plan: the timed calls give the same result, and sync returns
    positive mean stage intervals (then zeros once timing is off)."""
    inp, prob, plan = _plan_case("mid", "fp32")
    psi, e = dev(inp.psi_t), dev(inp.energies)
    ws, a, b = plan.new_workspace(), plan.new_output(), plan.new_output()
    plan.eps_inv_async(psi, e, a, ws)
    plan.sync()
    plan.time_stages(True)
    for _ in range(3):
        plan.eps_inv_async(psi, e, b, ws)
    rep = plan.sync()
    assert torch.equal(a, b)
    st = list(rep.stage_ms)
    assert all(x > 0 for x in st[:7]), st
    plan.time_stages(False)
    plan.eps_inv_async(psi, e, b, ws)
    assert all(x == 0 for x in plan.sync().stage_ms)


def test_plan_frequencies():
    inp, prob, plan = _plan_case("mid", "fp32", n_omega=4)
    psi = dev(inp.psi_t)
    direct = isdf.eps_inv(psi, inp.energies, inp.mu_idx, inp.miller, prob, omegas=inp.omegas).eps_inv.cpu()
    out = plan.new_output()
    plan.eps_inv_async(psi, dev(inp.energies), out, plan.new_workspace(), omegas=inp.omegas)
    plan.sync()
    assert torch.equal(out.cpu(), direct)


def test_plan_device_errors_surface_at_sync():
    inp, prob, plan = _plan_case("cfg0", "fp64")
    psi = dev(inp.psi_t)
    ws, out = plan.new_workspace(), plan.new_output()
    ref = oracle.eps_inv_isdf(inp, stages=get_stages("cfg0"))
    # energies without a gap: found by the device check, reported at sync
    e_bad = inp.energies.copy(); e_bad[0] = e_bad[-1] + 1.0
    plan.eps_inv_async(psi, dev(e_bad), out, ws)
    with pytest.raises(isdf.IsdfError) as err:
        plan.sync()
    assert err.value.status == -1
    # the status was cleared: a good call syncs cleanly and is correct
    plan.eps_inv_async(psi, dev(inp.energies), out, ws)
    plan.sync()
    check_eps(out[0].cpu().numpy(), ref, "fp64")
    # C rank deficient (all orbitals vanish at one point): not positive definite
    psi0 = inp.psi_t.copy(); psi0[:, inp.mu_idx[5]] = 0.0
    plan.eps_inv_async(dev(psi0), dev(inp.energies), out, ws)
    with pytest.raises(isdf.IsdfError) as err:
        plan.sync()
    assert err.value.status == -2
    # host-side argument errors are immediate
    with pytest.raises(ValueError):
        plan.eps_inv_async(psi, dev(inp.energies), out, ws, omegas=[0.1])


# The launch configurations the benchmark times: plan calls, and for the 64^3
# workload BF16x3 with two refinement steps of the FP64 core inverse.
BENCH_REFINE = {"cfg1": {"fp64": 0, "fp32": 0, "bf16x3": 0}, "cfg2": {"fp64": 0, "fp32": 0, "bf16x3": 2}}


@pytest.mark.parametrize("prec", PRECS)
def test_full_size_48cubed(prec):
    """The benchmark workload itself (48^3, 64/256 states, 640 points, 4096 plane
    waves), every element of eps~^{-1} against the oracle, in the launch
    configuration the benchmark times (plan, enqueue-only calls)."""
    name = "cfg1"
    inp = get_inputs(name)
    print(f"[full] case={name} prec={prec}", flush=True)
    prob = isdf.problem_for(inp, prec, refine_steps=BENCH_REFINE[name][prec])
    plan = isdf.Plan(prob, inp.mu_idx, inp.miller)
    out = plan.new_output()
    plan.eps_inv_async(dev(inp.psi_t), dev(inp.energies), out, plan.new_workspace())
    plan.sync()
    got = out[0].cpu().numpy()
    check_eps(got, oracle.eps_inv_isdf(inp, stages=get_stages(name)), prec)
    assert np.array_equal(got, got.conj().T)


_big = {}


def golden_64():
    """The stored oracle reference of the 64^3 workload (tests/golden/make_full_size.py),
    after confirming that the generator still produces the same inputs."""
    if not _big:
        import os
        z = np.load(os.path.join(os.path.dirname(__file__), "golden", "cfg2_oracle.npz"))
        inp = get_inputs("cfg2")
        assert np.array_equal(z["mu_idx"], inp.mu_idx), "interpolation points differ from the stored reference"
        assert np.abs(z["psi_fingerprint"] - inp.psi_t[:, :16]).max() <= 1e-12
        assert np.abs(z["energies"] - inp.energies).max() <= 1e-15
        _big["z"] = {k: z[k] for k in z.files}
        _big["inp"] = inp
        _big["psi"] = dev(inp.psi_t)
    return _big["inp"], _big["z"], _big["psi"]


@pytest.mark.parametrize("prec", PRECS)
def test_full_size_64cubed(prec):
    """The 64^3 solid-like workload (256 / 1024 states, 2048 points, 8192 plane
    waves) at full size in the plan launch configuration the benchmark times
    (BF16x3 with two refinement steps), against the stored oracle reference
    element by element: 16 rows of eps~^{-1} (its screening part included), 16
    grid rows of Theta, 16 plane-wave rows of U and 64 entries of the core M."""
    inp, z, psi = golden_64()
    print(f"[full64] prec={prec}", flush=True)
    prob = isdf.problem_for(inp, prec, refine_steps=BENCH_REFINE["cfg2"][prec])
    plan = isdf.Plan(prob, inp.mu_idx, inp.miller)
    out = plan.new_output()
    plan.eps_inv_async(psi, dev(inp.energies), out, plan.new_workspace())
    rep = plan.sync()
    rows = torch.as_tensor(z["rows"], device=out.device)
    got = out[0].index_select(0, rows).cpu().numpy()
    eye = np.eye(inp.ng)[z["rows"]]
    check_eps(got, z["eps_rows"], prec, eye=eye, tag="16 rows: ")
    assert torch.equal(out[0], out[0].conj().T)
    assert bool((out[0][0, 1:] == 0).all()) and out[0][0, 0].item() == 1.0
    if prob.refine_steps:
        res = [rep.refine_residual[k] for k in range(rep.n_refine_reported)]
        print(f"  refinement residuals {res}", flush=True)
        assert rep.n_refine_reported == 3 and res[-1] <= 1e-12
    del out
    pm = isdf.problem_for(inp, prec)
    m = isdf.core_m(psi, inp.energies, inp.mu_idx, pm)
    pairs = z["m_pairs"]
    check_stage(m.cpu().numpy()[pairs[:, 0], pairs[:, 1]], z["m_entries"], TOL_STAGE[prec] * 1e-2, "M entries: ")
    u = isdf.coulomb_u(psi, inp.mu_idx, inp.miller, pm)
    check_stage(u.index_select(0, torch.as_tensor(z["u_rows_idx"], device=u.device)).cpu().numpy(), z["u_rows"],
                TOL_STAGE[prec], "U rows: ")
    del u
    th = isdf.fit_theta(psi, inp.mu_idx, pm)       # (N_mu, Nr)
    got_th = th.index_select(1, torch.as_tensor(z["theta_rows_idx"], device=th.device)).cpu().numpy().T
    del th
    check_stage(got_th, z["theta_rows"], TOL_STAGE[prec], "Theta rows: ")


def test_batched_frequencies_and_systems():
    """The batched configuration the benchmark times: the 48^3 system and the eight
    uneven systems (24^3 ... 40^3, Nv 16 ... 48, Nc = 4 Nv, N_mu = 10 Nv, NG = 32 Nv),
    each with 32 imaginary frequencies log-spaced in [0.01, 100] eV, in one
    multi-system call (mixed path).  Every system's eps~^{-1} at every frequency
    (three of the 48^3 system's 32) against the oracle with that frequency's
    weights Delta / (Delta^2 + omega^2)."""
    names = ["cfg1"] + [f"batch{i}" for i in range(8)]
    n_omega = 32
    plans, psis, es, wss, outs, inps = [], [], [], [], [], []
    for name in names:
        inp = synth.make_inputs(name, n_omega=n_omega)
        plans.append(isdf.Plan(isdf.problem_for(inp, "fp32"), inp.mu_idx, inp.miller, n_omega=n_omega))
        psis.append(dev(inp.psi_t)); es.append(dev(inp.energies))
        wss.append(plans[-1].new_workspace()); outs.append(plans[-1].new_output())
        inps.append(inp)
    print("[batch] 9 systems x 32 frequencies", flush=True)
    isdf.eps_inv_multi(plans, psis, es, outs, wss, omegas=[i.omegas for i in inps])
    for p in plans:
        p.sync()
    for name, inp, out in zip(names, inps, outs):
        st = get_stages(name) if name == "cfg1" else oracle.isdf_stages(inp)
        ks = [0, 15, 31] if name == "cfg1" else range(n_omega)
        worst = {}
        for k in ks:
            stw = dict(st)
            stw["m"] = oracle.core_matrix(inp.psi_t, inp.energies, inp.nv, inp.mu_idx, omega=inp.omegas[k])
            ref = oracle.eps_inv_isdf(inp, stages=stw)
            e = eps_errors(out[k].cpu().numpy(), ref)
            for key, val in e.items():
                worst[key] = max(worst.get(key, 0.0), val)
            assert e["rel_fro"] <= TOL_EPS["fp32"] and e["max_abs"] <= TOL_EPS["fp32"], (name, k, e)
            assert e["rel_fro_screening"] <= TOL_SCREEN["fp32"], (name, k, e)
            assert e["max_rel_screening"] <= TOL_SCREEN["fp32"], (name, k, e)
        print(f"  {name}: worst over {len(ks)} frequencies {worst}", flush=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_core_contour_integral_64cubed(prec):
    """Algorithm 2 at the 64^3 size (Nv Nc = 262144 pairs, 2048 points): 64 sampled
    core entries against the oracle's direct pair sum."""
    inp = get_inputs("cfg2")
    print(f"[cauchy64] prec={prec}", flush=True)
    rng = np.random.default_rng(65)
    pairs = rng.integers(0, inp.nmu, size=(64, 2))
    pairs[:8, 1] = pairs[:8, 0]
    ref = oracle.core_entries(inp.psi_t, inp.energies, inp.nv, inp.mu_idx, pairs)
    m = isdf.core_m(dev(inp.psi_t), inp.energies, inp.mu_idx, isdf.problem_for(inp, prec, core_method=1))
    got = m.cpu().numpy()[pairs[:, 0], pairs[:, 1]]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  sampled max rel {err:.3e}", flush=True)
    assert err <= (1e-11 if prec == "fp64" else TOL_STAGE["fp32"] * 1e-2), err


@pytest.mark.parametrize("name,prec", [("kmaj", "fp32"), ("core32", "fp32"), ("core32", "bf16x3")])
def test_frequencies_full_tiles(name, prec):
    """Frequency batch on full-tile cases: k-major output products per frequency
    (kmaj), and the cores M(omega) of all frequencies in one launch of the k-major
    single-precision core (core32)."""
    inp = synth.make_inputs(name, n_omega=3)
    st = get_stages(name)
    print(f"[freq] case={name} prec={prec}", flush=True)
    res = isdf.eps_inv(dev(inp.psi_t), inp.energies, inp.mu_idx, inp.miller, isdf.problem_for(inp, prec),
                       omegas=inp.omegas)
    got = res.eps_inv.cpu().numpy()
    for k, om in enumerate(inp.omegas):
        stw = dict(st)
        stw["m"] = oracle.core_matrix(inp.psi_t, inp.energies, inp.nv, inp.mu_idx, omega=om)
        check_eps(got[k], oracle.eps_inv_isdf(inp, stages=stw), prec, tag=f"w{k} ")


def test_plan_graph_capture():
    """A plan call captured into a HIP graph (both library streams) replays to the
    eager result; eager calls and synchronisations run between the replays."""
    inp, prob, plan = _plan_case("kmaj", "fp32")
    print("[graph] case=kmaj prec=fp32", flush=True)
    psi, e = dev(inp.psi_t), dev(inp.energies)
    ws, out = plan.new_workspace(), plan.new_output()
    plan.eps_inv_async(psi, e, out, ws)
    plan.sync()
    ref = out.clone()
    graph_out = plan.new_output()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.eps_inv_async(psi, e, graph_out, ws)
    for _ in range(3):
        graph_out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(graph_out, ref)
        plan.eps_inv_async(psi, e, out, ws)
        plan.sync()
        assert torch.equal(out, ref)
    check_eps(ref[0].cpu().numpy(), oracle.eps_inv_isdf(inp, stages=get_stages("kmaj")), "fp32")


def _multi_case(private_streams):
    names = ["tiny", "mid", "kmaj"]
    plans, psis, es, wss, outs, refs = [], [], [], [], [], []
    for i, name in enumerate(names):
        inp = get_inputs(name)
        prob = isdf.problem_for(inp, "fp32")
        solo = isdf.Plan(prob, inp.mu_idx, inp.miller)
        psi, e = dev(inp.psi_t), dev(inp.energies)
        o = solo.new_output()
        solo.eps_inv_async(psi, e, o, solo.new_workspace())
        solo.sync()
        refs.append(o.clone())
        stream = torch.cuda.Stream() if (private_streams and i > 0) else None
        plans.append(isdf.Plan(prob, inp.mu_idx, inp.miller, stream=stream))
        psis.append(psi); es.append(e)
        wss.append(plans[-1].new_workspace()); outs.append(plans[-1].new_output())
    return plans, psis, es, wss, outs, refs


def test_multi_system_concurrent():
    """Systems of different sizes in one multi call, each on its own stream:
    every output equals its single-plan result."""
    print("[multi] concurrent", flush=True)
    plans, psis, es, wss, outs, refs = _multi_case(True)
    isdf.eps_inv_multi(plans, psis, es, outs, wss)
    for p in plans:
        p.sync()
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)


def test_multi_system_graph():
    """Systems of different sizes in one multi call on one stream, captured into one
    graph; replays (with eager calls in between) equal the single-plan results."""
    print("[multi] graph", flush=True)
    plans, psis, es, wss, outs, refs = _multi_case(False)
    isdf.eps_inv_multi(plans, psis, es, outs, wss)
    for p in plans:
        p.sync()
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        isdf.eps_inv_multi(plans, psis, es, outs, wss)
    for _ in range(2):
        for o in outs:
            o.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r)
        isdf.eps_inv_multi(plans, psis, es, outs, wss)
        for p in plans:
            p.sync()


@pytest.mark.skip(reason="capturing systems forked onto several streams (nested forks from a joined "
                         "stream) crashed the HIP runtime in stream-capture end once; the library now refuses "
                         "that form (ISDF_E_UNSUPPORTED) and concurrent systems in one graph go through "
                         "isdf_multi_graph_create")
def test_multi_system_concurrent_graph():
    plans, psis, es, wss, outs, refs = _multi_case(True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        isdf.eps_inv_multi(plans, psis, es, outs, wss)


def test_multi_graph_runs_systems_concurrently():
    """isdf_multi_graph_create: each system captured on its own plan's stream, the
    captured kernels and their dependencies copied into one graph with no
    dependencies between the systems.  Every replay (with eager calls and
    synchronisations in between) equals the single-plan results bit for bit."""
    print("[multi] merged-graph launch", flush=True)
    plans, psis, es, wss, outs, refs = [], [], [], [], [], []
    for name in ["tiny", "mid", "kmaj"]:
        inp = get_inputs(name)
        prob = isdf.problem_for(inp, "fp32")
        solo = isdf.Plan(prob, inp.mu_idx, inp.miller)
        psi, e = dev(inp.psi_t), dev(inp.energies)
        o = solo.new_output()
        solo.eps_inv_async(psi, e, o, solo.new_workspace())
        solo.sync()
        refs.append(o.clone())
        plans.append(isdf.Plan(prob, inp.mu_idx, inp.miller, stream=torch.cuda.Stream()))
        psis.append(psi); es.append(e)
        wss.append(plans[-1].new_workspace()); outs.append(plans[-1].new_output())
    g = isdf.MultiGraph(plans, psis, es, outs, wss)
    torch.cuda.synchronize()
    for _ in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.launch()
        for p in plans:
            p.sync()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r)
        isdf.eps_inv_multi(plans, psis, es, outs, wss)   # eager, concurrent streams
        for p in plans:
            p.sync()
    with pytest.raises(isdf.IsdfError) as err:          # one workspace for two concurrent systems
        isdf.MultiGraph(plans[:2], psis[:2], es[:2], outs[:2], [wss[1], wss[1]])
    assert err.value.status == isdf.binding.E_ARG


def test_multi_under_capture_with_forks_is_refused():
    """isdf_plan_eps_inv_multi with plans on several streams inside a stream capture
    returns ISDF_E_UNSUPPORTED before enqueueing anything."""
    plans, psis, es, wss, outs, refs = _multi_case(True)
    x = torch.zeros(4, device="cuda")
    g = torch.cuda.CUDAGraph()
    with pytest.raises(isdf.IsdfError) as err:
        with torch.cuda.graph(g):
            x.add_(1.0)
            isdf.eps_inv_multi(plans, psis, es, outs, wss)
    assert err.value.status == isdf.binding.E_UNSUPPORTED
    torch.cuda.synchronize()
    isdf.eps_inv_multi(plans, psis, es, outs, wss)       # eagerly the same call runs
    for p in plans:
        p.sync()
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)


def test_plan_autotune():
    """The autotuner picks knobs from its candidate lists; the tuned plan still
    meets the parity bar, and out-of-range knobs are rejected."""
    inp, prob, plan = _plan_case("kmaj", "fp32")
    print("[autotune] case=kmaj", flush=True)
    psi, e = dev(inp.psi_t), dev(inp.energies)
    ws, out = plan.new_workspace(), plan.new_output()
    t = plan.autotune(psi, e, out, ws, reps=2)
    assert t["dft_zb"] in (4, 6, 8, 12, 16, 24) and t["core_split_pct"] in (50, 100, 200)
    assert t["gram_split"] in (4, 8, 16) and t["wg_per_cu"] in (1, 2) and t["best_ms"] > 0
    assert t["core_stream"] in (0, 1, 2) and t["side_prio"] in (0, 1) and t["dft_pipe"] in (0, 1)
    assert plan.get_tune()["dft_zb"] == t["dft_zb"]
    plan.eps_inv_async(psi, e, out, ws)
    plan.sync()
    check_eps(out[0].cpu().numpy(), oracle.eps_inv_isdf(inp, stages=get_stages("kmaj")), "fp32")
    for knobs in ({"dft_zb": 2, "core_split_pct": 200, "gram_split": 4, "wg_per_cu": 2},
                  {"dft_zb": 16, "core_split_pct": 50, "gram_split": 1, "wg_per_cu": 1}):
        plan.set_tune(**knobs)
        plan.eps_inv_async(psi, e, out, ws)
        plan.sync()
        check_eps(out[0].cpu().numpy(), oracle.eps_inv_isdf(inp, stages=get_stages("kmaj")), "fp32")
    with pytest.raises(isdf.IsdfError):
        plan.set_tune(dft_zb=0)
    with pytest.raises(isdf.IsdfError):
        plan.set_tune(core_stream=3)
    with pytest.raises(isdf.IsdfError):
        plan.set_tune(side_prio=2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_core_stream_placement_is_bit_identical(prec):
    """The first core on the second stream after Z (core_stream 1) or beside it (2),
    and the second stream's sweep at normal wave priority (side_prio 0), run the same
    kernels on the same data: the result equals the default placement bit for bit."""
    inp, prob, plan = _plan_case("mid", prec)
    psi, e = dev(inp.psi_t), dev(inp.energies)
    ws = plan.new_workspace()
    outs = []
    for cs, sp in ((0, 1), (1, 1), (2, 1), (0, 0), (2, 0)):
        outs.append(plan.new_output())
        plan.set_tune(core_stream=cs, side_prio=sp)
        plan.eps_inv_async(psi, e, outs[-1], ws)
        plan.sync()
    assert all(torch.equal(outs[0], o) for o in outs[1:])


@pytest.mark.parametrize("name", ["tiny", "cfg0", "mid", "tiles", "kmaj_even", "wide", "sig_even", "pipe3"])
def test_dft_pipe_and_single_role_pass_agree(name):
    """The warp-specialised DFT (dft_pipe 1, the default) and the single-role pass
    (dft_pipe 0) each meet the FP32 bars against the oracle, and agree with each
    other to FP32 rounding (their z sums are split into pieces differently).  tiny and
    cfg0 (at most 8 x-frequencies) and pipe3 (17 or more) spread the matrix-core waves
    unevenly over the SIMDs, so only some z-waves sum; the others spread them evenly."""
    inp, prob, plan = _plan_case(name, "fp32")
    print(f"[dft_pipe] case={name}", flush=True)
    psi, e = dev(inp.psi_t), dev(inp.energies)
    ws = plan.new_workspace()
    ref = oracle.eps_inv_isdf(inp, stages=get_stages(name))
    outs = []
    for pipe in (1, 0):
        outs.append(plan.new_output())
        plan.set_tune(dft_pipe=pipe)
        plan.eps_inv_async(psi, e, outs[-1], ws)
        plan.sync()
        check_eps(outs[-1][0].cpu().numpy(), ref, "fp32", tag=f"pipe={pipe} ")
    a, b = outs[0][0].cpu().numpy(), outs[1][0].cpu().numpy()
    assert np.abs(a - b).max() <= 1e-6 * max(1.0, np.abs(b).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_condition_estimate(prec):
    """cond_est = ||H||_F ||H^-1||_F brackets the 2-norm condition number of the
    core H = U^H U - M^-1 (here formed by the oracle) from above, within a factor n."""
    inp = get_inputs("mid")
    st = get_stages("mid")
    res = isdf.smw_apply(dev(st["u"]), dev(st["m"]), isdf.problem_for(inp, prec))
    h = st["u"].conj().T @ st["u"] - np.linalg.inv(st["m"])
    k2 = np.linalg.cond(h)
    ce = res.report.cond_est
    print(f"  cond2 {k2:.4e}  cond_est {ce:.4e}", flush=True)
    assert np.isfinite(ce) and k2 * (1 - 1e-6) <= ce <= inp.nmu * k2
