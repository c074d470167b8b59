"""ctypes binding of libisdfsmw.so (C ABI in include/isdf_smw.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (inputs, outputs, workspace) and the
HIP stream.  There is no fallback: if the library is not built, or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libisdfsmw.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "isdf_smw.h")

OK, E_ARG, E_NOT_PD, E_DEVICE, E_WORKSPACE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "ISDF_OK", -1: "ISDF_E_ARG", -2: "ISDF_E_NOT_PD", -3: "ISDF_E_DEVICE",
                -4: "ISDF_E_WORKSPACE", -5: "ISDF_E_UNSUPPORTED"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}


class IsdfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("cell", ctypes.c_double * 9), ("nv", ctypes.c_int32),
                ("nc", ctypes.c_int32), ("is_complex", ctypes.c_int32), ("pair_factor", ctypes.c_double),
                ("v_scale", ctypes.c_double), ("prec", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("coulomb_sum", ctypes.c_int32), ("core_method", ctypes.c_int32), ("core_tol", ctypes.c_double)]


class Tune(ctypes.Structure):
    _fields_ = [("dft_zb", ctypes.c_int32), ("core_split_pct", ctypes.c_int32), ("gram_split", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("core_stream", ctypes.c_int32), ("side_prio", ctypes.c_int32),
                ("dft_pipe", ctypes.c_int32), ("best_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Report(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_double * 8), ("refine_residual", ctypes.c_double * 9),
                ("min_pivot", ctypes.c_double), ("want_timing", ctypes.c_int32),
                ("n_refine_reported", ctypes.c_int32), ("cond_est", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_2403_12340_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        pi32, pdbl, pprob = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(Problem)
        prep = ctypes.POINTER(Report)
        sig = {
            "isdf_create": [ctypes.POINTER(vp), ctypes.c_int, vp],
            "isdf_destroy": [vp],
            "isdf_set_stream": [vp, vp],
            "isdf_workspace_bytes": [pprob, i32, i32, i32, ctypes.POINTER(sz)],
            "isdf_gvectors": [pprob, i32, pi32],
            "isdf_check_inputs": [pprob, pdbl, pi32, i32, pi32, i32, pdbl, i32, ctypes.c_char_p, sz],
            "isdf_eps_inv": [vp, pprob, vp, pdbl, pi32, i32, pi32, i32, pdbl, i32, vp, sz, vp, prep],
            "isdf_eps_inv_noalloc": [vp, pprob, vp, pdbl, pi32, i32, pi32, i32, pdbl, i32, vp, prep],
            "isdf_sigma_workspace_bytes": [pprob, i32, i32, i32, i32, ctypes.POINTER(sz)],
            "isdf_sigma_cohsex": [vp, pprob, vp, pdbl, pi32, i32, pi32, i32, pi32, i32, pi32, i32, vp, sz, vp, vp,
                                  prep],
            "isdf_fit_theta": [vp, pprob, vp, pi32, i32, vp, sz, vp],
            "isdf_core_m": [vp, pprob, vp, pdbl, pi32, i32, dbl, vp, sz, vp],
            "isdf_coulomb_u": [vp, pprob, vp, pi32, i32, pi32, i32, vp, sz, vp],
            "isdf_smw_apply": [vp, pprob, vp, vp, i32, i32, vp, sz, vp, prep],
            "isdf_grad_workspace_bytes": [pprob, i32, i32, ctypes.POINTER(sz)],
            "isdf_contour_nodes": [pdbl, i32, i32, dbl, pdbl, ctypes.POINTER(i32)],
            "isdf_eps_inv_grad": [vp, pprob, vp, pdbl, pi32, i32, pi32, i32, dbl, vp, vp, sz, vp, vp, pdbl],
            "isdf_plan_table_bytes": [pprob, pi32, i32, pi32, i32, i32, ctypes.POINTER(sz)],
            "isdf_plan_create": [vp, pprob, pi32, i32, pi32, i32, i32, vp, sz, ctypes.POINTER(vp)],
            "isdf_plan_destroy": [vp],
            "isdf_plan_workspace_bytes": [vp, ctypes.POINTER(sz)],
            "isdf_plan_eps_inv": [vp, vp, vp, pdbl, vp, sz, vp],
            "isdf_plan_sync": [vp, prep],
            "isdf_plan_time_stages": [vp, i32],
            "isdf_plan_set_tune": [vp, ctypes.POINTER(Tune)],
            "isdf_plan_get_tune": [vp, ctypes.POINTER(Tune)],
            "isdf_plan_autotune": [vp, vp, vp, pdbl, vp, sz, vp, i32, ctypes.POINTER(Tune)],
            "isdf_plan_eps_inv_multi": [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(sz), ctypes.POINTER(vp)],
            "isdf_multi_graph_create": [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(sz), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp)],
            "isdf_graph_launch": [vp, vp],
            "isdf_graph_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.isdf_last_error.argtypes = [vp]
        L.isdf_last_error.restype = ctypes.c_char_p
        L.isdf_version.argtypes = []
        L.isdf_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions the C header declares."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:isdf_status|const char\*)\s+(isdf_\w+)\s*\(", txt, re.M)))


def make_problem(n, cell, nv, nc, *, is_complex=True, pair_factor=2.0, v_scale=None,
                 prec="fp64", refine_steps=0, coulomb_sum=0, core_method=0, core_tol=0.0) -> Problem:
    p = Problem()
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    for d in range(3):
        p.n[d] = int(n[d])
    cell = np.asarray(cell, dtype=np.float64).reshape(3, 3)
    for i in range(9):
        p.cell[i] = float(cell.ravel()[i])
    p.nv, p.nc = int(nv), int(nc)
    p.is_complex = 1 if is_complex else 0
    p.pair_factor = float(pair_factor)
    if v_scale is None:
        v_scale = n[0] * n[1] * n[2] / abs(np.linalg.det(cell))
    p.v_scale = float(v_scale)
    p.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    p.refine_steps = int(refine_steps)
    p.coulomb_sum = int(coulomb_sum)
    p.core_method = int(core_method)
    p.core_tol = float(core_tol)
    return p


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def workspace_bytes(prob: Problem, n_mu: int, ng: int, n_omega: int = 0) -> int:
    out = ctypes.c_size_t(0)
    st = lib().isdf_workspace_bytes(ctypes.byref(prob), n_mu, ng, n_omega, ctypes.byref(out))
    if st != OK:
        raise IsdfError(st, "isdf_workspace_bytes rejected the problem")
    return int(out.value)


def gvectors(prob: Problem, ng: int) -> np.ndarray:
    out = np.zeros((ng, 3), dtype=np.int32)
    st = lib().isdf_gvectors(ctypes.byref(prob), ng, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if st != OK:
        raise IsdfError(st, "isdf_gvectors failed")
    return out


def check_inputs(prob: Problem, energies, mu_idx, miller, omegas=None) -> tuple[int, str]:
    e, pe = _f64(energies)
    mu, pmu = _i32(mu_idx)
    mi, pmi = _i32(miller)
    om = np.zeros(0) if omegas is None else np.asarray(omegas, dtype=np.float64)
    om, pom = _f64(om)
    buf = ctypes.create_string_buffer(512)
    st = lib().isdf_check_inputs(ctypes.byref(prob), pe, pmu, len(mu), pmi, len(mi), pom if len(om) else None,
                                 len(om), buf, 512)
    return st, buf.value.decode()


class Handle:
    """Library handle bound to one device.  Without a fixed stream it follows
    torch's current stream (refreshed on every call); with one (a torch stream)
    it stays bound to it."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        self.stream = stream
        cur = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        st = lib().isdf_create(ctypes.byref(h), device, ctypes.c_void_p(cur.cuda_stream))
        if st != OK:
            raise IsdfError(st, "isdf_create failed (no GPU?)")
        self.h = h

    def sync_stream(self):
        import torch
        if self.stream is None:
            lib().isdf_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def check(self, st: int, what: str):
        if st != OK:
            raise IsdfError(st, f"{what}: {lib().isdf_last_error(self.h).decode()}")

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().isdf_destroy(self.h)
        except Exception:
            pass


_handles: dict[int, Handle] = {}


def handle(device: int = 0) -> Handle:
    if device not in _handles:
        _handles[device] = Handle(device)
    h = _handles[device]
    h.sync_stream()
    return h


def _workspace(nbytes: int, device, ws=None):
    import torch
    if ws is not None and ws.numel() >= nbytes + 256:
        buf = ws
    else:
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


@dataclass
class Result:
    eps_inv: "object"      # torch complex128 (n_omega or 1, ng, ng)
    report: Report


def _check_psi(psi_t, prob):
    import torch
    if not isinstance(psi_t, torch.Tensor) or psi_t.device.type != "cuda":
        raise TypeError("psi_t must be a CUDA (HIP) torch tensor")
    nr = prob.n[0] * prob.n[1] * prob.n[2]
    if tuple(psi_t.shape) != (prob.nv + prob.nc, nr) or not psi_t.is_contiguous():
        raise ValueError(f"psi_t must be contiguous with shape (N, Nr) = ({prob.nv + prob.nc}, {nr})")
    want = torch.complex128 if prob.is_complex else torch.float64
    if psi_t.dtype != want:
        raise TypeError(f"psi_t dtype must be {want}")


def eps_inv(psi_t, energies, mu_idx, miller, prob: Problem, omegas=None, *, out=None, workspace=None,
            timing=False) -> Result:
    """eps~^{-1} on the plane-wave list (one matrix per frequency; static if omegas is None)."""
    import torch
    _check_psi(psi_t, prob)
    dev = psi_t.device
    h = handle(dev.index or 0)
    e, pe = _f64(energies)
    mu, pmu = _i32(mu_idx)
    mi, pmi = _i32(miller)
    om = np.zeros(0) if omegas is None else np.asarray(omegas, dtype=np.float64)
    om, pom = _f64(om)
    nw = max(len(om), 1)
    ng = len(mi)
    nbytes = workspace_bytes(prob, len(mu), ng, len(om))
    wsbuf, wsptr = _workspace(nbytes, dev, workspace)
    if out is None:
        out = torch.empty((nw, ng, ng), dtype=torch.complex128, device=dev)
    rep = Report()
    rep.want_timing = 1 if timing else 0
    st = lib().isdf_eps_inv(h.h, ctypes.byref(prob), ctypes.c_void_p(psi_t.data_ptr()), pe, pmu, len(mu), pmi, ng,
                            pom if len(om) else None, len(om), ctypes.c_void_p(wsptr), nbytes,
                            ctypes.c_void_p(out.data_ptr()), ctypes.byref(rep))
    h.check(st, "isdf_eps_inv")
    return Result(out, rep)


SCRATCH_MAX_BYTES = 64 << 20   # ISDF_SCRATCH_MAX_BYTES


def eps_inv_noalloc(psi_t, energies, mu_idx, miller, prob: Problem, omegas=None, *, out) -> Result:
    """isdf_eps_inv_noalloc: eps~^{-1} with the library's per-GPU scratch array as the
    workspace (problems up to SCRATCH_MAX_BYTES of workspace).  `out` is caller-owned
    (max(n_omega, 1), ng, ng) complex128; nothing is allocated on the device."""
    import torch
    _check_psi(psi_t, prob)
    dev = psi_t.device
    h = handle(dev.index or 0)
    e, pe = _f64(energies)
    mu, pmu = _i32(mu_idx)
    mi, pmi = _i32(miller)
    om = np.zeros(0) if omegas is None else np.asarray(omegas, dtype=np.float64)
    om, pom = _f64(om)
    ng = len(mi)
    if (out.dtype != torch.complex128 or tuple(out.shape) != (max(len(om), 1), ng, ng) or not out.is_contiguous()
            or out.device != dev):
        raise ValueError("out must be contiguous complex128 (max(n_omega, 1), ng, ng) on psi's device")
    rep = Report()
    st = lib().isdf_eps_inv_noalloc(h.h, ctypes.byref(prob), ctypes.c_void_p(psi_t.data_ptr()), pe, pmu, len(mu),
                                    pmi, ng, pom if len(om) else None, len(om), ctypes.c_void_p(out.data_ptr()),
                                    ctypes.byref(rep))
    h.check(st, "isdf_eps_inv_noalloc")
    return Result(out, rep)


def sigma_workspace_bytes(prob: Problem, n_mu: int, ng: int, n_mu_vn: int, n_mu_nn: int) -> int:
    out = ctypes.c_size_t(0)
    st = lib().isdf_sigma_workspace_bytes(ctypes.byref(prob), n_mu, ng, n_mu_vn, n_mu_nn, ctypes.byref(out))
    if st != OK:
        raise IsdfError(st, "isdf_sigma_workspace_bytes rejected the arguments")
    return int(out.value)


@dataclass
class SigmaResult:
    sigma: "object"        # torch float64 (3, N): Sigma_SEX_X, Sigma_X, Sigma_COH
    eps_inv: "object"      # torch complex128 (1, ng, ng), the static eps~^{-1} built on the way
    report: Report


def sigma_cohsex(psi_t, energies, mu_idx, mu_vn, mu_nn, miller, prob: Problem, workspace=None) -> SigmaResult:
    """isdf_sigma_cohsex: the static COHSEX self-energy diagonals of every band."""
    import torch
    _check_psi(psi_t, prob)
    dev = psi_t.device
    h = handle(dev.index or 0)
    e, pe = _f64(energies)
    mu, pmu = _i32(mu_idx)
    mvn, pvn = _i32(mu_vn)
    mnn, pnn = _i32(mu_nn)
    mi, pmi = _i32(miller)
    ng = len(mi)
    nbytes = sigma_workspace_bytes(prob, len(mu), ng, len(mvn), len(mnn))
    wsbuf, wsptr = _workspace(nbytes, dev, workspace)
    out = torch.empty((1, ng, ng), dtype=torch.complex128, device=dev)
    sig = torch.empty((3, prob.nv + prob.nc), dtype=torch.float64, device=dev)
    rep = Report()
    st = lib().isdf_sigma_cohsex(h.h, ctypes.byref(prob), ctypes.c_void_p(psi_t.data_ptr()), pe, pmu, len(mu),
                                 pvn, len(mvn), pnn, len(mnn), pmi, ng, ctypes.c_void_p(wsptr), nbytes,
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(sig.data_ptr()), ctypes.byref(rep))
    h.check(st, "isdf_sigma_cohsex")
    return SigmaResult(sig, out, rep)


def fit_theta(psi_t, mu_idx, prob: Problem, workspace=None):
    """Theta in real space, returned as (N_mu, Nr) complex128: theta[mu, k] = Theta(r_k, mu)."""
    import torch
    _check_psi(psi_t, prob)
    dev = psi_t.device
    h = handle(dev.index or 0)
    mu, pmu = _i32(mu_idx)
    nr = prob.n[0] * prob.n[1] * prob.n[2]
    nbytes = workspace_bytes(prob, len(mu), 1, 0)
    wsbuf, wsptr = _workspace(nbytes, dev, workspace)
    out = torch.empty((len(mu), nr), dtype=torch.complex128, device=dev)
    st = lib().isdf_fit_theta(h.h, ctypes.byref(prob), ctypes.c_void_p(psi_t.data_ptr()), pmu, len(mu),
                              ctypes.c_void_p(wsptr), nbytes, ctypes.c_void_p(out.data_ptr()))
    h.check(st, "isdf_fit_theta")
    return out


def core_m(psi_t, energies, mu_idx, prob: Problem, omega=0.0, workspace=None):
    """Core f C W C^H as (N_mu, N_mu) complex128."""
    import torch
    _check_psi(psi_t, prob)
    dev = psi_t.device
    h = handle(dev.index or 0)
    e, pe = _f64(energies)
    mu, pmu = _i32(mu_idx)
    nbytes = workspace_bytes(prob, len(mu), 1, 0)
    wsbuf, wsptr = _workspace(nbytes, dev, workspace)
    out = torch.empty((len(mu), len(mu)), dtype=torch.complex128, device=dev)
    st = lib().isdf_core_m(h.h, ctypes.byref(prob), ctypes.c_void_p(psi_t.data_ptr()), pe, pmu, len(mu),
                           float(omega), ctypes.c_void_p(wsptr), nbytes, ctypes.c_void_p(out.data_ptr()))
    h.check(st, "isdf_core_m")
    return out


def coulomb_u(psi_t, mu_idx, miller, prob: Problem, workspace=None):
    """U = V^{1/2} F Theta on the plane-wave list as (NG, N_mu) complex128."""
    import torch
    _check_psi(psi_t, prob)
    dev = psi_t.device
    h = handle(dev.index or 0)
    mu, pmu = _i32(mu_idx)
    mi, pmi = _i32(miller)
    nbytes = workspace_bytes(prob, len(mu), len(mi), 0)
    wsbuf, wsptr = _workspace(nbytes, dev, workspace)
    out = torch.empty((len(mi), len(mu)), dtype=torch.complex128, device=dev)
    st = lib().isdf_coulomb_u(h.h, ctypes.byref(prob), ctypes.c_void_p(psi_t.data_ptr()), pmu, len(mu), pmi,
                              len(mi), ctypes.c_void_p(wsptr), nbytes, ctypes.c_void_p(out.data_ptr()))
    h.check(st, "isdf_coulomb_u")
    return out


def smw_apply(u, m, prob: Problem, workspace=None, timing=False) -> Result:
    """eps~^{-1} = I + U (M^{-1} - U^H U)^{-1} U^H from device U (NG, N_mu) and M (N_mu, N_mu)."""
    import torch
    ng, nmu = u.shape
    if u.dtype != torch.complex128 or m.dtype != torch.complex128 or tuple(m.shape) != (nmu, nmu):
        raise ValueError("u must be (NG, N_mu) and m (N_mu, N_mu), both complex128")
    u, m = u.contiguous(), m.contiguous()
    dev = u.device
    h = handle(dev.index or 0)
    nbytes = workspace_bytes(prob, nmu, ng, 0)
    wsbuf, wsptr = _workspace(nbytes, dev, workspace)
    out = torch.empty((1, ng, ng), dtype=torch.complex128, device=dev)
    rep = Report()
    rep.want_timing = 1 if timing else 0
    st = lib().isdf_smw_apply(h.h, ctypes.byref(prob), ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                              nmu, ng, ctypes.c_void_p(wsptr), nbytes, ctypes.c_void_p(out.data_ptr()),
                              ctypes.byref(rep))
    h.check(st, "isdf_smw_apply")
    return Result(out, rep)


def contour_nodes(energies, nv: int, nc: int, tol: float = 1e-13):
    """isdf_contour_nodes: (lambda (n,), weights (n,)) of the core's contour rule (host only)."""
    e, pe = _f64(energies)
    out = np.zeros(4 * 256)
    n = ctypes.c_int32(0)
    st = lib().isdf_contour_nodes(pe, nv, nc, float(tol), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(n))
    if st != OK:
        raise IsdfError(st, "isdf_contour_nodes rejected the energies")
    k = n.value
    z = out[:2 * k].view(np.complex128)
    w = out[2 * k:4 * k].view(np.complex128)
    return z.copy(), w.copy()


def grad_workspace_bytes(prob: Problem, n_mu: int, ng: int) -> int:
    out = ctypes.c_size_t(0)
    st = lib().isdf_grad_workspace_bytes(ctypes.byref(prob), n_mu, ng, ctypes.byref(out))
    if st != OK:
        raise IsdfError(st, "isdf_grad_workspace_bytes rejected the problem")
    return int(out.value)


def eps_inv_grad(psi_t, energies, mu_idx, miller, prob: Problem, w, omega=0.0, workspace=None):
    """isdf_eps_inv_grad: (L, dL/d energies (N,), dL/d psi at the points (N, N_mu) complex128)
    for L = Re tr(W eps~^{-1}); W is a device (NG, NG) complex128 Hermitian tensor."""
    import torch
    _check_psi(psi_t, prob)
    dev = psi_t.device
    h = handle(dev.index or 0)
    e, pe = _f64(energies)
    mu, pmu = _i32(mu_idx)
    mi, pmi = _i32(miller)
    ng, nmu = len(mi), len(mu)
    if w.dtype != torch.complex128 or tuple(w.shape) != (ng, ng) or w.device != dev:
        raise ValueError("w must be a (NG, NG) complex128 tensor on the orbitals' device")
    w = w.contiguous()
    nbytes = grad_workspace_bytes(prob, nmu, ng)
    wsbuf, wsptr = _workspace(nbytes, dev, workspace)
    ge = torch.empty(prob.nv + prob.nc, dtype=torch.float64, device=dev)
    gp = torch.empty((prob.nv + prob.nc, nmu), dtype=torch.complex128, device=dev)
    loss = ctypes.c_double(0.0)
    st = lib().isdf_eps_inv_grad(h.h, ctypes.byref(prob), ctypes.c_void_p(psi_t.data_ptr()), pe, pmu, nmu, pmi, ng,
                                 float(omega), ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(wsptr), nbytes,
                                 ctypes.c_void_p(ge.data_ptr()), ctypes.c_void_p(gp.data_ptr()), ctypes.byref(loss))
    h.check(st, "isdf_eps_inv_grad")
    return float(loss.value), ge, gp


def _eps_inv_loss_function():
    import torch

    class EpsInvLoss(torch.autograd.Function):
        """L = Re tr(W eps~^{-1}) as a function of the orbital energies and of the
        orbital samples at the interpolation points (N, N_mu); the other grid
        values of psi_t are held fixed.  Forward and backward are one call of the
        hand-written adjoint (isdf_eps_inv_grad); gradients follow torch's
        convention for real losses (dL/dRe + i dL/dIm)."""

        @staticmethod
        def forward(ctx, energies, psi_mu, psi_t, w, mu_idx, miller, prob, omega):
            mu = torch.as_tensor(np.asarray(mu_idx, dtype=np.int64), device=psi_t.device)
            psi = psi_t.detach().clone()
            psi[:, mu] = psi_mu.detach().to(psi.dtype)
            lval, ge, gp = eps_inv_grad(psi, energies.detach().cpu().numpy(), mu_idx, miller, prob, w, omega)
            ctx.save_for_backward(ge.to(energies.device), gp if psi_mu.is_complex() else gp.real.contiguous())
            return torch.tensor(lval, dtype=torch.float64, device=energies.device)

        @staticmethod
        def backward(ctx, g):
            ge, gp = ctx.saved_tensors
            return g * ge, (g.to(gp.device) * gp), None, None, None, None, None, None

    return EpsInvLoss


def eps_inv_loss(energies, psi_mu, psi_t, w, mu_idx, miller, prob: Problem, omega=0.0):
    """Differentiable L = Re tr(W eps~^{-1}) in (energies, psi_mu) through EpsInvLoss."""
    return _eps_inv_loss_function().apply(energies, psi_mu, psi_t, w, mu_idx, miller, prob, omega)


class Plan:
    """isdf_plan_*: validated once, then enqueue-only calls (no host sync per call).

    energies are passed as a device float64 tensor; device-side errors surface
    at sync()."""

    def __init__(self, prob: Problem, mu_idx, miller, n_omega: int = 0, device: int = 0, stream=None):
        # a fixed torch stream gives the plan a private handle bound to it (for
        # systems that run concurrently in eps_inv_multi); otherwise the shared
        # per-device handle follows torch's current stream
        self.h = handle(device) if stream is None else Handle(device, stream)
        self.device = device
        self.prob = prob
        mu, pmu = _i32(mu_idx)
        mi, pmi = _i32(miller)
        self.nmu, self.ng, self.n_omega = len(mu), len(mi), int(n_omega)
        import torch
        tb = ctypes.c_size_t(0)
        st = lib().isdf_plan_table_bytes(ctypes.byref(prob), pmu, len(mu), pmi, len(mi), self.n_omega,
                                         ctypes.byref(tb))
        if st != OK:
            raise IsdfError(st, "isdf_plan_table_bytes rejected the plan's arguments")
        # the plan's device tables live in this caller-owned buffer for the plan's lifetime
        self._tables, tptr = _workspace(int(tb.value), f"cuda:{device}")
        p = ctypes.c_void_p()
        self.h.check(lib().isdf_plan_create(self.h.h, ctypes.byref(prob), pmu, len(mu), pmi, len(mi),
                                            self.n_omega, ctypes.c_void_p(tptr), int(tb.value), ctypes.byref(p)),
                     "isdf_plan_create")
        self.p = p
        out = ctypes.c_size_t(0)
        self.h.check(lib().isdf_plan_workspace_bytes(self.p, ctypes.byref(out)), "isdf_plan_workspace_bytes")
        self.workspace_bytes = int(out.value)

    def new_workspace(self):
        import torch
        return torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=f"cuda:{self.device}")

    def new_output(self):
        import torch
        return torch.empty((max(self.n_omega, 1), self.ng, self.ng), dtype=torch.complex128,
                           device=f"cuda:{self.device}")

    def eps_inv_async(self, psi_t, energies_dev, out, workspace, omegas=None):
        import torch
        _check_psi(psi_t, self.prob)
        if (not isinstance(energies_dev, torch.Tensor) or energies_dev.device.type != "cuda"
                or energies_dev.dtype != torch.float64 or energies_dev.numel() != self.prob.nv + self.prob.nc
                or not energies_dev.is_contiguous()):
            raise TypeError("energies must be a contiguous device float64 tensor of N values")
        if out.dtype != torch.complex128 or tuple(out.shape) != (max(self.n_omega, 1), self.ng, self.ng):
            raise ValueError("out must be complex128 of shape (max(n_omega, 1), ng, ng)")
        om = np.zeros(0) if omegas is None else np.asarray(omegas, dtype=np.float64)
        if len(om) != self.n_omega:
            raise ValueError(f"the plan was made for {self.n_omega} frequencies")
        om, pom = _f64(om)
        self.h.sync_stream()
        wsbuf, wsptr = _workspace(self.workspace_bytes, psi_t.device, workspace)
        st = lib().isdf_plan_eps_inv(self.p, ctypes.c_void_p(psi_t.data_ptr()),
                                     ctypes.c_void_p(energies_dev.data_ptr()), pom if len(om) else None,
                                     ctypes.c_void_p(wsptr), self.workspace_bytes, ctypes.c_void_p(out.data_ptr()))
        self.h.check(st, "isdf_plan_eps_inv")
        return out

    def autotune(self, psi_t, energies_dev, out, workspace, omegas=None, reps=3) -> dict:
        """isdf_plan_autotune on these arguments; leaves the plan tuned."""
        _check_psi(psi_t, self.prob)
        om = np.zeros(0) if omegas is None else np.asarray(omegas, dtype=np.float64)
        if len(om) != self.n_omega:
            raise ValueError(f"the plan was made for {self.n_omega} frequencies")
        om, pom = _f64(om)
        self.h.sync_stream()
        wsbuf, wsptr = _workspace(self.workspace_bytes, psi_t.device, workspace)
        t = Tune()
        self.h.check(lib().isdf_plan_autotune(self.p, ctypes.c_void_p(psi_t.data_ptr()),
                                              ctypes.c_void_p(energies_dev.data_ptr()), pom if len(om) else None,
                                              ctypes.c_void_p(wsptr), self.workspace_bytes,
                                              ctypes.c_void_p(out.data_ptr()), int(reps), ctypes.byref(t)),
                     "isdf_plan_autotune")
        return t.as_dict()

    def get_tune(self) -> dict:
        t = Tune()
        self.h.check(lib().isdf_plan_get_tune(self.p, ctypes.byref(t)), "isdf_plan_get_tune")
        return t.as_dict()

    def set_tune(self, **knobs):
        t = Tune()
        lib().isdf_plan_get_tune(self.p, ctypes.byref(t))
        for k, v in knobs.items():
            setattr(t, k, int(v))
        self.h.check(lib().isdf_plan_set_tune(self.p, ctypes.byref(t)), "isdf_plan_set_tune")

    def time_stages(self, on: bool = True):
        """Record per-stage HIP events in every call; sync() then reports their means."""
        self.h.check(lib().isdf_plan_time_stages(self.p, 1 if on else 0), "isdf_plan_time_stages")

    def sync(self) -> Report:
        """isdf_plan_sync: waits for the stream of the plan's last call or graph launch."""
        rep = Report()
        self.h.check(lib().isdf_plan_sync(self.p, ctypes.byref(rep)), "isdf_plan_sync")
        return rep

    def __del__(self):
        try:
            if getattr(self, "p", None):
                lib().isdf_plan_destroy(self.p)
        except Exception:
            pass


def eps_inv_multi(plans, psis, energies_devs, outs, workspaces, omegas=None):
    """isdf_plan_eps_inv_multi: enqueue several systems at once (forked off the
    first plan's stream and joined back).  Sync each plan afterwards."""
    n = len(plans)
    if not (len(psis) == len(energies_devs) == len(outs) == len(workspaces) == n):
        raise ValueError("one psi, energies, output and workspace per plan")
    import torch
    for p, psi, e, w in zip(plans, psis, energies_devs, workspaces):
        _check_psi(psi, p.prob)
        if e.dtype != torch.float64 or e.numel() != p.prob.nv + p.prob.nc or e.device.type != "cuda":
            raise TypeError("energies must be device float64 tensors of N values")
        if w is None:
            raise ValueError("pass each plan's workspace (it must outlive the enqueued work)")
    plans[0].h.sync_stream()
    vp = ctypes.c_void_p
    P = (vp * n)(*[p.p for p in plans])
    PS = (vp * n)(*[psi.data_ptr() for psi in psis])
    E = (vp * n)(*[e.data_ptr() for e in energies_devs])
    keep = []
    OM = None
    if omegas is not None:
        arrs = []
        for p, om in zip(plans, omegas):
            a = np.zeros(0) if om is None else np.asarray(om, dtype=np.float64)
            if len(a) != p.n_omega:
                raise ValueError("each plan's frequency count must match")
            arrs.append(np.ascontiguousarray(a))
        keep = arrs
        OM = (vp * n)(*[a.ctypes.data if len(a) else None for a in arrs])
    W = []
    for p, w, psi in zip(plans, workspaces, psis):
        wsbuf, wsptr = _workspace(p.workspace_bytes, psi.device, w)
        W.append(wsptr)
        keep.append(wsbuf)
    WS = (vp * n)(*W)
    SZ = (ctypes.c_size_t * n)(*[p.workspace_bytes for p in plans])
    O = (vp * n)(*[o.data_ptr() for o in outs])
    st = lib().isdf_plan_eps_inv_multi(n, P, PS, E, OM, WS, SZ, O)
    plans[0].h.check(st, "isdf_plan_eps_inv_multi")
    return outs


class MultiGraph:
    """isdf_multi_graph_create: several plans' calls as one HIP graph whose systems run
    concurrently (each captured on its own plan's stream, its kernels copied into one graph).
    The buffers are baked into the graph and kept alive by this object."""

    def __init__(self, plans, psis, energies_devs, outs, workspaces, omegas=None):
        n = len(plans)
        if not (len(psis) == len(energies_devs) == len(outs) == len(workspaces) == n):
            raise ValueError("one psi, energies, output and workspace per plan")
        for p, psi, e, w in zip(plans, psis, energies_devs, workspaces):
            _check_psi(psi, p.prob)
            if w is None:
                raise ValueError("pass each plan's workspace")
        vp = ctypes.c_void_p
        self._keep = [plans, psis, energies_devs, outs]
        P = (vp * n)(*[p.p for p in plans])
        PS = (vp * n)(*[psi.data_ptr() for psi in psis])
        E = (vp * n)(*[e.data_ptr() for e in energies_devs])
        OM = None
        if omegas is not None:
            arrs = [np.ascontiguousarray(np.zeros(0) if om is None else np.asarray(om, dtype=np.float64))
                    for om in omegas]
            for p, a in zip(plans, arrs):
                if len(a) != p.n_omega:
                    raise ValueError("each plan's frequency count must match")
            self._keep.append(arrs)
            OM = (vp * n)(*[a.ctypes.data if len(a) else None for a in arrs])
        W = []
        for p, w, psi in zip(plans, workspaces, psis):
            wsbuf, wsptr = _workspace(p.workspace_bytes, psi.device, w)
            W.append(wsptr)
            self._keep.append(wsbuf)
        WS = (vp * n)(*W)
        SZ = (ctypes.c_size_t * n)(*[p.workspace_bytes for p in plans])
        O = (vp * n)(*[o.data_ptr() for o in outs])
        g = ctypes.c_void_p()
        st = lib().isdf_multi_graph_create(n, P, PS, E, OM, WS, SZ, O, ctypes.byref(g))
        plans[0].h.check(st, "isdf_multi_graph_create")
        self.g = g
        self.plans = plans

    def launch(self, stream=None):
        """isdf_graph_launch on `stream` (a torch stream; default: torch's current one)."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.plans[0].device)
        st = lib().isdf_graph_launch(self.g, ctypes.c_void_p(s.cuda_stream))
        if st != OK:
            raise IsdfError(st, "isdf_graph_launch failed")

    def __del__(self):
        try:
            if getattr(self, "g", None):
                lib().isdf_graph_destroy(self.g)
        except Exception:
            pass


def problem_for(inp, prec="fp64", refine_steps=0, v_scale=None, coulomb_sum=0, core_method=0, core_tol=0.0) -> Problem:
    """Problem description for a synthetic input set (synth.Inputs)."""
    return make_problem(inp.n, inp.cell, inp.nv, inp.nc, is_complex=inp.is_complex,
                        v_scale=inp.v_scale if v_scale is None else v_scale, prec=prec,
                        refine_steps=refine_steps, coulomb_sum=coulomb_sum, core_method=core_method,
                        core_tol=core_tol)
