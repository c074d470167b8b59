"""C ABI checks that need no GPU: the library loads, exports every declared
function, and its host-side logic (plane-wave list, workspace sizing, argument
validation) behaves as documented."""
import ctypes
import pathlib

import numpy as np
import pytest

import paper_2403_12340_amd as isdf
import synth

ROOT = pathlib.Path(__file__).resolve().parent.parent


def test_library_exports_every_declared_symbol():
    lib = isdf.lib()
    names = isdf.header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert lib.isdf_version().startswith(b"isdf-smw-gfx950")


@pytest.mark.parametrize("name", ["tiny", "cfg0", "mid", "cfg1"])
def test_gvectors_match_generator(name):
    c = synth.CONFIGS[name]
    n = c["n"]
    prob = isdf.make_problem(n, np.eye(3) * synth.box_length(c["nv"]), c["nv"], c["nc"])
    got = isdf.gvectors(prob, c["ng"])
    np.testing.assert_array_equal(got, synth.miller_list(n, c["ng"]))


def test_workspace_bytes_monotone_and_validated():
    prob = isdf.make_problem(48, np.eye(3) * 20.0, 64, 256)
    a = isdf.workspace_bytes(prob, 640, 4096)
    b = isdf.workspace_bytes(prob, 700, 4096)
    c = isdf.workspace_bytes(prob, 640, 5000)
    assert 0 < a < b and a < c
    # FP32 stores the large intermediates in complex64: smaller
    p32 = isdf.make_problem(48, np.eye(3) * 20.0, 64, 256, prec="fp32")
    assert isdf.workspace_bytes(p32, 640, 4096) < a
    out = ctypes.c_size_t(0)
    bad = isdf.make_problem(48, np.eye(3) * 20.0, 64, 256)
    bad.nv = 0
    assert isdf.lib().isdf_workspace_bytes(ctypes.byref(bad), 640, 4096, 0, ctypes.byref(out)) == isdf.binding.E_ARG
    assert isdf.lib().isdf_workspace_bytes(ctypes.byref(prob), 0, 4096, 0, ctypes.byref(out)) == isdf.binding.E_ARG


def test_workspace_bytes_whole_grid_gram():
    """coulomb_sum = 1 sizes the Gram operands for every grid vector; other values are rejected."""
    prob = isdf.make_problem(48, np.eye(3) * 20.0, 64, 256, prec="fp32")
    full = isdf.make_problem(48, np.eye(3) * 20.0, 64, 256, prec="fp32", coulomb_sum=1)
    a = isdf.workspace_bytes(prob, 640, 4096)
    b = isdf.workspace_bytes(full, 640, 4096)
    # at least the N_mu x Nr complex64 X^T the whole-grid Gram reads
    assert b - a >= 640 * (48 ** 3 - 4096) * 8
    out = ctypes.c_size_t(0)
    bad = isdf.make_problem(48, np.eye(3) * 20.0, 64, 256, coulomb_sum=2)
    assert isdf.lib().isdf_workspace_bytes(ctypes.byref(bad), 640, 4096, 0, ctypes.byref(out)) == isdf.binding.E_ARG


@pytest.fixture(scope="module")
def cfg0():
    return synth.make_inputs("cfg0")


def test_check_inputs_accepts_valid(cfg0):
    prob = isdf.problem_for(cfg0)
    assert isdf.check_inputs(prob, cfg0.energies, cfg0.mu_idx, cfg0.miller) == (0, "")
    assert isdf.check_inputs(prob, cfg0.energies, cfg0.mu_idx, cfg0.miller, omegas=[0.0, 0.1, 3.0])[0] == 0


def test_check_inputs_rejects(cfg0):
    x = cfg0
    prob = isdf.problem_for(x)
    E = isdf.binding.E_ARG

    def st(**kw):
        args = dict(energies=x.energies, mu_idx=x.mu_idx, miller=x.miller, omegas=None)
        args.update(kw)
        p = kw.pop("prob", prob)
        return isdf.check_inputs(p, args["energies"], args["mu_idx"], args["miller"], args["omegas"])

    dup = x.mu_idx.copy(); dup[3] = dup[2]
    assert st(mu_idx=dup) == (E, "mu_idx has duplicate points")
    oob = x.mu_idx.copy(); oob[0] = x.nr
    assert st(mu_idx=oob)[0] == E
    assert st(mu_idx=np.arange(x.nv * x.nc + 1))[0] == E
    e = x.energies.copy(); e[x.nv - 1] = e[x.nv] + 0.01
    assert st(energies=e)[1].startswith("no gap")
    e = x.energies.copy(); e[0] = np.nan
    assert st(energies=e)[0] == E
    m = x.miller.copy(); m[5] = m[4]
    assert st(miller=m)[1] == "miller list has duplicates"
    m = x.miller.copy(); m[7, 0] = x.n // 2
    assert st(miller=m)[0] == E
    assert st(omegas=[0.1, -1.0])[0] == E
    p = isdf.problem_for(x); p.n[1] = 1
    assert st(prob=p)[0] == E
    p = isdf.problem_for(x); p.refine_steps = 9
    assert st(prob=p)[0] == E
    p = isdf.problem_for(x); p.cell[0] = 0.0; p.cell[4] = 0.0
    assert st(prob=p)[0] == E


def test_create_without_gpu_is_an_error():
    """No GPU here: creating a handle must fail cleanly, never fall back to the CPU."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert isdf.lib().isdf_create(ctypes.byref(h), 0, None) != 0
    assert isdf.lib().isdf_eps_inv(None, None, None, None, None, 0, None, 0, None, 0, None, 0, None, None) == isdf.binding.E_ARG


@pytest.mark.parametrize("name", ["tiny", "cfg0", "cfg1"])
def test_contour_nodes_match_oracle(name):
    """The library's host contour rule (its own arithmetic-geometric-mean Jacobi
    functions) against the oracle's (scipy's), node by node."""
    from oracle import cauchy as oc
    inp = synth.make_inputs(name)
    z, w = isdf.contour_nodes(inp.energies, inp.nv, inp.nc, 1e-13)
    ev, q, big_q = oc.gap_and_width(inp.energies, inp.nv)
    assert len(z) == oc.nodes_for_tolerance(q, big_q, 1e-13)
    zo, wo = oc.contour_nodes(q, big_q, len(z))
    assert np.abs(z - (zo + ev)).max() <= 1e-13 * np.abs(z).max()
    assert np.abs(w - wo).max() <= 1e-13 * np.abs(w).max()


def test_contour_nodes_validated():
    bad = np.array([1.0, 0.5, 2.0])   # occupied above empty
    with pytest.raises(isdf.IsdfError):
        isdf.contour_nodes(bad, 2, 1)
    prob = isdf.make_problem(12, np.eye(3) * 10.0, 8, 24, core_method=2)
    out = ctypes.c_size_t(0)
    assert isdf.lib().isdf_workspace_bytes(ctypes.byref(prob), 96, 256, 0, ctypes.byref(out)) == isdf.binding.E_ARG


def test_plan_table_bytes(cfg0):
    """The plan's device tables (status block, points, plane waves, DFT index lists)
    are sized on the host; invalid plan arguments are refused before any GPU call."""
    x = cfg0
    prob = isdf.problem_for(x)
    lib = isdf.lib()
    out = ctypes.c_size_t(0)
    mu = np.ascontiguousarray(x.mu_idx, dtype=np.int32)
    mi = np.ascontiguousarray(x.miller, dtype=np.int32)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    st = lib.isdf_plan_table_bytes(ctypes.byref(prob), mu.ctypes.data_as(pi32), len(mu), mi.ctypes.data_as(pi32),
                                   len(mi), 0, ctypes.byref(out))
    assert st == 0
    # at least the point indices, the Miller list and one index per plane wave
    assert out.value >= 4 * len(mu) + 12 * len(mi) + 4 * len(mi)
    assert out.value % 256 == 0
    bad = mu.copy(); bad[1] = bad[0]
    st = lib.isdf_plan_table_bytes(ctypes.byref(prob), bad.ctypes.data_as(pi32), len(bad), mi.ctypes.data_as(pi32),
                                   len(mi), 0, ctypes.byref(out))
    assert st == isdf.binding.E_ARG
    full = isdf.problem_for(x, coulomb_sum=1)
    big = ctypes.c_size_t(0)
    assert lib.isdf_plan_table_bytes(ctypes.byref(full), mu.ctypes.data_as(pi32), len(mu), mi.ctypes.data_as(pi32),
                                     len(mi), 0, ctypes.byref(big)) == 0
    assert big.value > out.value   # every grid vector in the Gram's list


def _header_structs():
    """Field (name, ctype, count) lists of every `typedef struct { ... } name;` in the header."""
    import re
    text = (ROOT / "include" / "isdf_smw.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    types = {"int32_t": ctypes.c_int32, "double": ctypes.c_double}
    out = {}
    for body, name in re.findall(r"typedef struct \{(.*?)\}\s*(\w+);", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            ty, names = decl.split(None, 1)
            for nm in names.split(","):
                m = re.fullmatch(r"\s*(\w+)(?:\[(\d+)\])?\s*", nm)
                fields.append((m.group(1), types[ty], int(m.group(2) or 1)))
        out[name] = fields
    return out


@pytest.mark.parametrize("cname,pyname", [("isdf_problem", "Problem"), ("isdf_report", "Report"),
                                          ("isdf_tune", "Tune")])
def test_binding_structs_match_header(cname, pyname):
    """The ctypes structures of the binding have the header's fields, in order, with its types."""
    from paper_2403_12340_amd import binding
    want = _header_structs()[cname]
    got = []
    for nm, ty in getattr(binding, pyname)._fields_:
        if hasattr(ty, "_length_"):
            got.append((nm, ty._type_, ty._length_))
        else:
            got.append((nm, ty, 1))
    assert got == want
