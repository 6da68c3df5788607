"""Host-side checks of the C-ABI library (no GPU needed): it loads and
exports every entry point include/elh.h declares; the binding's structures
match the header's field lists."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "elh.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(elh_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = _declared()
    for need in ("elh_create", "elh_apply", "elh_vcycle", "elh_solve", "elh_solve_adjoint",
                 "elh_gradient", "elh_destroy"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2307_03242_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libelh.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(_declared()) == sorted(_lib.EXPORTED)


def test_desc_layout_matches_header():
    from paper_2307_03242_amd import _lib
    src = open(HEADER).read()
    body = src[src.index("typedef struct {", src.index("ELH_C128 = 2")):src.index("} elh_desc;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    body = body.split("{", 1)[1]
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1]
        fields += [re.sub(r"\[.*\]", "", nm).strip() for nm in names.split(",")]
    assert fields == [f[0] for f in _lib.Desc._fields_]


def test_status_strings_without_gpu():
    from paper_2307_03242_amd import _lib
    lib = _lib.load()
    assert lib.elh_status_string(0) == b"ok"
    assert lib.elh_status_string(-1) == b"invalid argument"


def test_create_rejects_bad_arguments_without_gpu():
    """argument validation happens before any device call"""
    from paper_2307_03242_amd import _lib
    lib = _lib.load()
    d = _lib.Desc()
    d.dim = 3
    d.n[0], d.n[1], d.n[2] = 10, 8, 8
    d.h, d.beta, d.levels = 1.0, 2 / 3, 3          # 10 not divisible by 4
    d.nu1 = d.nu2 = 1
    d.coarse_sweeps, d.coarse_restart, d.coarse_maxit = 2, 5, 10
    d.precond_dtype = _lib.ELH_C128
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    assert lib.elh_create(ctypes.byref(d), dummy, dummy, dummy, None, ctypes.byref(h)) == _lib.ELH_ERR_ARG
    assert b"divisible" in lib.elh_last_error()
    d.n[0] = 8
    d.beta = 1.5
    assert lib.elh_create(ctypes.byref(d), dummy, dummy, dummy, None, ctypes.byref(h)) == _lib.ELH_ERR_ARG


class _NoCallLib:
    """stands in for libelh: any call into it fails the test"""

    def __getattr__(self, name):
        def call(*a, **k):
            raise AssertionError("library entry point %s reached" % name)
        return call


def _cpu_problem():
    """a Problem whose vectors may live on the host: the binding's argument
    checks run without a GPU, and nothing reaches the library"""
    import torch
    from paper_2307_03242_amd.api import Problem

    class HostProblem(Problem):
        def _vec(self, t, level):
            full = (self.dim + 1,) + self.shape
            if tuple(t.shape) == full:
                return 1
            if t.dim() == len(full) + 1 and tuple(t.shape[1:]) == full:
                return t.shape[0]
            raise ValueError("shape")

    p = object.__new__(HostProblem)
    p.lib = _NoCallLib()
    p.device = torch.device("cpu")
    p.dim, p.shape, p.levels = 3, (4, 4, 4), 2
    p.handle = ctypes.c_void_p(0)
    return p


def test_solve_and_gradient_check_their_buffers_without_gpu():
    """a caller-supplied solution buffer and the adjoint fields of the
    gradient must have the right-hand side's layout and dtype before any
    library call (the library reads and writes nrhs full complex128
    vectors through them)"""
    import torch
    p = _cpu_problem()
    q = torch.zeros((2, 4, 4, 4, 4), dtype=torch.complex128)
    for bad in (torch.zeros_like(q, dtype=torch.complex64), q[:1].clone(), torch.zeros(q.numel() // 2, dtype=q.dtype),
                torch.zeros((2, 4, 4, 4, 8), dtype=q.dtype)[..., :4]):
        with pytest.raises(ValueError):
            p.solve(q, out=bad)
    with pytest.raises(TypeError):
        p.gradient(q.to(torch.complex64), q.to(torch.complex64))
    for bad in (q.to(torch.complex64), q[:1].clone(), torch.zeros((2, 4, 4, 4, 8), dtype=q.dtype)[..., :4]):
        with pytest.raises(ValueError):
            p.gradient(q, bad)


def test_create_rejects_a_singular_shift_without_gpu():
    """gamma + alpha must be positive (the shifted operator is then
    nonsingular), neither negative, and omega positive: ELH_ERR_ARG before
    any device call"""
    from paper_2307_03242_amd import _lib
    lib = _lib.load()
    d = _lib.Desc()
    d.dim = 3
    d.n[0] = d.n[1] = d.n[2] = 8
    d.h, d.beta, d.levels, d.omega = 1.0, 2 / 3, 2, 0.5
    d.nu1 = d.nu2 = 1
    d.cycle_calls = 1
    d.coarse_sweeps, d.coarse_restart, d.coarse_maxit = 2, 5, 10
    d.precond_dtype = _lib.ELH_C128
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    for g, a, om in ((0.0, 0.0, 0.5), (-0.01, 0.3, 0.5), (0.01, -0.3, 0.5), (0.01, 0.3, 0.0),
                     (float("nan"), 0.3, 0.5), (0.01, 0.3, float("inf"))):
        d.gamma, d.alpha, d.omega = g, a, om
        assert lib.elh_create(ctypes.byref(d), dummy, dummy, dummy, None, ctypes.byref(h)) == _lib.ELH_ERR_ARG
        assert not h.value


def test_receiver_binding_checks_without_gpu():
    """receiver indices must be a device int64 vector, the mask a bool
    tensor of the vector's shape: ValueError before any library call"""
    import torch
    p = _cpu_problem()
    with pytest.raises(ValueError):
        p.receiver_indices(torch.zeros((4, 4, 4, 4), dtype=torch.int32))
    with pytest.raises(ValueError):
        p.receiver_indices(torch.zeros((3, 4, 4, 4), dtype=torch.bool))
    with pytest.raises(ValueError):
        p._idx(torch.arange(3))          # host tensor
    with pytest.raises(ValueError):
        p.inject(torch.zeros(3, dtype=torch.complex128), torch.arange(3))
