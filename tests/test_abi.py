"""C-ABI contract tests that need no GPU: the library loads, exports every
function include/randrand.h declares, fills defaults, and rejects invalid
arguments with RR_EINVAL before any device work (device calls on a machine
without a GPU return RR_EDEVICE)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "randrand.h")

b = pytest.importorskip("paper_2509_19747_amd.binding")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(rr_[a-z0-9_]+)\s*\(", txt))
    # typedef'd function pointer names are not exports
    fn_ptrs = set(re.findall(r"\(\*\s*(rr_[a-z0-9_]+)\s*\)", txt))
    return sorted(names - fn_ptrs)


def test_library_exports_every_declared_symbol():
    L = b.lib()
    decl = _declared()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), f"{name} not exported"


def test_defaults():
    o = b.rr_build_opts()
    b.lib().rr_build_opts_default(C.byref(o))
    assert o.l == 0 and o.power_iters == 4 and o.rho == 1.0 and o.tau_rule == b.TAU_OPT
    s = b.rr_solve_opts()
    b.lib().rr_solve_opts_default(C.byref(s))
    assert s.tol == 1e-6 and s.restart_eta == 1e-2 and s.maxit == 5000 and s.check_every == 8
    assert s.certify == 1


def test_status_strings_and_version():
    L = b.lib()
    for code in range(8):
        assert L.rr_status_string(code).startswith(b"RR_")
    assert b"randrand" in L.rr_version()


def _dense_op(n=10, lda=10, ptr=0x1000):
    return b.rr_operator(kind=b.OP_DENSE, n=n, A=ptr, lda=lda, pts=None, d=0, kconst=0, scale=1)


@pytest.mark.parametrize("bad", [
    dict(n=0), dict(lda=3), dict(ptr=None),
])
def test_build_rejects_bad_operator(bad):
    L = b.lib()
    kw = dict(n=10, lda=10, ptr=0x1000)
    kw.update(bad)
    op = _dense_op(**kw)
    mus = (C.c_double * 1)(1e-3)
    h = C.c_void_p()
    st = L.rr_build_precond(C.byref(op), mus, 1, None, None, None, C.byref(h))
    assert st == b.RR_EINVAL and not h.value


@pytest.mark.parametrize("mu,l,nmu", [(-1.0, 2, 1), (float("nan"), 2, 1), (1e-3, 11, 1),
                                      (1e-3, -1, 1), (1e-3, 6, 2), (1e-3, 2, 0)])
def test_build_rejects_bad_options(mu, l, nmu):
    L = b.lib()
    op = _dense_op()
    mus = (C.c_double * 2)(mu, mu)
    o = b.build_opts(l=l)
    h = C.c_void_p()
    st = L.rr_build_precond(C.byref(op), mus, nmu, C.byref(o), None, None, C.byref(h))
    assert st == b.RR_EINVAL
    assert L.rr_last_error()


def test_kernel_operator_validation():
    L = b.lib()
    op = b.rr_operator(kind=b.OP_RBF, n=10, A=None, lda=0, pts=0x1000, d=0, kconst=1.0, scale=1.0)
    h = C.c_void_p()
    mus = (C.c_double * 1)(1e-3)
    assert L.rr_build_precond(C.byref(op), mus, 1, None, None, None, C.byref(h)) == b.RR_EINVAL
    op.d = 3
    op.kconst = -1.0
    assert L.rr_build_precond(C.byref(op), mus, 1, None, None, None, C.byref(h)) == b.RR_EINVAL
    op.kind = 9
    assert L.rr_build_precond(C.byref(op), mus, 1, None, None, None, C.byref(h)) == b.RR_EINVAL


def test_apply_operator_block_validation():
    L = b.lib()
    op = _dense_op()
    buf = np.zeros(16)
    p = buf.ctypes.data_as(C.c_void_p)
    assert L.rr_apply_operator_block(C.byref(op), 0.0, b.PREC_FP64, p, 0, p, None) == b.RR_EINVAL
    assert L.rr_apply_operator_block(C.byref(op), 0.0, b.PREC_FP64, None, 1, p, None) == b.RR_EINVAL
    assert L.rr_apply_operator_block(C.byref(op), float("nan"), b.PREC_FP64, p, 1, p, None) == b.RR_EINVAL
    assert L.rr_apply_operator_block(C.byref(op), 0.0, 7, p, 1, p, None) == b.RR_EINVAL


def test_solve_rejects_null_handle_and_bad_tol():
    L = b.lib()
    info = b.rr_solve_info()
    o = b.solve_opts(tol=0.0)
    assert L.rr_solve(None, 0, None, None, C.byref(o), C.byref(info), None) == b.RR_EINVAL
    assert info.status == b.RR_EINVAL
    o = b.solve_opts(tol=1e-6)
    assert L.rr_solve(None, 0, None, None, C.byref(o), C.byref(info), None) == b.RR_EINVAL


def test_device_calls_without_gpu_report_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = b.lib()
    op = _dense_op()
    mus = (C.c_double * 1)(1e-3)
    h = C.c_void_p()
    st = L.rr_build_precond(C.byref(op), mus, 1, None, None, None, C.byref(h))
    assert st == b.RR_EDEVICE
    out = np.zeros(4)
    st = L.rr_random_matrix(0, 1, 2, 2, out.ctypes.data_as(C.c_void_p), None)
    assert st == b.RR_EDEVICE


def test_serve_rejects_null_config():
    L = b.lib()
    stats = b.rr_serve_stats()
    nf = b.NEXT_FN(lambda u, t, r: -1)
    df = b.DELIVER_FN(lambda u, r, i, t: None)
    assert L.rr_serve(None, nf, df, None, C.byref(stats)) == b.RR_EINVAL


def test_ctypes_structures_match_the_header_layout(tmp_path):
    """Every structure the binding mirrors has the header's size and field offsets
    (a C program built with gcc from include/randrand.h prints them)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    structs = [b.rr_operator, b.rr_build_opts, b.rr_solve_opts, b.rr_solve_info, b.rr_allocator,
               b.rr_request, b.rr_serve_config, b.rr_serve_stats]
    lines = ["#include <stddef.h>", "#include <stdio.h>", f'#include "{HEADER}"', "int main(void) {"]
    for s in structs:
        name = s.__name__
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in s._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c11", str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line.strip()}
    for s in structs:
        name = s.__name__
        assert got[(name, "size")] == C.sizeof(s), name
        for f, _ in s._fields_:
            assert got[(name, f)] == getattr(s, f).offset, (name, f)
