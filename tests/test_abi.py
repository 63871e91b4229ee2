"""C ABI checks that need no GPU: the library loads, exports every call the
header declares, and rejects bad arguments on the host before any device work."""
import ctypes
import os
import re

import pytest

import paper_1307_2666_amd as hif
from paper_1307_2666_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hif.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hif_[a-z_A-Z]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = hif.load_library()
    names = _declared()
    assert "hif_factor" in names and "hif_solve_T" in names and "hif_matvec" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.EXPORTS)


def test_opts_default():
    o = hif.default_opts()
    assert (o.precision, o.second_kind, o.symmetric, o.variant, o.n_proxy, o.proxy_radius, o.max_bytes) == \
        (0, -1, -1, 0, 0, 0.0, 0)
    assert hif.load_library().hif_opts_default(None) == B.HIF_EINVAL


def _factor_raw(points=1, n=16, dim=2, kern=True, h=0.25, eps=1e-6, leaf=4, opts=None, out=True):
    lib = hif.load_library()
    k = B.hif_kernel(h, None, None)
    handle = ctypes.c_void_p()
    pts = ctypes.c_void_p(0x1000) if points else None  # never dereferenced: checks fail first
    st = lib.hif_factor(pts, n, dim, ctypes.byref(k) if kern else None, None, None, None, eps, leaf,
                        ctypes.byref(opts) if opts is not None else None, None,
                        ctypes.byref(handle) if out else None)
    return st, lib.hif_last_error().decode(), handle


@pytest.mark.parametrize("kw,needle", [
    (dict(points=0), "points"),
    (dict(n=0), "n must"),
    (dict(dim=4), "dim"),
    (dict(kern=False), "kernel"),
    (dict(h=0.0), "kernel.h"),
    (dict(h=float("nan")), "kernel.h"),
    (dict(eps=0.0), "eps"),
    (dict(eps=1.0), "eps"),
    (dict(eps=float("nan")), "eps"),
    (dict(leaf=0), "leaf"),
    (dict(out=False), "out"),
])
def test_factor_rejects_bad_arguments(kw, needle):
    st, msg, handle = _factor_raw(**kw)
    assert st == B.HIF_EINVAL
    assert needle in msg
    assert not handle.value


@pytest.mark.parametrize("field,value,status", [
    ("precision", 7, B.HIF_EINVAL),
    ("second_kind", 2, B.HIF_EINVAL),
    ("symmetric", -2, B.HIF_EINVAL),
    ("variant", 5, B.HIF_EINVAL),
    ("n_proxy", -1, B.HIF_EINVAL),
    ("proxy_radius", 0.25, B.HIF_EINVAL),
])
def test_factor_rejects_bad_options(field, value, status):
    o = hif.default_opts()
    setattr(o, field, value)
    st, msg, _ = _factor_raw(opts=o)
    assert st == status and field.split("_")[0] in msg


def test_sweeps_reject_null_handle():
    lib = hif.load_library()
    for name in ("hif_solve", "hif_solve_T", "hif_apply", "hif_apply_T"):
        assert getattr(lib, name)(None, None, None, 1, None) == B.HIF_EINVAL
    assert lib.hif_stats(None, None) == B.HIF_EINVAL
    lib.hif_free(None)  # no-op


def test_gmres_rejects_bad_arguments():
    lib = hif.load_library()
    buf = ctypes.c_double(0.0)
    p = ctypes.cast(ctypes.pointer(buf), ctypes.c_void_p)
    q = ctypes.cast(ctypes.pointer(ctypes.c_double(0.0)), ctypes.c_void_p)
    assert lib.hif_gmres(None, p, q, 1, 1e-10, 10, None, None, None) == B.HIF_EINVAL
    assert b"handle" in lib.hif_last_error()
    assert lib.hif_gmres_T(None, p, q, 1, 1e-10, 10, None, None, None) == B.HIF_EINVAL
    assert b"handle" in lib.hif_last_error()


def test_apply_A_rejects_bad_arguments():
    lib = hif.load_library()
    x, y = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert lib.hif_apply_A(None, x, y, 1, 0, None, None) == B.HIF_EINVAL
    assert b"handle" in lib.hif_last_error()
    o = hif.default_opts()
    assert o.fft_matvec == 0
    o.fft_matvec = 2
    st, msg, _ = _factor_raw(opts=o)
    assert st == B.HIF_EINVAL and "fft_matvec" in msg
    o = hif.default_opts()
    assert o.sweep_wait_us == 0
    o.sweep_wait_us = -1
    st, msg, _ = _factor_raw(opts=o)
    assert st == B.HIF_EINVAL and "sweep_wait_us" in msg


def test_factor_batch_rejects_bad_arguments():
    lib = hif.load_library()
    h = ctypes.c_void_p(0x1000)
    assert lib.hif_factor_batch(None, 0, None, 4, None, None) == B.HIF_OK  # empty batch
    assert lib.hif_factor_batch(None, -1, None, 4, None, None) == B.HIF_EINVAL
    assert lib.hif_factor_batch(None, 2, None, 4, h, None) == B.HIF_EINVAL
    probs = (B.hif_problem * 1)()
    assert lib.hif_factor_batch(ctypes.cast(probs, ctypes.c_void_p), 1, None, -1, h, None) == B.HIF_EINVAL
    assert b"nworkers" in lib.hif_last_error()
    assert lib.hif_factor_batch(ctypes.cast(probs, ctypes.c_void_p), 1, None, 17, h, None) == B.HIF_EINVAL
    # level-synchronous mode (nworkers = 0): a problem with bad arguments fails
    # alone, on the host, and is reported at its index
    out = (ctypes.c_void_p * 2)(0x1, 0x1)
    st = (ctypes.c_int * 2)(7, 7)
    probs2 = (B.hif_problem * 2)()
    probs2[1].points = 0x1000
    probs2[1].n = 0
    assert lib.hif_factor_batch(ctypes.cast(probs2, ctypes.c_void_p), 2, None, 0, ctypes.cast(out, ctypes.c_void_p),
                                ctypes.cast(st, ctypes.c_void_p)) == B.HIF_EINVAL
    assert list(st) == [B.HIF_EINVAL, B.HIF_EINVAL] and out[0] is None and out[1] is None
    assert b"problem 0: points is NULL" in lib.hif_last_error()


def test_diag_grad_rejects_bad_arguments():
    lib = hif.load_library()
    x, y, z = (ctypes.c_void_p(0x1000 * k) for k in (1, 2, 3))
    assert lib.hif_diag_grad(None, y, z, 4, 1, None) == B.HIF_EINVAL
    assert lib.hif_diag_grad(x, y, z, 0, 1, None) == B.HIF_EINVAL
    assert lib.hif_diag_grad(x, y, z, 4, 0, None) == B.HIF_EINVAL
    assert lib.hif_diag_grad(x, y, x, 4, 1, None) == B.HIF_EINVAL
    assert b"alias" in lib.hif_last_error()


def test_diff_solve_checks_shapes_on_the_host():
    import torch
    P = torch.zeros(16, 2, dtype=torch.float64)
    with pytest.raises(ValueError, match="a must"):
        hif.diff.solve(P, torch.ones(15), torch.ones(16), 1e-6, 4, h=0.25)
    with pytest.raises(ValueError, match="f must"):
        hif.diff.solve(P, torch.ones(16), torch.ones(2, 15), 1e-6, 4, h=0.25)
    with pytest.raises(ValueError, match="tol"):
        hif.diff.solve(P, torch.ones(16), torch.ones(16), 1e-6, 4, h=0.25, refine=True, tol=0.0)


def test_matvec_rejects_bad_arguments():
    lib = hif.load_library()
    k = B.hif_kernel(0.1, None, None)
    p = ctypes.c_void_p(0x1000)
    x = ctypes.c_void_p(0x2000)
    y = ctypes.c_void_p(0x3000)
    assert lib.hif_matvec(None, 4, 2, ctypes.byref(k), None, None, None, x, y, 1, None) == B.HIF_EINVAL
    assert lib.hif_matvec(p, 4, 2, ctypes.byref(k), None, None, None, x, x, 1, None) == B.HIF_EINVAL
    assert lib.hif_matvec(p, 4, 5, ctypes.byref(k), None, None, None, x, y, 1, None) == B.HIF_EINVAL
    assert lib.hif_matvec(p, 4, 2, ctypes.byref(k), None, None, None, x, y, 0, None) == B.HIF_EINVAL
    assert lib.hif_matvec(p, 4, 2, None, None, None, None, x, y, 1, None) == B.HIF_EINVAL


def test_partition_and_id_reject_bad_arguments():
    lib = hif.load_library()
    p = ctypes.c_void_p(0x1000)
    assert lib.hif_partition(p, 4, 2, p, 1, 2, p, None) == B.HIF_EINVAL  # faces need 3D
    assert lib.hif_partition(p, 4, 2, p, 0, 0, p, None) == B.HIF_EINVAL
    assert lib.hif_partition(None, 4, 2, p, 0, 2, p, None) == B.HIF_EINVAL
    assert lib.hif_id_batched(p, p, p, p, p, -1, 4, p, p, p, None, None, None) == B.HIF_EINVAL
    assert lib.hif_id_batched(p, p, p, p, p, 0, 4, p, p, p, None, None, None) == B.HIF_OK
    assert lib.hif_id_batched(p, p, p, p, p, 2, 5000, p, p, p, None, None, None) == B.HIF_EINVAL
    assert lib.hif_id_batched(p, p, p, p, p, 2, 4, p, p, p, p, None, None) == B.HIF_EINVAL


def test_solve_noalloc_rejects_bad_arguments():
    lib = hif.load_library()
    x, y = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert lib.hif_solve_noalloc(None, x, y, 1, None) == B.HIF_EINVAL
    assert b"handle" in lib.hif_last_error()
    h = ctypes.c_void_p(0x3000)  # never dereferenced: the checks fail first
    assert lib.hif_solve_noalloc(h, None, y, 1, None) == B.HIF_EINVAL
    assert lib.hif_solve_noalloc(h, x, y, 0, None) == B.HIF_EINVAL
    assert hif.HIF_SOLVE_NOALLOC_MAX == 4 << 20


def test_struct_layouts_match_the_header(tmp_path):
    # Every ctypes mirror of an include/hif.h struct has the C compiler's size
    # and field offsets (a field added on one side only would shift the rest).
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [("hif_kernel", B.hif_kernel), ("hif_opts", B.hif_opts), ("hif_problem", B.hif_problem),
               ("hif_tuning", B.hif_tuning), ("hif_stats_t", B.hif_stats_t)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hif.h"', "int main(void) {"]
    want = []
    for cname, py in structs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(py))
        for fname, _ in py._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {fname}));')
            want.append(getattr(py, fname).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c11", "-I", inc, "-o", str(exe), str(src)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == want
    # and the same members in the same order (a C-only field could hide in padding)
    with open(os.path.join(inc, "hif.h")) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    for cname, py in structs:
        body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + cname + r"\s*;", text)
        assert body, cname
        members = []
        for decl in body.group(1).split(";"):
            for d in decl.split(","):  # several declarators: "const double *a, *b, *c"
                d = re.sub(r"\[[^\]]*\]", "", d).strip()
                if d:
                    members.append(re.findall(r"\w+", d)[-1])
        assert members == [fname for fname, _ in py._fields_], cname
