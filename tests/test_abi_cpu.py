"""The C ABI library loads without a GPU, exports every entry point include/mrq.h declares, and
rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re
import tempfile

import numpy as np
import pytest

import paper_2411_06158_amd as mrq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mrq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mrq_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mrq_build", "mrq_search", "mrq_search_mixed", "mrq_export", "mrq_save", "mrq_load", "mrq_free",
                 "mrq_last_error", "mrq_server_create", "mrq_server_submit", "mrq_server_poll"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = mrq.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(mrq.EXPORTED) == declared_functions()


def test_option_defaults():
    b = mrq.BuildOpts()
    mrq.lib().mrq_build_opts_default(C.byref(b))
    assert b.seed == 4001 and b.kmeans_iters == 25
    s = mrq.SearchOpts()
    mrq.lib().mrq_search_opts_default(C.byref(s))
    assert (s.mode, s.bq, s.stage2, s.use_ext, s.group) == (0, 4, 1, 1, 0)
    assert abs(s.eps0 - 1.9) < 1e-6 and s.m == 3.0
    assert b.sq8 == 0 and (s.method, s.rerank) == (mrq.MRQ_METHOD_MRQ, 0)


def test_option_struct_layout_matches_header(tmp_path):
    """The binding's option structs have the size and field offsets the C header gives them."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    fields = {"mrq_build_opts": [n for n, _ in mrq.BuildOpts._fields_],
              "mrq_search_opts": [n for n, _ in mrq.SearchOpts._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mrq.h"', "int main(void) {"]
    for st, names in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for n in names:
            lines.append(f'printf("{st}.{n} %zu\\n", offsetof({st}, {n}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for st, cls in (("mrq_build_opts", mrq.BuildOpts), ("mrq_search_opts", mrq.SearchOpts)):
        assert int(got[st]) == C.sizeof(cls)
        for n in fields[st]:
            assert int(got[f"{st}.{n}"]) == getattr(cls, n).offset, (st, n)


def _build(X, N, D, d, B, nlist):
    h = C.c_void_p()
    st = mrq.lib().mrq_build(None if X is None else X.ctypes.data, N, D, d, B, nlist, None, None, C.byref(h))
    return st, h


@pytest.mark.parametrize("N,D,d,B,nlist,msg", [
    (0, 8, 4, 1, 1, "N"), (100, 1, 1, 1, 1, "D"), (100, 8, 9, 1, 4, "d_r"), (100, 8, 1, 1, 4, "d_r"),
    (100, 8, 4, 0, 4, "bits"), (100, 8, 4, 9, 4, "bits"), (100, 8, 4, 1, 0, "nlist"), (100, 8, 4, 1, 101, "nlist"),
    (20000, 8, 4, 1, 16385, "nlist"),
])
def test_build_rejects_bad_arguments(N, D, d, B, nlist, msg):
    X = np.zeros((max(N, 1), D), np.float32)
    st, h = _build(X, N, D, d, B, nlist)
    assert st == mrq.MRQ_EINVAL and not h.value
    assert msg in mrq.lib().mrq_last_error().decode()


def test_null_pointers_rejected():
    st, _ = _build(None, 10, 4, 2, 1, 1)
    assert st == mrq.MRQ_EINVAL
    ids = np.zeros(10, np.int64)
    dd = np.zeros(10, np.float32)
    q = np.zeros(4, np.float32)
    assert mrq.lib().mrq_search(None, q.ctypes.data, 1, 10, 1, ids.ctypes.data, dd.ctypes.data, None, None) == mrq.MRQ_EINVAL
    assert mrq.lib().mrq_export(None, b"/tmp/x") == mrq.MRQ_EINVAL
    srv = C.c_void_p()
    assert mrq.lib().mrq_server_create(None, 0, 8, None, C.byref(srv)) == mrq.MRQ_EINVAL
    assert mrq.lib().mrq_server_poll(None, None, None, None, None, 1, 1, None) == -1
    mrq.lib().mrq_free(None)  # ignored


def test_load_rejects_missing_and_corrupt_files():
    h = C.c_void_p()
    assert mrq.lib().mrq_load(b"/nonexistent/index.mrqs", C.byref(h)) == mrq.MRQ_EIO
    with tempfile.NamedTemporaryFile(suffix=".mrqs", delete=False) as f:
        f.write(b"NOTANIDX" + b"\0" * 64)
        path = f.name
    try:
        assert mrq.lib().mrq_load(path.encode(), C.byref(h)) == mrq.MRQ_EIO
        assert "MRQS0005" in mrq.lib().mrq_last_error().decode()
    finally:
        os.unlink(path)


@pytest.mark.parametrize("spectrum,D,want", [
    ("power1.2", 960, 128),     # 128 leading axes of i^-1.2 over 960 hold 85.5 % of the variance
    ("flat", 960, 960),         # 80 % needs 768 axes: the next power of two passes D, so D
    ("flat", 100, 100),         # fewer than 128 dimensions: all of them
    ("power0.5", 1536, 1024),   # i^-0.5 over 1536: 512 axes hold 57 %, 1024 hold 81 %
    ("flat", 2048, 1024),       # 80 % needs 2048 > 1536, the largest supported power of two
    ("head", 1536, 256),        # 90 % in the top 200 axes
])
def test_choose_dr_follows_eq8(spectrum, D, want):
    i = np.arange(1, D + 1, dtype=np.float64)
    lam = {"power1.2": i ** -1.2, "flat": np.ones(D), "power0.5": i ** -0.5,
           "head": np.where(i <= 200, 0.9 / 200, 0.1 / (D - 200))}[spectrum]
    assert mrq.choose_dr(lam) == want


def test_choose_dr_rejects_bad_input():
    assert mrq.lib().mrq_choose_dr(None, 10) == -1
