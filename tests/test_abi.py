"""The C library loads, exports every entry point declared in include/riop.h,
and the binding's ctypes structures have the C layout (checked by compiling a
probe of the header with gcc).  Host-side argument validation is exercised
without touching a GPU."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "riop.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(riop_[a-z_]+)\s*\(", text)))


def test_library_exports_header_symbols():
    from paper_1307_4370_amd import _lib
    L = _lib.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), f"{name} declared in riop.h but not exported"
    assert set(names) == set(_lib.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (riop_[a-z_]+)$", out, re.M))
    assert exported == set(names)


def test_version():
    import paper_1307_4370_amd as P
    assert P.version().startswith("riop ")


def test_struct_layouts_match_header():
    from paper_1307_4370_amd import _lib
    probe = r"""
#include <stdio.h>
#include <stddef.h>
#include "riop.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("riop_desc %zu\nriop_info %zu\nriop_sdmm_params %zu\nriop_sdmm_stats %zu\n",
         sizeof(riop_desc), sizeof(riop_info), sizeof(riop_sdmm_params), sizeof(riop_sdmm_stats));
  P(riop_desc, M) P(riop_desc, tile) P(riop_desc, reserved)
  P(riop_info, M) P(riop_info, kb_beta) P(riop_info, device_bytes)
  P(riop_sdmm_params, gamma) P(riop_sdmm_params, weights) P(riop_sdmm_params, history)
  P(riop_sdmm_stats, gamma) P(riop_sdmm_stats, nu)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "p.c"), os.path.join(d, "p")
        open(src, "w").write(probe)
        subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", f"-I{os.path.dirname(HEADER)}", src, "-o", exe],
                       check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.rsplit(" ", 1) for l in lines if l)
    S = {"riop_desc": _lib.Desc, "riop_info": _lib.Info, "riop_sdmm_params": _lib.SdmmParams,
         "riop_sdmm_stats": _lib.SdmmStats}
    for cname, cls in S.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
    for key, val in got.items():
        if "." in key:
            cname, field = key.split(".")
            assert getattr(S[cname], field).offset == int(val), key


def test_host_validation_without_gpu():
    from paper_1307_4370_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.riop_plan_create(None, None, None, ctypes.byref(h)) == -1
    assert b"desc" in L.riop_last_error()
    bad = [dict(n=30, levels=2), dict(n=64, J=7), dict(n=64, levels=7), dict(n=64, dict_mask=0),
           dict(n=64, dict_mask=1 << 9), dict(n=64, prec=3), dict(n=64, tile=12)]
    for kw in bad:
        d = _lib.Desc(n=kw.get("n", 64), oversample=2, M=10, J=kw.get("J", 8), levels=kw.get("levels", 2),
                      dict_mask=kw.get("dict_mask", 511), prec=kw.get("prec", 1), tile=kw.get("tile", 0))
        st = L.riop_plan_create(ctypes.byref(d), None, None, ctypes.byref(h))
        assert st in (-1, -2, -5), (kw, st)
        assert h.value is None
    d = _lib.Desc(n=64, oversample=3, M=10, J=8, levels=2, dict_mask=511, prec=1)
    assert L.riop_plan_create(ctypes.byref(d), None, None, ctypes.byref(h)) == -5
    # Above the largest image side the FFT passes take (K = 2n <= 6144).
    d = _lib.Desc(n=4096, oversample=2, M=10, J=8, levels=2, dict_mask=511, prec=1)
    assert L.riop_plan_create(ctypes.byref(d), None, None, ctypes.byref(h)) == -2
    assert b"3072" in L.riop_last_error()
    assert L.riop_plan_destroy(None) == 0


def test_product_does_not_reference_the_oracle():
    """The product package (library sources and binding) never uses the oracle."""
    pkg = os.path.join(ROOT, "paper_1307_4370_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read().lower()
                assert "oracle" not in text, os.path.join(dirpath, f)
