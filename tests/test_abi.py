"""Host-side checks of the C ABI (no GPU needed):

* libgbr.so loads and exports every function include/gbr.h declares, and the
  binding marshals exactly those names;
* pure host entry points (strerror, version) answer;
* the product package never imports the oracle.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = ""
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt += open(os.path.join(ROOT, "include", f)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gbr3?_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2305_00762_amd import gbr
    L = gbr.load()
    names = declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(gbr.SIGNATURES), set(names) ^ set(gbr.SIGNATURES)


def test_host_only_calls():
    from paper_2305_00762_amd import gbr
    assert gbr.strerror(gbr.GBR_ESTATE).startswith("non-finite")
    assert gbr.strerror(0) == "ok"
    assert "gfx950" in gbr.version()


def test_null_context_rejected():
    from paper_2305_00762_amd import gbr
    L = gbr.load()
    assert L.gbr_set_geometry(None, 0, 1, 0, 1, 0, 0) == gbr.GBR_EINVAL
    assert L.gbr_residual(None, None, None, None) == gbr.GBR_EINVAL
    assert L.gbr_rk_stage(None, 1, None, None, None, None, None) == gbr.GBR_EINVAL
    assert L.gbr_destroy(None) == gbr.GBR_OK


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2305_00762_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", src, re.M), f
                assert "meg7_oracle" not in src, f
