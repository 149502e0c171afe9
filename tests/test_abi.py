"""The C-ABI library loads on the host and exports every symbol the header
declares (no GPU needed: no compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:uvc_status|const char\*|void|int32_t)\s+(uvc_\w+)\s*\(", src, re.M)
    return names


def test_header_symbols_exported():
    from paper_2103_14137_amd import uvc
    L = uvc.lib()
    names = _declared()
    assert len(names) >= 11
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert L.uvc_version() >= 100
    assert L.uvc_last_error() is not None


def test_product_path_has_no_oracle_dependency():
    """Nothing in the package imports, loads or names the oracle."""
    pkg = os.path.join(ROOT, "paper_2103_14137_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                for pat in (r"^\s*(from|import)\s+oracle", r"liboracle", r"oracle\.(ref|exact|lp|mlp)"):
                    assert not re.search(pat, src, re.M), (os.path.join(dirpath, f), pat)
