"""The GPU library and its binding share no code with the oracle: nothing under the
package or the C header loads anything from oracle/, and the oracle loads nothing from the
package except the seeded input generators (synth.py, which holds none of the method's
arithmetic)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1806_10550_amd")


def _sources(top, exts):
    for d, _, files in os.walk(top):
        if "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_product_never_loads_the_oracle():
    pat = re.compile(r"^\s*(from\s+oracle|import\s+oracle)|liboracle|oracle/", re.M)
    files = list(_sources(PKG, (".py", ".hip", ".h", ".cpp"))) + [os.path.join(ROOT, "include", "thinfilm.h")]
    assert files
    for p in files:
        with open(p) as f:
            assert not pat.search(f.read()), p


def test_oracle_loads_only_the_input_generators_from_the_package():
    allowed = {"synth"}
    pat = re.compile(r"paper_1806_10550_amd(?:\.(\w+)|\s+import\s+(\w+))")
    for p in _sources(os.path.join(ROOT, "oracle"), (".py", ".c", ".h")):
        with open(p) as f:
            for a, b in pat.findall(f.read()):
                assert (a or b) in allowed, (p, a or b)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """With the HIP library absent the binding raises; there is no fallback path."""
    import pytest

    from paper_1806_10550_amd import lib as L
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libthinfilm.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        L.lib()
    with pytest.raises(RuntimeError, match="not built"):
        L.Grid(8, 8, 0.5)
