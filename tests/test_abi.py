"""The C-ABI library loads on the CPU and exports every function include/sqrtba.h declares (no GPU calls)."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sqrtba.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sqrtba_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_steps_of_the_method():
    names = declared_functions()
    for step in ["set_cameras", "set_landmarks", "set_observations", "linearize", "marginalize", "damp",
                 "solve", "back_substitute", "update", "commit", "lm_solve"]:
        assert f"sqrtba_{step}" in names


def test_library_exports_every_declared_symbol():
    import paper_2103_01843_amd as pkg

    lib = pkg.lib()  # loads; raises ImportError if the build is missing
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert sorted(pkg.EXPORTED) == names
    assert lib.sqrtba_version() >= 1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2103_01843_amd.sqrtba as s

    monkeypatch.setattr(s, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(s, "_lib", None)
    with pytest.raises(ImportError):
        s.lib()
