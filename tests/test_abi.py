"""CPU-side checks of the C interface: the built library loads and exports every
function that include/qax.h declares, and the binding declares the same set."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qax.h")
LIB = os.path.join(ROOT, "paper_2606_31380_amd", "libqax.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(qax_\w+)\s*\(", src)
    return sorted(set(n for n in names if not n.startswith("qax_status")))


def test_header_declares_entry_points():
    names = declared()
    assert "qax_pair_sum" in names and "qax_solve" in names and "qax_assemble_self" in names
    assert len(names) >= 15


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(qax_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_matches_header():
    from paper_2606_31380_amd import qax
    L = qax.lib()
    for n in declared():
        assert hasattr(L, n), n
    assert sorted(qax.EXPORTS) == declared()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no fallback: without the built library every entry point raises
    from paper_2606_31380_amd import qax
    monkeypatch.setattr(qax, "LIB_PATH", str(tmp_path / "libqax.so"))
    monkeypatch.setattr(qax, "_LIB", None)
    with pytest.raises(RuntimeError, match="not built"):
        qax.lib()
    with pytest.raises(RuntimeError, match="not built"):
        qax.qax_create(0, 0)
