"""The C-ABI library loads and exports every function include/domdec.h declares (no GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "domdec.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    # "type name(" or "type* name(" at the start of a line (not "type (*member)(")
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+(?:\s+|\s*\*\s*)([a-z_0-9]+)\s*\(", text,
                       flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("domdec_init", "domdec_iterate", "sinkhorn_batch", "flow_update", "extract_plan"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2405_09400_amd as dd
    path = dd.lib_path()
    if not os.path.exists(path):
        pytest.fail("libdomdec.so is not built (run __graft_entry__.build())")
    L = dd.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(dd.binding.SYMBOLS) == _declared()


def test_strerror_without_context_is_safe():
    import paper_2405_09400_amd as dd
    assert isinstance(dd.lib().domdec_strerror(None, -1), bytes)
