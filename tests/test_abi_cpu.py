"""Host-side checks of the C ABI without a GPU: the library loads, exports every
function include/gs.h declares, the binding wraps each under the same name, and
the host-only layout call computes the documented offsets."""
import os
import re

import pytest

import scenegen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    return sorted(set(re.findall(r"^\s*(?:gs_status|void|int32_t|const char\*)\s+(gs_\w+)\s*\(", src, re.M)))


def test_header_declarations_match_binding():
    import paper_2503_13086_amd as gs
    declared = _declared()
    assert declared == sorted(gs.EXPORTS)
    for name in declared:
        assert callable(getattr(gs, name))


def test_library_exports_every_symbol():
    import ctypes
    import paper_2503_13086_amd as gs
    if not os.path.exists(gs.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(gs.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert gs.gs_abi_version() == 1


def test_layout_offsets():
    import paper_2503_13086_amd as gs
    if not os.path.exists(gs.LIB_PATH):
        pytest.skip("library not built")
    cams = [scenegen.camera(__import__("numpy").eye(3), [0, 0, 0], 10, 10, 5, 5, w, h) for w, h in
            [(100, 75), (16, 16), (1, 1), (1600, 1067)]]
    po, to = gs.gs_layout(cams, 16)
    assert po == [0, 7500, 7756, 7757, 7757 + 1600 * 1067]
    assert to == [0, 7 * 5, 7 * 5 + 1, 7 * 5 + 2, 7 * 5 + 2 + 100 * 67]
    with pytest.raises(gs.GsError):
        gs.gs_layout([], 16)


def test_product_path_does_not_import_oracle():
    """The package and its binding never import the oracle."""
    pkg = os.path.join(ROOT, "paper_2503_13086_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt, f
