"""The C-ABI library loads and exports every entry point its header declares (CPU, no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "emshower.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ("init_physics_tables", "init_geometry", "transport_events", "tally_read"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2203_09467_amd as ems
    lib = ctypes.CDLL(ems.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(ems.EXPORTED) == _declared()


def test_workspace_size_and_argument_errors_without_gpu():
    import paper_2203_09467_amd as ems
    cfg = ems.Config(1 << 16, 128, 100, 1 << 16, 1, ems.EMS_FP64, 0.0, 0, 0)
    n = ems.workspace_bytes(cfg)
    # two pool buffers of 88 B per slot dominate
    assert n >= 2 * 88 * (1 << 16)
    bad = ems.Config(8, 128, 100, 1 << 16, 1, ems.EMS_FP64, 0.0, 0, 0)
    assert ems.workspace_bytes(bad) == 0
    h = ctypes.c_void_p()
    st = ems._lib.ems_create(ctypes.byref(cfg), None, n, ctypes.byref(h))
    assert st == -1 and not h.value
    assert b"workspace" in ems._lib.ems_last_error()
    # misaligned workspace pointer
    st = ems._lib.ems_create(ctypes.byref(cfg), ctypes.c_void_p(0x1001), n, ctypes.byref(h))
    assert st == -1
    # too small
    st = ems._lib.ems_create(ctypes.byref(cfg), ctypes.c_void_p(0x100000), n - 1, ctypes.byref(h))
    assert st == -3
    assert ems._lib.transport_events(None, None, 1, None, None) == -1


def test_product_package_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2203_09467_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt and "oracle.h" not in txt, f
