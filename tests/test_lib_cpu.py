"""Host-side checks of the C library (no GPU needed): it loads, exports every
entry point the public header declares, and the binding's tables agree."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "romhip.h")
LIB = os.path.join(ROOT, "paper_2605_28684_amd", "libromhip.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:rom_status|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_header():
    from paper_2605_28684_amd import romhip
    assert set(declared_functions()) == set(romhip.SYMBOLS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_config_struct_layout_matches_header():
    from paper_2605_28684_amd import romhip
    # 11 int32 + 2 pointers + 4 int32 + ... : the binding's struct must match the C layout
    src = open(HEADER).read()
    body = src[src.index("typedef struct {"):src.index("} rom_config;")]
    fields = re.findall(r"(int32_t|double|const int64_t\*|const double\*)\s+([\w, ]+);", body)
    c_names = []
    for _, names in fields:
        c_names += [x.strip() for x in names.split(",")]
    py_names = [f[0].rstrip("_") for f in romhip.rom_config._fields_]
    assert c_names == py_names
