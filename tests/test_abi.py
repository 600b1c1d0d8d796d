"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and reports its identity and errors without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("cascade.h", "cascade_learned.h")]


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cs_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2606_12577_amd import cascade
    return cascade.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("cs_create", "cs_set_hierarchy", "cs_setup", "cs_vcycle", "cs_solve", "cs_get_smoother",
                 "cs_set_smoother", "cs_smooth", "cs_save_setup", "cs_load_setup"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2606_12577_amd import cascade
    names = declared_functions()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(cascade.SIGNATURES), "binding signatures must cover the header exactly"


def test_identity_and_status_strings(lib):
    assert lib.cs_abi_version() == 4
    assert lib.cs_status_string(0) == b"ok"
    assert lib.cs_status_string(-5) == b"improper colouring"
    assert lib.cs_status_string(12345) == b"unknown status"


def test_null_arguments_are_rejected(lib):
    assert lib.cs_create(None, 0, None) == -1
    assert lib.cs_setup(None, None) == -1
    assert lib.cs_vcycle(None, None, None, 1) == -1
    lib.cs_destroy(None)


def test_no_device_reports_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert lib.cs_create(ctypes.byref(h), 0, None) == -3
    assert b"no HIP device" in lib.cs_last_error(None)


def test_library_is_gfx950_only():
    """The shared object carries gfx950 code objects (checked by name in the
    offload bundle) and was built from this tree's sources."""
    path = os.path.join(ROOT, "paper_2606_12577_amd", "libcascade.so")
    data = open(path, "rb").read()
    assert b"gfx950" in data


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the C layout of the header:
    a host program compiled from include/cascade.h prints size and field
    offsets of cs_level, cs_options and cs_info (gcc, no GPU)."""
    import shutil
    import subprocess
    from paper_2606_12577_amd import cascade
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {name: getattr(cascade, name) for name in ("cs_level", "cs_options", "cs_info")}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "cascade.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
