"""The C-ABI library loads and exports every entry point include/apic.h
declares; host-side argument checks work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apic.h")
LIB = os.path.join(ROOT, "paper_1603_06188_amd", "libapic.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apic_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1603_06188_amd.build import build_library
        build_library()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "apic_p2g" in names and "apic_step" in names and len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


def test_binding_mirrors_header():
    from paper_1603_06188_amd import binding
    assert sorted(binding.EXPORTED) == _declared()


def test_struct_layout_matches_c(tmp_path):
    from paper_1603_06188_amd import binding
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "apic.h"\n#include <stddef.h>\nint main(){printf("%zu %zu %zu %zu %zu %zu",'
                   'sizeof(apic_scene), sizeof(apic_params), sizeof(apic_particles), sizeof(apic_grid_desc),'
                   'offsetof(apic_scene, workspace), offsetof(apic_params, mu));}\n')
    exe = tmp_path / "sz"
    assert os.system(f"gcc -I {ROOT}/include {src} -o {exe}") == 0
    got = os.popen(str(exe)).read().split()
    want = [ctypes.sizeof(binding.ApicScene), ctypes.sizeof(binding.ApicParams), ctypes.sizeof(binding.ApicParticles),
            ctypes.sizeof(binding.ApicGridDesc), binding.ApicScene.workspace.offset, binding.ApicParams.mu.offset]
    assert [int(x) for x in got] == want


def test_host_validation_without_gpu():
    from paper_1603_06188_amd import binding as b
    g = b.ApicGridDesc()
    g.dim, g.degree, g.precision, g.options = 3, 2, b.APIC_F32, 0
    for a in range(3):
        g.cells[a] = 128
    g.dx = 1.0 / 128
    nbytes = b.apic_workspace_bytes(g, 2_097_152)
    # grid planes + shadow state dominate: at least 2M * 104 B
    assert nbytes > 2_097_152 * 104
    for field, value in (("dim", 4), ("degree", 1), ("precision", 7), ("options", 8)):
        old = getattr(g, field)
        setattr(g, field, value)
        with pytest.raises(b.ApicError) as e:
            b.apic_workspace_bytes(g, 10)
        assert e.value.code == -1
        setattr(g, field, old)
    g.cells[1] = 2000
    with pytest.raises(b.ApicError):
        b.apic_workspace_bytes(g, 10)
    g.cells[1] = 128
    with pytest.raises(b.ApicError):
        b.apic_workspace_bytes(g, -1)
    # a scene with no workspace is rejected before anything is enqueued
    s = b.ApicScene()
    s.grid = g
    rc = b._lib.apic_p2g(ctypes.byref(s), None)
    assert rc == -4 and "workspace" in b.apic_last_error()
