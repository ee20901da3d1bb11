"""Host-side checks of the C ABI library (no GPU needed, no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2110_04865_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(msf_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_library_is_built_for_gfx950():
    assert os.path.exists(pkg.SO_PATH), "run __graft_entry__.build() first"
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", pkg.SO_PATH], capture_output=True,
                         text=True)
    if out.returncode == 0 and out.stdout.strip():
        assert "gfx950" in out.stdout


def test_exports_every_declared_symbol():
    L = ctypes.CDLL(pkg.SO_PATH)
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), f"{name} declared in msf.h but not exported"
    assert set(names) == set(pkg.EXPORTS)


def test_binding_loads_and_reports_version():
    L = pkg.lib()
    assert L.msf_version().decode().startswith("msf-gfx950")
    assert L.msf_last_error() is not None


def test_footprint_monotone():
    a = pkg.footprint(1000, 4000)
    b = pkg.footprint(2000, 4000)
    c = pkg.footprint(2000, 8000)
    assert 0 < a < b < c


def test_null_arguments_are_rejected_without_device():
    L = pkg.lib()
    # NULL context: rejected before any device call
    cnt = ctypes.c_int64(-7)
    rc = L.msf_solve(None, 3, 1, None, None, 0, 0, None, ctypes.byref(cnt), None)
    assert rc == 1 and cnt.value == -7
    assert b"ctx" in L.msf_last_error()
    rc = L.msf_shortcut(None, 3, None, None)
    assert rc == 1
    rc = L.msf_shortcut_strategy(None, 3, None, pkg.SHORTCUT_FULL, 0.0, None)
    assert rc == 1


@pytest.mark.skipif(os.path.exists("/dev/kfd") and os.access("/dev/kfd", os.R_OK),
                    reason="a GPU is present")
def test_context_without_gpu_fails_cleanly():
    L = pkg.lib()
    h = ctypes.c_void_p()
    rc = L.msf_ctx_create(0, None, ctypes.byref(h))
    assert rc in (3, 1)  # MSF_EDEVICE (no device) or MSF_EINVAL
    assert not h.value


def test_stats_struct_matches_header(tmp_path):
    """The binding's msf_stats mirror has the header's size and field offsets
    (the library writes sizeof(msf_stats) bytes into it)."""
    fields = [f[0] for f in pkg.Stats._fields_]
    src = tmp_path / "layout.c"
    src.write_text(
        "#include <stddef.h>\n#include <stdio.h>\n#include \"msf.h\"\n"
        "int main(void) {\n"
        "  printf(\"size %zu\\n\", sizeof(msf_stats));\n"
        + "".join(f"  printf(\"{f} %zu\\n\", offsetof(msf_stats, {f}));\n" for f in fields)
        + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict((k, int(v)) for k, v in (ln.split() for ln in out.splitlines()))
    assert got["size"] == ctypes.sizeof(pkg.Stats)
    for f in fields:
        assert got[f] == getattr(pkg.Stats, f).offset, f


def test_binding_rejects_bad_device_tensors():
    """The binding checks every device tensor before its pointer reaches the
    library (placement, layout, element size, length); no GPU needed."""
    torch = pytest.importorskip("torch")
    import numpy as np

    with pytest.raises(pkg.MSFError, match="device tensor"):
        pkg._dev(np.zeros(4, np.int32), "p", 4, 4)
    with pytest.raises(pkg.MSFError, match="on the GPU"):
        pkg._dev(torch.zeros(4, dtype=torch.int32), "p", 4, 4)

    class FakeCuda:  # stands in for a GPU tensor on a machine without one
        __module__ = "torch.fake"

        def __init__(self, n, elem, contiguous=True):
            self.n, self.elem, self.c = n, elem, contiguous
            self.is_cuda = True
            self.dtype = f"{elem}-byte"

        def is_contiguous(self):
            return self.c

        def element_size(self):
            return self.elem

        def numel(self):
            return self.n

        def data_ptr(self):
            return 4096

    with pytest.raises(pkg.MSFError, match="contiguous"):
        pkg._dev(FakeCuda(8, 4, contiguous=False), "r", 8, 4)
    with pytest.raises(pkg.MSFError, match="8-byte"):
        pkg._dev(FakeCuda(8, 4), "r", 8, 8)
    with pytest.raises(pkg.MSFError, match="needs 9"):
        pkg._dev(FakeCuda(8, 8), "r", 9, 8)
    assert pkg._dev(FakeCuda(9, 8), "r", 9, 8).value == 4096
