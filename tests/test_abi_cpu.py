"""Host-side checks of the C ABI (no GPU needed): the built library loads and
exports every entry point include/rf.h declares; the binding's structures
match the header's layout."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_12894_amd", "librf.so")
HEADER = os.path.join(ROOT, "include", "rf.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:rf_status|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        subprocess.run([os.path.join(ROOT, "paper_2511_12894_amd", "build_lib.sh")], check=True)
    return ctypes.CDLL(LIB)


def test_header_declares_the_four_calls():
    names = _declared_functions()
    for n in ("mf_ref_snr", "ratio_kernel_build", "snr_reconstruct", "snr_peaks"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    for name in _declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_binding_lists_every_declared_symbol():
    from paper_2511_12894_amd import rf
    assert sorted(rf.EXPORTED) == _declared_functions()


def test_struct_layouts():
    from paper_2511_12894_amd import rf
    assert ctypes.sizeof(rf.RfGrid) == 48
    assert ctypes.sizeof(rf.RfTmpl) == 16
    assert ctypes.sizeof(rf.RfPeak) == 8
    assert ctypes.sizeof(rf.RfTrigger) == 20


def test_struct_offsets_match_the_header(tmp_path):
    """Size and every field offset of each binding structure equal what a C
    compiler makes of include/rf.h."""
    from paper_2511_12894_amd import rf
    pairs = [("rf_grid", rf.RfGrid), ("rf_tmpl", rf.RfTmpl), ("rf_peak", rf.RfPeak),
             ("rf_trigger", rf.RfTrigger), ("rf_peak_args", rf.RfPeakArgs), ("rf_batch_tuning", rf.RfBatchTuning)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for cname, cls in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])


def test_null_context_is_rejected_without_gpu(lib):
    lib.mf_ref_snr.restype = ctypes.c_int
    assert lib.mf_ref_snr(None, None, None, None, None, 0, None, None) == 1   # RF_E_INVAL
    lib.rf_ctx_create.restype = ctypes.c_int
    assert lib.rf_ctx_create(0, None, None) == 1
    # kernel-set files: a null context is rejected before any file or device access
    lib.rf_kernels_save.restype = ctypes.c_int
    lib.rf_kernels_load.restype = ctypes.c_int
    assert lib.rf_kernels_save(None, None, b"/nonexistent/x") == 1
    out = ctypes.c_void_p(7)
    assert lib.rf_kernels_load(None, b"/nonexistent/x", ctypes.byref(out)) == 1
    assert out.value is None
