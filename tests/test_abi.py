"""Host-only checks of the C-ABI: every declared symbol is exported; argument checks fail cleanly."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(mrf_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    import paper_2310_05647_amd as m
    names = _declared()
    assert len(names) >= 8
    missing = [n for n in sorted(names) if not hasattr(m.lib, n)]
    assert not missing, missing


def test_library_was_built_from_these_sources():
    """The loaded libmrf.so carries the SHA-256 of the sources it was compiled from; it must be
    this tree's (a stale binary after a source change fails here, and in smoke())."""
    import paper_2310_05647_amd as m
    info = m.build_info()
    assert info["arch"] == "gfx950" and len(info["sources-sha256"]) == 64
    assert m.built_from_current_sources(), info


def test_status_strings_and_version():
    import paper_2310_05647_amd as m
    assert m.lib.mrf_status_string(0) == b"MRF_OK"
    assert m.lib.mrf_status_string(7) == b"MRF_NOT_SUPPORTED"
    assert m.lib.mrf_version() >= 100


def test_nufft_plan_rejects_bad_descriptors_before_touching_the_device():
    import paper_2310_05647_amd as m
    from paper_2310_05647_amd._lib import NufftDesc
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    cases = [(NufftDesc(64, 10, 100, 5, 2, 0), 7), (NufftDesc(64, 10, 100, 6, 3, 0), 7),
             (NufftDesc(48, 10, 100, 6, 2, 0), 2), (NufftDesc(64, 0, 100, 6, 2, 0), 1),
             (NufftDesc(64, 10, 100, 6, 2, 12), 1), (NufftDesc(512, 10, 100, 6, 2, 16), 2)]
    for desc, expect in cases:
        st = m.lib.mrf_nufft_plan_create(ctypes.byref(desc), fake, None, ctypes.byref(h))
        assert st == expect, (desc.n, desc.kb_width, st, m.lib.mrf_last_error())
        assert m.lib.mrf_last_error() != b""
    assert m.lib.mrf_nufft_plan_create(None, fake, None, ctypes.byref(h)) == 1


def test_ctypes_structs_match_the_header_layout(tmp_path):
    """Each ctypes mirror in the binding has the size and field offsets of its C struct, as a host
    C compiler lays out include/mrf.h."""
    import shutil
    import subprocess
    from paper_2310_05647_amd import _lib
    cc = shutil.which("gcc")
    if cc is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs gcc and the ROCm headers")
    pairs = [("mrf_nufft_desc", _lib.NufftDesc), ("mrf_recon_params", _lib.ReconParams),
             ("mrf_mlp_train_cfg", _lib.MlpTrainCfg), ("mrf_recon_stats", _lib.ReconStats)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mrf.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        a, b, v = ln.split()
        got[(a, b)] = int(v)
    for cname, py in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
