"""The C ABI library loads and exports every symbol include/sdpd.h declares;
host-side parameter checks reject bad input before touching the GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1707_04232_amd import sdpd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "sdpd.h")).read()
    return re.findall(r"^\s*(?:int|const char \*)\s*(sdpd_\w+)\(", hdr, re.M)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sdpd_build_cells", "sdpd_density", "sdpd_forces", "sdpd_fd_metropolis",
                     "sdpd_step"):
        assert required in names
    assert set(names) == set(sdpd.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = sdpd.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing


def test_abi_version_and_messages():
    L = sdpd.lib()
    assert L.sdpd_abi_version() == 8
    for rc in (0, -1, -2, -3, -4, -5, -6):
        assert L.sdpd_strerror(rc)
    assert L.sdpd_strerror(-99) == b"unknown status"


def test_struct_layout_matches_header(tmp_path):
    # compile the real header with gcc and compare sizes and offsets
    src = tmp_path / "layout.c"
    fields = [("sdpd_params", f) for f, _ in sdpd._Params._fields_] + \
             [("sdpd_state", f) for f, _ in sdpd._State._fields_] + \
             [("sdpd_stats", f) for f, _ in sdpd._Stats._fields_] + \
             [("sdpd_tuning", f) for f, _ in sdpd._Tuning._fields_] + \
             [("sdpd_cotangent", f) for f, _ in sdpd._Cotangent._fields_] + \
             [("sdpd_gradient", f) for f, _ in sdpd._Gradient._fields_]
    body = "\n".join(f'printf("%zu\\n", offsetof({t}, {f}));' for t, f in fields)
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"sdpd.h\"\nint main(void){\n"
                   + body + '\nprintf("%zu %zu %zu %zu %zu %zu\\n", sizeof(sdpd_params),'
                   ' sizeof(sdpd_state), sizeof(sdpd_stats), sizeof(sdpd_tuning),'
                   ' sizeof(sdpd_cotangent), sizeof(sdpd_gradient));\nreturn 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    want = [getattr(sdpd._Params, f).offset for f, _ in sdpd._Params._fields_] + \
           [getattr(sdpd._State, f).offset for f, _ in sdpd._State._fields_] + \
           [getattr(sdpd._Stats, f).offset for f, _ in sdpd._Stats._fields_] + \
           [getattr(sdpd._Tuning, f).offset for f, _ in sdpd._Tuning._fields_] + \
           [getattr(sdpd._Cotangent, f).offset for f, _ in sdpd._Cotangent._fields_] + \
           [getattr(sdpd._Gradient, f).offset for f, _ in sdpd._Gradient._fields_] + \
           [C.sizeof(sdpd._Params), C.sizeof(sdpd._State), C.sizeof(sdpd._Stats),
            C.sizeof(sdpd._Tuning), C.sizeof(sdpd._Cotangent), C.sizeof(sdpd._Gradient)]
    assert got == want


BAD = [
    dict(Cv=0.4),                      # Cv <= kB / 2 makes d_ij >= 1
    dict(zeta=2.0),                    # zeta >= 5 eta / 3
    dict(eta=0.0),
    dict(box=9.0),                     # fewer than 4 cells
    dict(ncell=(5, 4, 4)),             # odd cell count
    dict(ncell=(6, 4, 4)),             # cells smaller than h
    dict(cell_cap=65),
    dict(cell_cap=0),
    dict(fd=7),
    dict(kernel=3),
    dict(fd_every=0),
    dict(dt=-1.0),
    dict(A=-1.0),                      # A = 0 is the default, A < 0 is refused
    dict(n=-1),
    dict(prec=2),
]


@pytest.mark.parametrize("bad", BAD)
def test_create_rejects_bad_parameters_on_host(bad):
    kw = dict(n=1000, box=10.0)
    kw.update(bad)
    p = sdpd.SdpdParams(**kw)
    h = C.c_void_p()
    assert sdpd.lib().sdpd_create(C.byref(p.c()), None, C.byref(h)) == sdpd.EINVAL
    assert not h.value


def test_null_arguments_are_rejected():
    L = sdpd.lib()
    assert L.sdpd_create(None, None, None) == sdpd.EINVAL
    assert L.sdpd_destroy(None) == sdpd.EINVAL
    assert L.sdpd_sync(None) == sdpd.EINVAL
    assert L.sdpd_step(None, None, 0, 1, None) == sdpd.EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(sdpd, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sdpd, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        sdpd.lib()
