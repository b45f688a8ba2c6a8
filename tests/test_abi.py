"""The C-ABI library loads, exports what include/nsplat.h declares, and rejects
bad arguments on the host before any device work (no GPU needed)."""
from __future__ import annotations

import ctypes
import subprocess

import numpy as np
import pytest

from paper_2606_31764_amd import _lib as L


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_exports_every_declared_symbol(lib):
    out = subprocess.check_output(["nm", "-D", "--defined-only", L.LIB_PATH]).decode()
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    declared = L.header_symbols()
    assert len(declared) >= 13
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert getattr(lib, s) is not None


def _ctx(lib):
    h = ctypes.c_void_p()
    lib.nsplat_create(ctypes.byref(h), 0)   # EHIP without a device, but the context exists
    assert h.value
    return h


class _Fake:
    """Host-side descriptor with non-NULL (never dereferenced) device pointers."""

    def __init__(self, n_curves=2, channels=3, hw=((64, 48),)):
        self.hw = np.ascontiguousarray(hw, np.int32)
        fake = ctypes.c_void_p(0x1000)
        self.curves = L.Curves(n_curves, channels, 16, 10, 0, 0, 0, *([fake] * 11))
        self.scenes = L.Scenes(len(self.hw), ctypes.c_void_p(self.hw.ctypes.data), fake, fake)
        self.params = L.Params(10, 0.5, 2, 1.5, 5, 3, 0.1, 1.0, 6.0, 0.99, 1e-6, 0.25, 4, 16, 64, 0, None)
        self.caps = L.Caps(1000, 4000, 100)


def _bufs(lib, f, ws_bytes=None):
    fake = ctypes.c_void_p(0x100000)
    need = lib.nsplat_workspace_size(ctypes.byref(f.curves), ctypes.byref(f.scenes), ctypes.byref(f.params),
                                     ctypes.byref(f.caps))
    return L.Buffers(fake, fake, fake, fake, fake, fake, need if ws_bytes is None else ws_bytes, f.caps), need


def test_workspace_and_tiles(lib):
    f = _Fake(hw=((64, 48), (100, 33)))
    assert lib.nsplat_num_tiles(ctypes.byref(f.scenes), 16) == 4 * 3 + 7 * 3
    assert lib.nsplat_num_tiles(ctypes.byref(f.scenes), 8) == 8 * 6 + 13 * 5
    b, need = _bufs(lib, f)
    assert need > 0 and need % 256 == 0


@pytest.mark.parametrize("mutate,code", [
    (lambda f: setattr(f.curves, "channels", 2), L.EINVAL),
    (lambda f: setattr(f.curves, "n_curves", -1), L.EINVAL),
    (lambda f: setattr(f.curves, "key_xy", None), L.EINVAL),
    (lambda f: setattr(f.params, "tile", 12), L.EINVAL),
    (lambda f: setattr(f.params, "batch", 0), L.EINVAL),
    (lambda f: setattr(f.params, "batch", 1000), L.EINVAL),
    (lambda f: setattr(f.params, "alpha_max", 1.0), L.EINVAL),
    (lambda f: setattr(f.params, "rho", 0.0), L.EINVAL),
    (lambda f: setattr(f.params, "h", 0.0), L.EINVAL),
    (lambda f: setattr(f.scenes, "n_scenes", 0), L.EINVAL),
    (lambda f: f.hw.__setitem__((0, 0), 0), L.EINVAL),
])
def test_host_validation_rejects(lib, mutate, code):
    h = _ctx(lib)
    f = _Fake()
    mutate(f)
    b, _ = _bufs(lib, _Fake())
    rc = lib.nsplat_sample(h, ctypes.byref(f.curves), ctypes.byref(f.scenes), ctypes.byref(f.params),
                           ctypes.byref(b), 0, None)
    assert rc == code
    assert lib.nsplat_last_error(h)
    lib.nsplat_destroy(h)


def test_small_workspace_and_null_context(lib):
    h = _ctx(lib)
    f = _Fake()
    b, need = _bufs(lib, f, ws_bytes=1024)
    for fn in (lib.nsplat_sample,):
        assert fn(h, ctypes.byref(f.curves), ctypes.byref(f.scenes), ctypes.byref(f.params), ctypes.byref(b), 0,
                  None) == L.ECAPACITY
    assert b"workspace" in lib.nsplat_last_error(h)
    assert lib.nsplat_bin(None, None, None, None, None, None) == L.EINVAL
    assert lib.nsplat_forward(h, ctypes.byref(f.curves), ctypes.byref(f.scenes), ctypes.byref(f.params),
                              ctypes.byref(_bufs(lib, f)[0]), None, None, None, 0, None) == L.EINVAL
    assert lib.nsplat_anneal_h(h, None, None, 0, 10, 8.0, 1.0, 0.1, 0.8, None) == L.EINVAL
    lib.nsplat_destroy(h)


def test_abi_version_matches_header(lib):
    import re
    txt = open(L.HEADER).read()
    v = int(re.search(r"#define NSPLAT_ABI_VERSION (\d+)", txt).group(1))
    assert L.ABI_VERSION == v
    assert lib.nsplat_abi_version() == v


def test_struct_layouts_match_header(tmp_path):
    # sizes and field offsets of the ctypes structures against the C compiler's
    # view of include/nsplat.h (a binding that misreads a structure hands the
    # library shifted device pointers)
    import os
    structs = {"nsplat_curves": L.Curves, "nsplat_scenes": L.Scenes, "nsplat_params": L.Params,
               "nsplat_caps": L.Caps, "nsplat_buffers": L.Buffers, "nsplat_grads": L.Grads, "nsplat_reg": L.Reg,
               "nsplat_values": L.Values, "nsplat_adam": L.Adam}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "nsplat.h"', "int main(void) {"]
    expect = []
    for cname, cls in structs.items():
        lines.append('  printf("%%zu\\n", sizeof(%s));' % cname)
        expect.append(ctypes.sizeof(cls))
        for f in cls._fields_:
            lines.append('  printf("%%zu\\n", offsetof(%s, %s));' % (cname, f[0]))
            expect.append(getattr(cls, f[0]).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(L.HEADER), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).decode().split()]
    assert got == expect


def test_binding_refuses_other_abi_version(lib, monkeypatch):
    # a library whose structure layout differs must not be driven at all
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "ABI_VERSION", L.ABI_VERSION + 1)
    with pytest.raises(RuntimeError, match="ABI version"):
        L.load()
