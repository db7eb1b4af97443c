"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/irbe.h declares, and the Python mirror of irbe_config has the
layout of the C struct."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "irbe.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(irbe_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2204_13595_amd import irbe
    if not os.path.exists(irbe.LIB_PATH):
        from paper_2204_13595_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(irbe.LIB_PATH)
    names = _declared()
    assert "irbe_create" in names and "irbe_compute_forces_backward" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(irbe.EXPORTED)


def test_config_layout_matches_header():
    from paper_2204_13595_amd import irbe
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "irbe.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(irbe_config), offsetof(irbe_config, n_atoms),
         offsetof(irbe_config, p_shell), offsetof(irbe_config, seed), offsetof(irbe_config, capacity_hint),
         offsetof(irbe_config, skin), offsetof(irbe_config, lj_cut), offsetof(irbe_config, shell_entries));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(irbe_dyn_config), offsetof(irbe_dyn_config, n_atoms),
         offsetof(irbe_dyn_config, dt), offsetof(irbe_dyn_config, kT), offsetof(irbe_dyn_config, seed),
         offsetof(irbe_dyn_config, tau));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", f"-I{os.path.dirname(HEADER)}", c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    C = irbe.Config
    assert [int(x) for x in out[:8]] == [ctypes.sizeof(C), C.n_atoms.offset, C.p_shell.offset, C.seed.offset,
                                         C.capacity_hint.offset, C.skin.offset, C.lj_cut.offset,
                                         C.shell_entries.offset]
    D = irbe.DynConfig
    assert [int(x) for x in out[8:]] == [ctypes.sizeof(D), D.n_atoms.offset, D.dt.offset, D.kT.offset,
                                         D.seed.offset, D.tau.offset]


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2204_13595_amd import irbe
    saved = irbe._lib
    irbe._lib = None
    try:
        with pytest.raises(FileNotFoundError):
            irbe.load_library(str(tmp_path / "missing.so"))
    finally:
        irbe._lib = saved


def test_handle_requires_gpu():
    import torch
    from paper_2204_13595_amd import irbe
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        irbe.Handle(1536, 2.4834)


@pytest.mark.parametrize("entries", [7, 16, -1])
def test_bad_shell_entries_rejected_before_any_device_call(entries):
    """irbe_create validates the configuration before it touches a device: an
    unknown shell_entries value (0 and 32 are the valid ones) is IRBE_EINVAL."""
    from paper_2204_13595_amd import irbe
    if not os.path.exists(irbe.LIB_PATH):
        from paper_2204_13595_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(irbe.LIB_PATH)
    lib.irbe_create.argtypes = [ctypes.POINTER(irbe.Config), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.irbe_last_error.restype = ctypes.c_char_p
    lib.irbe_last_error.argtypes = [ctypes.c_void_p]
    cfg = irbe.Config(irbe.IRBE_ABI_VERSION, irbe.IRBE_MIXED_FP32, 1536, 2.4834, 3.0, 138.935458, 0.5, 1.2, 100,
                      100, 2, 0, 13595, 0.0, 0.0, 0.0, entries)
    h = ctypes.c_void_p()
    st = lib.irbe_create(ctypes.byref(cfg), None, ctypes.byref(h))
    assert st == -1 and not h.value
    assert b"shell_entries" in lib.irbe_last_error(None)
