"""The C ABI library loads, exports every entry point include/lo.h declares,
and the ctypes structures match the C layout (no device calls)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lo.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(lo_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lo_plan", "lo_plan_destroy", "lo_step", "lo_run", "lo_effective_H", "lo_backward",
                     "lo_status_string", "lo_last_diag", "lo_kinetic_table", "lo_set_coef", "lo_time_kernels"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1210_4090_amd import _lib
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in _lib.SIGNATURES, name


def test_library_exports_only_declared_c_symbols():
    """Helpers stay internal: every unmangled function the library exports is
    one the header declares."""
    from paper_1210_4090_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {f[2] for f in (line.split() for line in out.stdout.splitlines())
                if len(f) == 3 and f[1] == "T" and not f[2].startswith("_Z")}
    assert exported == set(declared_functions())


def test_status_strings():
    from paper_1210_4090_amd import _lib
    L = _lib.lib()
    for s in range(6):
        assert L.lo_status_string(s)
    assert L.lo_status_string(99) == b"unknown status"


def test_ctypes_layout_matches_c(tmp_path):
    """Compile a probe against include/lo.h with gcc and compare offsets."""
    from paper_1210_4090_amd._lib import LoDesc, LoPotential
    src = tmp_path / "probe.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "lo.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(lo_desc), offsetof(lo_desc, n),
         offsetof(lo_desc, period), offsetof(lo_desc, tau), offsetof(lo_desc, P), offsetof(lo_desc, kstar_tab),
         offsetof(lo_desc, kstar_half), offsetof(lo_desc, window), offsetof(lo_desc, method),
         offsetof(lo_desc, flags), offsetof(lo_desc, t0), sizeof(lo_potential));
  printf("%zu %zu %zu %zu %zu\n", offsetof(lo_potential, nmodes), offsetof(lo_potential, basis),
         offsetof(lo_potential, coef), offsetof(lo_potential, tcoef), offsetof(lo_potential, ntcoef));
  return 0; }
''')
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    a, b = subprocess.check_output([str(exe)]).decode().split("\n")[:2]
    c = [int(v) for v in a.split()]
    assert c == [ctypes.sizeof(LoDesc), LoDesc.n.offset, LoDesc.period.offset, LoDesc.tau.offset, LoDesc.P.offset,
                 LoDesc.kstar_tab.offset, LoDesc.kstar_half.offset, LoDesc.window.offset, LoDesc.method.offset,
                 LoDesc.flags.offset, LoDesc.t0.offset, ctypes.sizeof(LoPotential)]
    d = [int(v) for v in b.split()]
    assert d == [LoPotential.nmodes.offset, LoPotential.basis.offset, LoPotential.coef.offset,
                 LoPotential.tcoef.offset, LoPotential.ntcoef.offset]


def test_plan_rejects_bad_descriptors_without_touching_the_device():
    """Validation happens before any device allocation."""
    from paper_1210_4090_amd import _lib
    from paper_1210_4090_amd.lo import make_desc
    L = _lib.lib()
    h = ctypes.c_void_p()
    for d in (make_desc([2, 8], 0.1, [0, 0]), make_desc([8, 8], -1.0, [0, 0]),
              make_desc([8, 8], 0.1, [float("nan"), 0])):
        assert L.lo_plan(ctypes.byref(d), None, ctypes.byref(h)) == _lib.LO_ERR_INVALID
    d = make_desc([8], 0.1, [0.0])
    d.ndim = 4
    assert L.lo_plan(ctypes.byref(d), None, ctypes.byref(h)) == _lib.LO_ERR_INVALID
    assert L.lo_plan(None, None, ctypes.byref(h)) == _lib.LO_ERR_INVALID


def test_missing_library_fails_loudly():
    """Without the built HIP library the binding raises; there is no CPU
    fallback (run in a child process so the loaded library is untouched)."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1210_4090_amd import _lib\n"
        "_lib.LIB_PATH = '/nonexistent/liblo.so'\n"
        "try:\n"
        "    _lib.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised', 'missing' in str(e))\n"
        "else:\n"
        "    print('loaded')\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.stdout.strip() == "raised True", out.stdout + out.stderr


def test_noalloc_step_refuses_before_device_work():
    """lo_step_noalloc checks its descriptor before touching a device: a grid
    beyond the static array, or a caller's kinetic table, is refused (this
    runs without a GPU)."""
    from paper_1210_4090_amd import _lib
    from paper_1210_4090_amd.lo import make_desc
    import numpy as np
    L = _lib.lib()
    big = make_desc([2048, 2049], 0.01, [0.0, 0.0])
    st = L.lo_step_noalloc(ctypes.byref(big), None, ctypes.c_void_p(8), 0, None, None)
    assert st == _lib.LO_ERR_UNSUPPORTED
    keep = []
    tab = make_desc([64], 0.01, [0.0], kstar_tabs=[np.linspace(1.0, 0.0, 9) ** 2], keep=keep)
    st = L.lo_step_noalloc(ctypes.byref(tab), None, ctypes.c_void_p(8), 0, None, None)
    assert st == _lib.LO_ERR_UNSUPPORTED
    assert L.lo_step_noalloc(None, None, ctypes.c_void_p(8), 0, None, None) == _lib.LO_ERR_INVALID
    small = make_desc([2], 0.01, [0.0])
    assert L.lo_step_noalloc(ctypes.byref(small), None, ctypes.c_void_p(8), 0, None, None) == _lib.LO_ERR_INVALID
