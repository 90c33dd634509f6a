"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/mpcd.h declares, its structs have the same layout in
C and in the binding, and calls that cannot reach a device fail cleanly."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpcd.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|void|const char\*)\s+(mpcd_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def m():
    from paper_2212_11878_amd import mpcd
    return mpcd


def test_exports_every_declared_function(m):
    names = _declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(m.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(m._SIGNATURES), set(names) ^ set(m._SIGNATURES)


def test_struct_layout_matches_header(m, tmp_path):
    structs = {
        "mpcd_box_desc": m.mpcd_box_desc,
        "mpcd_options": m.mpcd_options,
        "mpcd_observables": m.mpcd_observables,
        "mpcd_kernel_stat": m.mpcd_kernel_stat,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpcd.h"', "int main(void){"]
    for sname, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (sname, sname))
        for fname, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (sname, fname, sname, fname))
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for sname, cls in structs.items():
        assert int(out[sname]) == ctypes.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert int(out["%s.%s" % (sname, fname)]) == getattr(cls, fname).offset, (sname, fname)


def test_status_strings_and_version(m):
    assert m.mpcd_abi_version() == m.ABI_VERSION == 4
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert m.mpcd_strerror(code) and m.mpcd_strerror(code) != "unknown status"
    assert m.mpcd_strerror(12345) == "unknown status"


def test_null_arguments_rejected(m):
    lib = m._lib
    assert lib.mpcd_create(None, None) == m.MPCD_EINVAL
    assert lib.mpcd_step(None, 1) == m.MPCD_EINVAL
    assert lib.mpcd_release(None, 0) == m.MPCD_EINVAL
    assert lib.mpcd_observe(None, 0, None) == m.MPCD_EINVAL
    assert lib.mpcd_get_mass(None, 0, None) == m.MPCD_EINVAL
    assert lib.mpcd_get_vacf(None, 0, None, None, None, 0, None) == m.MPCD_EINVAL
    assert lib.mpcd_set_vacf(None, 0, None, 0, None, 0) == m.MPCD_EINVAL
    # the measurement copy checks its arguments before touching a device
    assert lib.mpcd_hbm_copy(None, None, 16, 0, None) == m.MPCD_EINVAL
    assert lib.mpcd_hbm_copy(ctypes.c_void_p(16), ctypes.c_void_p(32), 15, 0, None) == m.MPCD_EINVAL
    assert lib.mpcd_hbm_copy(ctypes.c_void_p(8), ctypes.c_void_p(32), 16, 0, None) == m.MPCD_EINVAL
    assert lib.mpcd_hbm_copy(ctypes.c_void_p(16), ctypes.c_void_p(32), 0, 0, None) == m.MPCD_OK
    lib.mpcd_destroy(None)


def test_create_without_device_fails_cleanly(m):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    opt = m.mpcd_options()
    rc, h = m.mpcd_create(opt)
    assert rc == m.MPCD_EDEVICE
    assert not h.value
    opt.binning = 7
    assert m.mpcd_create(opt)[0] == m.MPCD_EINVAL


def test_brick_edges_must_be_powers_of_two(m):
    """Options are checked before any device is touched: brick edges are 0
    (automatic) or powers of two in [2, 64]."""
    for edges, ok in (((0, 0, 0), True), ((8, 4, 4), True), ((2, 64, 16), True), ((6, 4, 4), False),
                      ((8, 8, 128), False), ((1, 8, 8), False), ((8, 3, 8), False)):
        opt = m.mpcd_options()
        for i in range(3):
            opt.brick[i] = edges[i]
        rc, h = m.mpcd_create(opt)
        if rc == m.MPCD_OK:
            m._lib.mpcd_destroy(h)
        if ok:
            assert rc != m.MPCD_EINVAL, edges
        else:
            assert rc == m.MPCD_EINVAL, edges


def test_one_hip_runtime_whatever_the_import_order():
    """The binding and PyTorch share one HIP runtime in the process, also when
    the binding is imported before torch."""
    code = ("import paper_2212_11878_amd.mpcd\n"
            "print(len(set(l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l)))\n")
    out = subprocess.run([__import__("sys").executable, "-c", code], cwd=ROOT, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


def _build_c_client(out_dir):
    """Compile tests/c_abi_client.c (C99, gcc) against include/mpcd.h and link
    it to the built libmpcd.so."""
    from paper_2212_11878_amd import mpcd
    exe = os.path.join(str(out_dir), "c_abi_client")
    libdir = os.path.dirname(mpcd.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-O2", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_client.c"), "-L", libdir, "-lmpcd",
                    "-Wl,-rpath," + libdir, "-lm", "-o", exe], check=True)
    return exe


def test_c_client_compiles_and_links(tmp_path):
    """The header is plain C99 and the library links from C alone; without a
    device the client stops at mpcd_create with MPCD_EDEVICE."""
    import torch
    exe = _build_c_client(tmp_path)
    if torch.cuda.is_available():
        return
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 77 and out.stdout.strip() == "no device", (out.returncode, out.stdout)
