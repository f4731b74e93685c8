"""The C-ABI library: it loads, exports every function include/ declares, and
rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2409_10743_amd as dbx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(dbscan_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = dbx.load_library()
    names = _declared()
    assert len(names) >= 15
    for name in sorted(names):
        assert hasattr(lib, name), f"{name} declared but not exported"


def test_version_and_strerror():
    lib = dbx.load_library()
    assert b"gfx950" in lib.dbscan_version()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.dbscan_strerror(code)


def test_phase_names():
    lib = dbx.load_library()
    names = [lib.dbscan_phase_name(k).decode() for k in range(len(dbx.PHASES))]
    assert tuple(names) == dbx.PHASES
    assert lib.dbscan_phase_name(len(dbx.PHASES)) is None


@pytest.mark.parametrize("n,eps,mp,null", [
    (-1, 1.0, 2, False), (5, float("nan"), 2, False), (5, float("inf"), 2, False),
    (5, -0.5, 2, False), (5, 1e20, 2, False), (5, 1.0, 0, False), (5, 1.0, -7, False),
    (5, 1.0, 2, True), (1 << 30, 1.0, 2, False)])
def test_invalid_arguments_rejected_on_the_host(n, eps, mp, null):
    lib = dbx.load_library()
    buf = (ctypes.c_float * 16)()
    lab = (ctypes.c_int32 * 16)()
    ptr = None if null else ctypes.cast(buf, ctypes.c_void_p)
    st = lib.dbscan_cluster(ptr, n, ctypes.c_float(eps), mp, ctypes.cast(lab, ctypes.c_void_p),
                            None)
    assert st == -1
    assert lib.dbscan_last_error()
    # labels untouched on EINVAL
    assert list(lab) == [0] * 16


def test_empty_input_is_ok_without_a_device():
    lib = dbx.load_library()
    assert lib.dbscan_cluster(None, 0, ctypes.c_float(1.0), 2, None, None) == 0
    assert lib.dbscan_cluster_host(None, 0, ctypes.c_float(1.0), 2, None) == 0


def test_scratch_bytes_linear_in_n():
    lib = dbx.load_library()
    a = lib.dbscan_scratch_bytes(1 << 20, 2, 1)
    b = lib.dbscan_scratch_bytes(1 << 21, 2, 1)
    assert 80 * (1 << 20) < a < 140 * (1 << 20)
    assert 1.9 < b / a < 2.1
    assert lib.dbscan_scratch_bytes(1 << 20, 5, 1) > a  # minPts > 2 keeps border state
    assert lib.dbscan_scratch_bytes(-1, 2, 1) == 0


def test_python_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        dbx.cluster(torch.zeros((4, 3)), 1.0, 2)
    assert np is not None


def test_python_structs_match_the_header(tmp_path):
    """The binding's ctypes structures have the header's layout: a C program
    built with the host compiler prints sizeof and every field offset."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"dbscan_options": dbx._Options, "dbscan_server_options": dbx._ServerOptions,
               "dbscan_serving_stats": dbx._ServingStats}
    lines = []
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"dbscan_mi355x.h\"\n"
                   "int main(void) {\n" + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True,
                                                          capture_output=True,
                                                          text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[f"{cname} size"]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, f"{cname}.{f}"
