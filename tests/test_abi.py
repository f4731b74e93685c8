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


def test_binding_checks_label_buffers_before_any_call():
    """A caller's `out` is checked before the library gets its bare pointer:
    int32, on the points' device, contiguous, at least n elements."""
    torch = pytest.importorskip("torch")
    dev = torch.device("cpu")  # the checks themselves need no GPU
    ok = torch.empty(10, dtype=torch.int32)
    assert dbx._labels_out(ok, 10, dev) is ok
    assert dbx._labels_out(None, 7, dev).shape == (7,)
    bad = [(torch.empty(10, dtype=torch.int64), TypeError),
           (np.empty(10, np.int32), TypeError),
           (torch.empty(9, dtype=torch.int32), ValueError),
           (torch.empty(20, dtype=torch.int32)[::2], ValueError)]
    for out, err in bad:
        with pytest.raises(err):
            dbx._labels_out(out, 10, dev)
    with pytest.raises(ValueError):  # another device
        dbx._labels_out(torch.empty(10, dtype=torch.int32), 10, torch.device("cuda", 0))


def test_binding_checks_offsets():
    np.testing.assert_array_equal(dbx._offsets([0, 3, 3, 10], 10), [0, 3, 3, 10])
    for off in ([1, 10], [0, 6, 5, 10], [0, 11], [0, 9], [], [[0, 10]]):
        with pytest.raises(ValueError):
            dbx._offsets(off, 10)


def test_server_checks_host_label_buffers():
    s = dbx.Server(slots=1, fake_us_per_mpoint=10.0)
    p = np.zeros((10, 3), np.float32)
    for out, err in [(np.empty(10, np.int64), TypeError), (np.empty(9, np.int32), ValueError),
                     (np.empty(20, np.int32)[::2], ValueError), ([0] * 10, TypeError)]:
        with pytest.raises(err):
            s.submit(p, 0.1, 2, out=out)
    ro = np.empty(10, np.int32)
    ro.flags.writeable = False
    with pytest.raises(ValueError):
        s.submit(p, 0.1, 2, out=ro)
    good = np.zeros(12, np.int32)
    t = s.submit(p, 0.1, 2, out=good)
    assert s.wait(t, 10.0) == 0
    assert (good[:10] == -1).all()
    s.close()


def test_noalloc_rejects_on_the_host():
    """The no-allocation entry point checks its arguments and its size limit
    before any device call: EINVAL as dbscan_cluster, ETOOBIG past the
    fixed array's maximum, labels untouched; n = 0 does nothing."""
    lib = dbx.load_library()
    buf = (ctypes.c_float * 16)()
    lab = (ctypes.c_int32 * 16)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    out = ctypes.cast(lab, ctypes.c_void_p)
    assert lib.dbscan_cluster_noalloc(None, 0, ctypes.c_float(1.0), 2, None, None) == 0
    assert lib.dbscan_cluster_noalloc(p, 5, ctypes.c_float(-1.0), 2, out, None) == -1
    assert lib.dbscan_cluster_noalloc(p, 5, ctypes.c_float(1.0), 0, out, None) == -1
    st = lib.dbscan_cluster_noalloc(p, dbx.NOALLOC_MAX_POINTS + 1, ctypes.c_float(1.0), 2, out,
                                    None)
    assert st == -5
    assert b"maximum" in lib.dbscan_last_error()
    assert list(lab) == [0] * 16
    # the fixed array holds the largest job it admits
    assert lib.dbscan_scratch_bytes(dbx.NOALLOC_MAX_POINTS, 5, 1) <= 102760448
