"""Host-side helpers of bench.py (no GPU): the leaf-depth walk over the
library's tree layout, and the rocprofv3 summaries written to profiles/."""
import csv
import os

import numpy as np

import bench


def _karras_tree(keys):
    """Binary radix tree over sorted distinct keys, laid out as the library
    lays it out: node [l, r] split at g (the last position whose common
    prefix with key l is longer than that of keys l and r) is number r when
    it is a left child and l when a right child, the root number 0; each
    record holds its left child (leaf g with the top bit, or node g) and its
    rope (leaf or node r+1, -1 after the last leaf).  Returns the records as
    float32 [n-1, 8] and the depth of the deepest leaf, found by recursion."""
    n = len(keys)
    rec = np.zeros((n - 1, 8), dtype=np.int32)

    def clz(x):
        return 64 - int(x).bit_length()

    def build(l, r, number, depth):
        if l == r:
            return depth
        d = clz(keys[l] ^ keys[r])
        g = max(i for i in range(l, r) if clz(keys[l] ^ keys[i]) > d)
        rec[number, 3] = (g | 0x80000000) - (1 << 32) if g == l else g
        rec[number, 7] = -1 if r == n - 1 else r + 1
        a = build(l, g, g, depth + 1)
        b = build(g + 1, r, g + 1, depth + 1)
        return max(a, b)

    deepest = build(0, n - 1, 0, 1)
    return rec.view(np.float32), deepest


def test_leaf_depth_matches_recursion():
    rng = np.random.default_rng(5)
    for n in (2, 3, 17, 200, 1000):
        keys = np.unique(rng.integers(0, 1 << 40, size=n * 2, dtype=np.int64))[:n]
        keys = sorted(int(k) for k in keys)
        rec, deepest = _karras_tree(keys)
        assert bench.leaf_depth(rec, 0, len(keys)) == deepest
    # a chain: keys 1, 2, 4, 8, ... give the deepest possible tree
    keys = [1 << i for i in range(30)]
    rec, deepest = _karras_tree(keys)
    assert deepest == 30
    assert bench.leaf_depth(rec, 0, 30) == 30
    assert bench.leaf_depth(np.zeros((1, 8), np.float32), 0, 1) == 1


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_trace_summary(tmp_path):
    d = tmp_path / "trace"
    _write(str(d / "host" / "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
            "StdDev"],
           [["k_pairs<0>", 4, 2_800_000, 700_000, 60.0, 1, 1, 0],
            ["k_onesweep<false, 16>", 32, 2_000_000, 62_500, 40.0, 1, 1, 0]])
    rows = [["k_pairs<0>", 0, 700_000]] * 4 + [["k_onesweep<false, 16>", 0, 7_000]] * 16 + \
           [["k_onesweep<false, 16>", 0, 118_000]] * 16
    _write(str(d / "host" / "run_kernel_trace.csv"),
           ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    out = tmp_path / "trace_x.txt"
    bench.summarize_trace(str(d), "x", "cmd", "line", str(out))
    text = out.read_text()
    assert "k_pairs<0>" in text and "700.00" in text
    assert "k_onesweep<false, 16>: 16 of 32 launches did work, avg 118.00 us" in text


def test_pmc_summary(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    gib_kib = (1 << 30) / 1024
    _write(str(tmp_path / "cf" / "run_counter_collection.csv"), hdr,
           [[1, "copy", "FETCH_SIZE", gib_kib / 2]])
    _write(str(tmp_path / "cw" / "run_counter_collection.csv"), hdr,
           [[1, "fill", "WRITE_SIZE", gib_kib], [2, "copy", "WRITE_SIZE", gib_kib]])
    _write(str(tmp_path / "f" / "run_counter_collection.csv"), hdr,
           [[1, "k_pairs<0>", "FETCH_SIZE", 1000.0], [2, "k_pairs<0>", "FETCH_SIZE", 1000.0]])
    _write(str(tmp_path / "w" / "run_counter_collection.csv"), hdr,
           [[1, "k_pairs<0>", "WRITE_SIZE", 100.0], [2, "k_pairs<0>", "WRITE_SIZE", 100.0]])
    bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                        str(tmp_path / "cw"), "x", 1000, ["a", "b"], ("pairs",),
                        str(tmp_path))
    vals = dict(line.split(": ", 1) for line in
                (tmp_path / "pmc_k_pairs_x.txt").read_text().splitlines()
                if ": " in line and not line.startswith("#"))
    # fetch counts half the bytes, write all of them
    assert int(vals["hbm_bytes_per_launch"]) == 1000 * 1024 * 2 + 100 * 1024
    assert vals["source_sha256"] == bench.source_sha("pairs")


def test_short_kernel_names():
    assert bench._short("void dbx::(anonymous namespace)::k_onesweep<false, 16>(unsigned long*, "
                        "unsigned int)") == "k_onesweep<false, 16>"
    assert bench._short("dbx::(anonymous namespace)::k_prep(unsigned int*, unsigned long)") == \
        "k_prep"
    assert bench._short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"
