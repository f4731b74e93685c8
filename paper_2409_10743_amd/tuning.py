"""Autotuner results kept in a JSON file, so that a workload is tuned once
per device and later runs reuse the options (Context.autotune(...,
cache=...)).  The key names the device, the kind of call, the input size
class (n rounded to a power of two: timings of neighbouring sizes pick the
same options) and the exact parameters that change the work (eps as the
binary32 value the library uses, minPts, algorithm; for batches the per-set
arrays).  Writes replace the file atomically (a temporary file in the same
folder, then os.replace), so a reader never sees half a file; an unreadable
or malformed file counts as empty and is rewritten by the next put."""
import hashlib
import json
import math
import os
import tempfile

import numpy as np


def size_class(n: int) -> int:
    """log2 of n rounded to the nearest integer (0 for n <= 1)."""
    return 0 if n <= 1 else int(round(math.log2(n)))


def plain_key(device: str, n: int, eps: float, min_pts: int, algorithm: str) -> str:
    e = float(np.float32(eps))
    return f"plain|{device}|n~2^{size_class(int(n))}|eps={e!r}|min_pts={int(min_pts)}|{algorithm}"


def batched_key(device: str, offsets, eps, min_pts) -> str:
    off = np.asarray(offsets, dtype=np.int64)
    e = np.ascontiguousarray(eps, dtype=np.float32)
    m = np.ascontiguousarray(min_pts, dtype=np.int32)
    h = hashlib.sha256(e.tobytes() + m.tobytes()).hexdigest()[:16]
    total = int(off[-1]) if off.size else 0
    return f"batched|{device}|sets={off.size - 1}|n~2^{size_class(total)}|params={h}"


class TuneCache:
    def __init__(self, path):
        self.path = os.fspath(path)

    def _load(self) -> dict:
        try:
            with open(self.path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            return {}
        return data if isinstance(data, dict) else {}

    def get(self, key: str):
        v = self._load().get(key)
        return dict(v) if isinstance(v, dict) else None

    def put(self, key: str, result: dict) -> None:
        data = self._load()
        data[key] = dict(result)
        folder = os.path.dirname(os.path.abspath(self.path))
        fd, tmp = tempfile.mkstemp(prefix=".tune-", suffix=".json", dir=folder)
        try:
            with os.fdopen(fd, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except BaseException:
            if os.path.exists(tmp):
                os.unlink(tmp)
            raise

    def __len__(self) -> int:
        return len(self._load())
