"""Writes datagen/manifest.json: the sha256 of the exact bytes every
workload generator produces (float32 points, int64 set offsets), with the
numpy version that produced them.  The GPU side and the oracle both
regenerate their inputs in-process from these seeded generators; the
manifest pins those bytes, so a run on another machine (or numpy) can show
it saw the same input (datagen.check_manifest).

    python -m datagen.make_manifest            (from the repository root)
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import MANIFEST, input_digests


def main() -> None:
    doc = {"numpy": np.__version__, "sha256": input_digests()}
    with open(MANIFEST, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(doc, indent=1))


if __name__ == "__main__":
    main()
