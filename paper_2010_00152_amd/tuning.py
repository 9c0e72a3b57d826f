"""Persisted table of autotuned launch configurations for batched runs.

A batched workload is keyed by its aggregate set and a coarse signature of
its instance sizes: the share of instances in each decade of row counts,
rounded to tenths.  The table maps a key to the launch configuration that
the library's autotuner (isa_tune_batch) found fastest on such a workload,
and the time it measured.  The file is JSON."""
from __future__ import annotations

import json
import math
import os


def signature(rows, aggs: int) -> str:
    dec = [0] * 10
    for n in rows:
        dec[min(9, int(math.log10(max(1, int(n)))))] += 1
    tot = max(1, len(rows))
    return "aggs=%d;decades=%s" % (aggs, ",".join(str(round(10 * c / tot)) for c in dec))


class TuningTable:
    def __init__(self, path: str | None = None):
        self.path = path
        self.entries = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def lookup(self, key: str):
        e = self.entries.get(key)
        return dict(e["config"]) if e else None

    def record(self, key: str, config: dict, ms: float):
        self.entries[key] = {"config": dict(config), "ms": ms}
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.entries, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
