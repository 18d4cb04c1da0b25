"""A persistent cache of autotuning choices (JSON), host side.

rom_autotune times the candidates of a tuning target on the device and keeps
the fastest for one handle; this cache remembers the choice across handles
and processes, keyed by what decides it: the target, the problem, the
precision, the problem size (total degrees of freedom, rounded down to a
power of two), the reduced dimension and the GPU architecture.  A cached
choice is applied with rom_set_tuning (no timing); a missing one is tuned and
stored.  No arithmetic of the method happens here.
"""
import json
import math
import os

from . import romhip as R

TARGETS = {R.TUNE_RESIDUAL: "residual", R.TUNE_DEIM_PASS: "deim_pass", R.TUNE_BT_PART: "bt_part"}


def device_arch():
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def cache_key(target, problem, precision, total_dof, r, arch):
    """Key of one choice: target|problem|precision|log2 bucket of the size|r|arch."""
    bucket = int(math.floor(math.log2(max(int(total_dof), 1))))
    return "%s|p%d|f%d|n2^%d|r%d|%s" % (TARGETS[target], int(problem), int(precision), bucket,
                                        int(r), arch)


class TuningCache:
    """Choices by key, stored as a JSON object in `path` (created on first save)."""

    def __init__(self, path):
        self.path = path
        self.entries = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
            if not isinstance(data, dict) or data.get("version") != 1:
                raise ValueError("not a tuning cache of this version: %s" % path)
            self.entries = {str(k): int(v) for k, v in data["choices"].items()}

    def save(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"version": 1, "choices": self.entries}, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def apply(self, handle, q=None, targets=(R.TUNE_RESIDUAL, R.TUNE_DEIM_PASS, R.TUNE_BT_PART),
              arch=None):
        """Set every target's choice on the handle: from the cache when present
        (and valid for the handle), else by rom_autotune, then stored.  Targets
        that need q are skipped without it; targets with one candidate are
        skipped.  Returns {target name: (choice, "cache" | "tuned")}."""
        arch = arch or device_arch()
        done = {}
        for t in targets:
            n = handle.set_tuning(t, -1)
            if n <= 1 or (q is None and t != R.TUNE_DEIM_PASS):
                continue
            key = cache_key(t, handle.cfg.problem, handle.precision, handle.total_dof, handle.r,
                            arch)
            c = self.entries.get(key)
            if c is not None and 0 <= c < n:
                handle.set_tuning(t, c)
                done[TARGETS[t]] = (c, "cache")
            else:
                c = handle.autotune(t, q)
                self.entries[key] = c
                done[TARGETS[t]] = (c, "tuned")
        self.save()
        return done
