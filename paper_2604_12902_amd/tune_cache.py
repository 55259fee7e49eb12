"""Autotune cache: scheduling knobs chosen for a (device, batch shape, library
code) key, kept in a JSON file so that a run on a known shape does not search
again.

A key names the device architecture and compute-unit count, the batch (its
name, machine count, budget and the SHA-256 of its packed inputs) and the
SHA-256 of the library's HIP sources with comments and whitespace removed: an
entry outlives edits to comments but not to code, and a different device or
batch never reuses it.
"""
from __future__ import annotations

import json
import os

from . import counters

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "tune_cache.json")
SOURCES = (os.path.join(HERE, "csrc", "rasp_kernels.hip"), os.path.join(HERE, "csrc", "rasp_runtime.hip"))


def library_sha256() -> str:
    text = []
    for p in SOURCES:
        with open(p, encoding="utf-8") as f:
            text.append(f.read())
    return counters.code_sha256("\n".join(text))


def make_key(arch: str, cus: int, batch, budget: int, extra: str = "") -> str:
    return json.dumps({"arch": arch, "cus": int(cus), "batch": batch.name, "num_vms": int(batch.N),
                       "budget": int(budget), "inputs_sha256": batch.sha256(),
                       "library_sha256": library_sha256(), "extra": extra}, sort_keys=True)


def _read(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def get(key: str, path: str = PATH):
    """The knobs stored under `key`, or None."""
    return _read(path).get(key)


def put(key: str, value: dict, path: str = PATH) -> None:
    """Store `value` under `key`, dropping entries of older library code."""
    t = _read(path)
    sha = json.loads(key)["library_sha256"]
    t = {k: v for k, v in t.items() if json.loads(k).get("library_sha256") == sha}
    t[key] = value
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
