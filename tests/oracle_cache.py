"""Cached oracle results for full-size parity tests.

TEST INFRASTRUCTURE.  Every value stored here is computed by the FP64 direct
sum of eq. greenSum (``oracle.direct``) on inputs from ``workloads``; nothing
comes from the GPU library.  The arrays are written to ``tests/oracle_data/``
(not version-controlled) the first time a test asks for them and reused while
the generator and oracle sources are unchanged (their hash is part of the file
name).  Run ``python tests/oracle_cache.py`` to fill the cache ahead of time.
"""

from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CACHE = os.path.join(HERE, "oracle_data")


def _inputs_hash() -> str:
    h = hashlib.sha256()
    for rel in ("workloads/generators.py", "oracle/direct.c", "oracle/direct.py"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def full_direct(name: str, self_mode: int = 0) -> np.ndarray:
    """P at every target of workload `name` from the FP64 direct-sum oracle (cached)."""
    from oracle import direct
    from workloads import generators as G

    os.makedirs(CACHE, exist_ok=True)
    path = os.path.join(CACHE, f"{name}_self{self_mode}_{_inputs_hash()}.npy")
    if os.path.exists(path):
        return np.load(path)
    w = G.workload(name)
    ref = direct.direct_grid(w["f"], w["grid"].h, w["tx"], w["ty"], self_mode=self_mode)
    tmp = path + ".tmp.npy"
    np.save(tmp, ref)
    os.replace(tmp, path)
    return ref


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["vortex512"]:
        r = full_direct(nm)
        print(nm, r.shape, float(np.abs(r).max()))
