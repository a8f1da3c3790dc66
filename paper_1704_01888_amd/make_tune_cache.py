"""Tune the sweep shapes of this GPU and write them as a cache file.

    python -m paper_1704_01888_amd.make_tune_cache [path]

For every lattice side with a choice of shapes up to 256 and the population
classes 1-3 (R_cap from 2^11 to 2^14, 2^14 to 2^17, above), `Context.tune`
times every shape on a run of R = 8000, 50000 or 200000 replicas (q = 10,
theta = 10) and keeps the fastest; the entries go to `path` (by default the
package's cache file beside this module, which `Context` loads when it is
created; lines of other architectures in it are kept).  Classes of 200000
replicas are skipped where a population buffer would exceed 16 GB.
"""
from __future__ import annotations

import json
import os
import sys

from . import Context, tune_cache_path

SIDES = (8, 12, 16, 20, 24, 32, 48, 64, 96, 128, 192, 256)
POPULATIONS = (8000, 50000, 200000)


def main(path: str | None = None) -> str:
    ctx = Context(0, tune_cache=False)
    path = path or tune_cache_path(ctx.device)
    for L in SIDES:
        for R in POPULATIONS:
            if R * L * L > 16 << 30:
                continue
            e = ctx.tune(L, 10, R)
            print(json.dumps({k: e[k] for k in ("L", "r_class", "lanes", "waves_per_block",
                                                "attempts_per_ns")}), flush=True)
    # this architecture's lines replace its old ones; other architectures' stay
    mine = path + ".new"
    ctx.tune_save(mine)
    arch = json.loads(open(mine).readline())["arch"] if os.path.getsize(mine) else None
    keep = []
    if os.path.exists(path):
        keep = [ln for ln in open(path) if ln.strip() and json.loads(ln)["arch"] != arch]
    with open(path, "w") as f:
        f.writelines(keep)
        f.writelines(open(mine))
    os.remove(mine)
    ctx.close()
    return path


if __name__ == "__main__":
    print(main(sys.argv[1] if len(sys.argv) > 1 else None), file=sys.stderr)
