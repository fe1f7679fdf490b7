"""Write tests/golden/bfs_calibration.json from the input generator and the
CPU oracle alone (no GPU, nothing from the library).

Breadth-first exploration of the synthetic 16-process model (the non-random
state-vector workload standing in for the state-space sequences of Sec. 5.2
and Table 1): the initial state is visited first; at each level the
successors of the frontier, duplicates included, form one find-or-put batch
applied to the oracle set, and the keys the oracle reports new, in batch
order, are the next frontier.  Recorded per level and seed: the batch size,
the states new at that level, the visited count after it, and set digests
(oracle.set_digest) of the visited set and of the level's new states.

Run from the repository root:
    python tests/golden/make_bfs_calibration.py
Seven levels for seeds 1 and 2 take a few minutes and about 30 GB of memory
(the level-6 batch of seed 1 holds 715 M keys).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import Oracle, set_digest  # noqa: E402
from paper_1712_09494_amd.inputs import BfsModel  # noqa: E402

LEVELS = 7
COMMAND = "python tests/golden/make_bfs_calibration.py"
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bfs_calibration.json")


def explore(seed: int, levels: int = LEVELS) -> dict:
    model = BfsModel(seed)
    o = Oracle([model.initial_state])
    frontier = np.array([model.initial_state], dtype=np.uint64)
    rec = {"batch_sizes": [], "new_counts": [], "visited_after": [], "visited_digest": [], "new_digest": []}
    for level in range(levels):
        t0 = time.time()
        batch = model.successors(frontier)
        flags = o.find_or_put(batch)
        frontier = batch[flags == 1]
        rec["batch_sizes"].append(int(batch.size))
        del batch, flags
        rec["new_counts"].append(int(frontier.size))
        rec["visited_after"].append(o.size)
        rec["visited_digest"].append(set_digest(o.keys))
        rec["new_digest"].append(set_digest(frontier))
        print(f"seed {seed} level {level}: new {frontier.size}, visited {o.size} ({time.time() - t0:.1f} s)",
              flush=True)
    return rec


def main():
    out = {
        "what": "Synthetic 16-process model (4 bits per process, 2-4 local transitions per local state, "
                "4 pairwise synchronising actions), BFS from the all-zero state with the initial state "
                "already visited. Per level: the successor batch (duplicates included), the states new at "
                "that level, the visited count after find-or-put of the batch, and set digests "
                "(oracle.set_digest: count, sum and xor of two mixes of every member) of the visited set "
                "and of the level's new states.",
        "source": "Written by the command below, which calls only the input generator "
                  "(paper_1712_09494_amd.inputs.BfsModel) and the CPU oracle (oracle.Oracle). Stands in "
                  "for the paper's non-random state-space sequences (Sec. 5.2, Table 1), whose states "
                  "occur 5-8 times on average.",
        "command": COMMAND,
    }
    for seed in (1, 2):
        out[f"seed{seed}"] = explore(seed)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
