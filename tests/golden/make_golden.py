"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Calls only ``oracle`` (and the seeded generators for inputs); nothing here
comes from the HIP path.  The paper prints no worked example with values
(its Figure 1 survives only as a caption), so the stored cases are oracle
results on seeded synthetic inputs.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import gen  # noqa: E402
import oracle  # noqa: E402


def main():
    n, e, w = gen.workload_er_4096()
    ids, cnt, tot = oracle.msf(n, e, w, oracle.W_U32)
    rounds = oracle.as_rounds(n, e, w, oracle.W_U32)
    out = dict(workload="Erdos-Renyi n=4096 m=32768 seed=1 uint32 weights",
               count=cnt, total_u64=int(tot[0]), id_sum=int(ids.sum()),
               first_ids=[int(x) for x in ids[:16]],
               hooks_per_round=[int(h) for h in rounds["hooks"]])
    with open(os.path.join(HERE, "er4096_seed1.json"), "w") as f:
        json.dump(out, f, indent=1)
    n, e, w = gen.grid(16, 16, 16, 0.05, seed=3)
    ids, cnt, tot = oracle.msf(n, e, w, oracle.W_U32)
    out = dict(workload="grid 16^3, 5% of edges dropped, seed=3, uint32 weights",
               count=cnt, total_u64=int(tot[0]), id_sum=int(ids.sum()))
    with open(os.path.join(HERE, "grid16_seed3.json"), "w") as f:
        json.dump(out, f, indent=1)
    n, e, w = gen.rmat(12, 16, seed=2)
    ids, cnt, tot = oracle.msf(n, e, w, oracle.W_F32)
    out = dict(workload="R-MAT scale 12 edge factor 16 seed=2 float32 weights",
               count=cnt, total_f64=tot[1], id_sum=int(ids.sum()))
    with open(os.path.join(HERE, "rmat12_seed2.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
