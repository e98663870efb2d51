"""Write the golden fixtures of this directory.  Calls only oracle/ (FP64
oracle) and fieldgen/ (seeded inputs); no value comes from the GPU path.

  abc32.json        ABC flow on the 32^3 periodic grid (A=sqrt3, B=sqrt2, C=1),
                    16 seeds, h = 0.01, 200 steps: oracle end points and codes.
  turb24.json       a 24^3 turbulence block (+1 ghost layer, rank grid 3^3 at
                    (1,1,1)), 32 seeds, h = 0.5, 300 steps: end points, steps,
                    codes, outbox destinations.
Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import fieldgen as fg  # noqa: E402
import oracle  # noqa: E402


def abc_case():
    blk = fg.abc_block(32)
    seeds = fg.uniform_seeds(1, 16, (0, 0, 0), (2 * np.pi,) * 3)
    r = oracle.Field.from_block(blk).trace(seeds, float(np.float32(0.01)), 200, keep_verts=False)
    return dict(description="ABC 32^3 periodic FP32 nodes, h=float32(0.01), 200 steps (oracle, FP64)",
                seeds=seeds.tolist(), final_pos=r["final_pos"].tolist(), steps=r["steps"].tolist(),
                code=r["code"].tolist())


def turb_case():
    blk = fg.turbulence_block(2, edge=24, rank_grid=(3, 3, 3), rank_coord=(1, 1, 1))
    seeds = fg.uniform_seeds(2, 32, (0, 0, 0), (24, 24, 24), sub=5)
    r = oracle.Field.from_block(blk).trace(seeds, 0.5, 300, keep_verts=False)
    return dict(description="turbulence 24^3 + ghost FP32 nodes, h=0.5, 300 steps, rank grid 3^3 (oracle, FP64)",
                seeds=seeds.tolist(), final_pos=r["final_pos"].tolist(), steps=r["steps"].tolist(),
                code=r["code"].tolist(), out_dest=r["out_dest"].tolist())


if __name__ == "__main__":
    for name, fn in (("abc32.json", abc_case), ("turb24.json", turb_case)):
        with open(os.path.join(HERE, name), "w") as fh:
            json.dump(fn(), fh, indent=0)
        print("wrote", name)
