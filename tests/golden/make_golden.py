"""Writes oracle_small.json: summary values of the FP64 oracle on the small camera-space workload.

Calls only the oracle and the seeded input generator.  The stored values guard
the oracle against unintended changes; any deliberate change to its arithmetic
regenerates this file in the same commit and names the passage that justifies it.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle  # noqa: E402
from paper_2605_17855_amd import scenes  # noqa: E402


def summary():
    sc, cam = scenes.small_camera_space()
    out = oracle.render(sc, cam)
    rec = out["records"]
    lr = {str(g): oracle.load_reduction(rec, cam, g) for g in (2, 4)}
    return {
        "workload": "4096 Gaussians, 128x128, SH degree 0, seed 1",
        "visible": int(rec["visible"].sum()),
        "tile_entries": int(out["start"][-1]),
        "e_pix": int(out["e_pix"]),
        "image_channel_sums": [float(out["image"][c].sum()) for c in range(3)],
        "tfinal_sum": float(out["tfinal"].sum()),
        "ambiguous_pixels": int((out["ambiguous"] != 0).sum()),
        "load_reduction": {k: {"n_total": v[0], "n_group": v[1]} for k, v in lr.items()},
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_small.json"), "w") as f:
        json.dump(summary(), f, indent=1)
        f.write("\n")
