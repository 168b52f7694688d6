"""Writes trellis_whole_video.json: the FP64 oracle's optima of the paper's
whole-video trellis (synth.paper_blocks(0) with its 50 models, the
benchmark's workload: M = 30 models against all 754 points of a 723-frame
video; Section 2.2, the loop bounds of Section 3.4), for
the first model with no closeness limit and the first four at T = 10.  Only
the oracle runs here (the literal recursion on lists holding the whole
video); the no-limit case takes a few minutes on one core.

    python tests/golden/make_trellis_whole_video.py
"""
import dataclasses
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1505_00581_amd import synth  # noqa: E402

CASES = ((0, [0]), (10, [0, 1, 2, 3]))  # (T, models)


def main():
    w = synth.paper_blocks(0, n_models=50)  # the benchmark's video (the scene depends on n_models)
    s = w.scenes[0]
    rows = []
    for T, models in CASES:
        p = dataclasses.replace(w.params, T=T)
        for q in models:
            r = oracle.match_trellis(w.models[q], s, p)
            rows.append(dict(T=T, model=q, energy=float(r["energy"][0]), energy_u=float(r["energy_u"][0]),
                             assign=[int(v) for v in r["assign"][0]]))
            print(f"T={T} model {q}: E = {rows[-1]['energy']:.12g}", flush=True)
    out = dict(workload="synth.paper_blocks(0, n_models=50): M = 30 models against all 754 points of a 723-frame video",
               source="oracle.match_trellis (FP64 literal recursion), written by make_trellis_whole_video.py",
               rows=rows)
    with open(os.path.join(HERE, "trellis_whole_video.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
