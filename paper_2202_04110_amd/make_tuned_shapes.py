"""Writes the launch-shape table shipped with the package (tuned_shapes.json):
runs the library's autotuner (lbp_autotune: HIP-event timing of every
candidate launch shape and fused-iteration variant) on each benchmark
workload and records its choices.  Run on the target GPU:

    python -m paper_2202_04110_amd.make_tuned_shapes OUT.json

then copy OUT.json over paper_2202_04110_amd/tuned_shapes.json.  Shapes never
change results, only speed.
"""
from __future__ import annotations

import os
import sys

from . import lbp, tune
from . import workloads as W

# (graph, damping, temperature) of every benchmark workload
CASES = [
    (lambda: W.potts_grid(512, 5, seed=2), 0.5, 1.0),
    (lambda: W.potts_grid(2048, 5, seed=2), 0.5, 1.0),
    (lambda: W.ising_grid(32, seed=1), 0.5, 0.0),
    (lambda: W.rbm(784, 500, seed=3), 0.5, 0.0),
    (lambda: W.rbm(784, 500, seed=3), 0.5, 0.05),
    (lambda: W.deconv(seed=4), 0.5, 0.0),
    (lambda: W.triplet_grid(256, 3, seed=12), 0.5, 1.0),
]


def main(out: str, reps: int = 20) -> None:
    if os.path.exists(out):
        os.remove(out)
    ctx = lbp.Context(0)
    for make, d, T in CASES:
        spec = make()
        g = lbp.Graph(ctx, spec)
        r = tune.apply_or_tune(g, d, T, reps=reps, path=out, packaged=False)
        print("%s T=%g: %s, fused %s, shapes %s" % (spec.name, T, r["source"], r["fused"],
                                                    [(s["wpb"], s["swizzle"], s["fused_wpb"], s["fused_variant"])
                                                     for s in r["shapes"]]), flush=True)
        g.free()
    ctx.close()


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "tuned_shapes.new.json")
