"""Writes bf16_quantisation.json: the pose difference between the FP64 oracle
run on FP32 inputs and on the same inputs rounded to BF16 (round to nearest
even), over the first 24 pairs of the batched workload (256 pairs,
log-uniform 20k-400k points). Only the oracle is called; the GPU tests take
twice these maxima as the BF16-storage bound against FP32 originals.

Usage: python tests/golden/make_bf16_bound.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import irls, metrics  # noqa: E402


def main(n_pairs=24):
    b32 = synth.config2(n_pairs=n_pairs)
    b16 = b32.to_bf16()
    errs = []
    for k in range(n_pairs):
        p, q, c = b32.decoded_pair(k)
        r32 = irls.irls_align(p, q, c, b32.tau, b32.delta, b32.iters)
        p, q, c = b16.decoded_pair(k)
        r16 = irls.irls_align(p, q, c, b16.tau, b16.delta, b16.iters)
        errs.append(metrics.pose_errors((r16["s"], r16["R"], r16["t"]), (r32["s"], r32["R"], r32["t"])))
        print(k, len(p), errs[-1], flush=True)
    e = np.array(errs)
    out = dict(pairs=n_pairs, workload="batched config, first pairs", rotation_rad_max=float(e[:, 0].max()),
               scale_rel_max=float(e[:, 1].max()), translation_rel_max=float(e[:, 2].max()),
               rotation_rad_median=float(np.median(e[:, 0])), scale_rel_median=float(np.median(e[:, 1])),
               translation_rel_median=float(np.median(e[:, 2])))
    with open(os.path.join(HERE, "bf16_quantisation.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
