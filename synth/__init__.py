"""Seeded synthetic workloads for dense Sim(3) alignment and the Sim(3) pose
graph. The same arrays feed the FP64 oracle and the HIP library; this package
holds no step of the method itself (no estimation, no solve), only data
synthesis: surfaces, unprojection, ground-truth similarities, noise, outliers,
and the BF16 storage encoding.

The paper's datasets (TUM-RGBD, 7-Scenes, Replica) and its feed-forward
network are not available; these inputs reproduce only their shapes: images
resized to a 518-pixel long side (Sec. IV-A, datasets) and submaps of 5
keyframes (hyperparameters).
"""

from .pointmaps import (Batch, bf16_decode, bf16_encode, config0, config1, config2,
                        config3, make_batch, pair_from_frames)
from .posegraph import config4_graph, random_walk

__all__ = ["Batch", "bf16_decode", "bf16_encode", "config0", "config1", "config2", "config3",
           "make_batch", "pair_from_frames", "config4_graph", "random_walk"]
