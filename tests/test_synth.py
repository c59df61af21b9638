"""Seeded generators: reproducibility, the stated distributions, and the BF16
storage encoding (round to nearest even, checked against torch's conversion)."""

import numpy as np
import torch

import synth
from synth.pointmaps import config2_counts


def test_config0_reproducible_and_shaped():
    a, b = synth.config0(), synth.config0()
    assert a.n_pairs == 1 and a.n_points == 3072 and a.tau == 0.0
    for k in a.planes:
        assert a.planes[k].dtype == np.float32
        assert np.array_equal(a.planes[k], b.planes[k])
    p, q, c = a.decoded_pair(0)
    assert p[:, 2].min() >= 1 and p[:, 2].max() <= 6 and c.min() >= 1 and c.max() <= 5
    s, R, t = a.gt[0]
    resid = np.linalg.norm(s * p @ R.T + t - q, axis=1)
    assert (resid > 0.2).sum() >= 300          # ~10% outliers (a few land near their inlier)
    assert np.median(resid) < 0.03


def test_config1_valid_fraction():
    b = synth.config1(n_pairs=3)
    assert b.n_points == 3 * 392 * 518
    frac = (b.planes["c"] >= 1.5).mean()
    assert abs(frac - 0.883) < 0.01
    pz = b.planes["pz"]
    assert pz.min() >= 1.0 - 1e-6 and pz.max() <= 10.0 + 1e-5


def test_config2_counts_log_uniform():
    V, square = config2_counts()
    assert len(V) == 256 and V.min() >= 20000 and V.max() <= 400000
    lv = np.log(V)
    assert abs(lv.mean() - 0.5 * (np.log(2e4) + np.log(4e5))) < 0.15
    assert 0.35 < square.mean() < 0.65
    b = synth.config2(n_pairs=4)
    assert np.array_equal(b.counts(), V[:4])
    assert (b.planes["c"] >= 1.5).all()


def test_bf16_round_to_nearest_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=10000).astype(np.float32) * 10,
                        np.array([0.0, -0.0, 1.0, np.inf, -np.inf, 3.4e38, 1e-40], dtype=np.float32)])
    ours = synth.bf16_encode(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    # ties: mantissa exactly halfway rounds to even
    halfway = np.array([0x3F808000, 0x3F818000], dtype=np.uint32).view(np.float32)
    assert list(synth.bf16_encode(halfway)) == [0x3F80, 0x3F82]
    assert np.array_equal(synth.bf16_decode(ours)[:-1],
                          torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16).float().numpy()[:-1])


def test_posegraph_shape():
    E, T = synth.config4_graph(n_nodes=100, n_loops=10)
    assert E.shape == (109, 2) and T.shape == (100, 4, 4)
    loops = E[99:]
    assert (loops[:, 1] - loops[:, 0] >= 20).all() and len({tuple(e) for e in loops}) == 10
