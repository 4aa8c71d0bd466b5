"""The seeded input generators: reproducibility, shapes and the stated recipes."""

import numpy as np

import gen


def test_trefoil_recipe():
    g, e = gen.trefoil(256, seed=0)
    assert g.shape == (256, 3) and e.shape == (256, 2) and e.dtype == np.int32
    t = 2 * np.pi * np.arange(256) / 256
    clean = np.stack([np.sin(t) + 2 * np.sin(2 * t), np.cos(t) - 2 * np.cos(2 * t), -np.sin(3 * t)], 1)
    jit = g - clean
    assert abs(jit.std() - np.sqrt(1e-3)) < 0.003      # variance 1e-3
    g2, _ = gen.trefoil(256, seed=0)
    assert np.array_equal(g, g2)


def test_fourier_knot_reproducible_and_closed():
    g, e, tries = gen.fourier_knot(4096, seed=1)
    g2, _, _ = gen.fourier_knot(4096, seed=1)
    assert np.array_equal(g, g2) and tries >= 1
    assert np.array_equal(e[:, 1], np.roll(e[:, 0], -1))


def test_packing_instance_shapes():
    inst = gen.packing_batch(4, seed=3)
    for g, e, sizes in inst:
        assert len(g) == sizes.sum() == len(e)
        assert 200 * 0.9 <= len(e) <= 8000 * 1.1 + 32 * 8
        assert (sizes >= 8).all() and 1 <= len(sizes) <= 32
        assert np.linalg.norm(g - 0.5, axis=1).min() > 0.25


def test_round_to_f32():
    x = np.array([[0.1, 1 / 3, np.pi]])
    y = gen.round_to_f32(x)
    assert y.dtype == np.float64 and np.array_equal(y.astype(np.float32).astype(np.float64), y)
