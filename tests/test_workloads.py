"""Seeded workload generators: determinism, neutrality and shapes."""
import numpy as np

from workloads import config1, config2, config3, config5, small_box, small_periodic, config4


def test_deterministic():
    a, b = config2(), config2()
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.boxes, b.boxes)
    assert np.array_equal(a.density.D[0], b.density.D[0])


def test_shapes_and_neutrality():
    c1 = config1()
    assert c1.K == 41 and c1.N(0) == 128 and c1.pos.tolist() == [[0.0, 0.0, 0.0]]
    c2 = config2()
    assert c2.K == 384 and c2.N(1) == 4096 and c2.Z.sum() == 0 and c2.boxes.shape == (16, 6)
    assert np.all(c2.boxes[:, :3] + c2.boxes[:, 3:] <= 4096)
    c3 = config3()
    assert c3.K == 64 * 60 and c3.N(2) == 256 and c3.Z.sum() == 0
    assert set(np.unique(c3.Z)) <= {-2.0, -1.0, 1.0, 2.0}
    c5 = config5()
    assert c5.Z.sum() == 0 and c5.M0 == 64
    for s in (c1, c2, c3, c5):
        assert np.all(s.pos >= -0.5 * s.b) and np.all(s.pos < 0.5 * s.b)


def test_small_generators():
    s = small_box(3)
    assert s.Z.sum() == 0 and len(s.boxes) == 3
    p = small_periodic(4)
    assert p.Z.sum() == 0 and p.periodic


def test_config4_population():
    systems = config4(count=24)
    assert len(systems) == 24
    for s in systems:
        assert 4 <= s.L[0] <= 48 and s.n in (64, 96, 128, 192, 256) and 1 <= s.M0 <= 32
        assert 30 <= s.R <= 60
