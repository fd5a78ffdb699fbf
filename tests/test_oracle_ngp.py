"""Pins of the hash-grid + MLP oracle F(X|Theta) (Sec. III-C)."""
import math

import numpy as np
import pytest

from oracle import ngp as N

SMALL = N.NgpConfig(levels=4, feat=2, log2_table=10, n_min=4, n_max=32, hidden=8, scale_max=0.05)


def test_level_resolutions_grow_geometrically_from_n_min_to_n_max():
    cfg = N.NgpConfig()
    r = [N.level_resolution(cfg, l) for l in range(cfg.levels)]
    assert r[0] == cfg.n_min and r[-1] in (cfg.n_max - 1, cfg.n_max)
    assert all(b > a for a, b in zip(r, r[1:]))
    b = math.exp(math.log(cfg.n_max / cfg.n_min) / (cfg.levels - 1))
    assert r[5] == math.floor(16 * b ** 5)


def test_dense_levels_are_exactly_those_that_fit_the_table():
    cfg = N.NgpConfig()   # 2^19 entries: dense while (N+1)^3 <= 524288, i.e. N <= 79
    for l in range(cfg.levels):
        n = N.level_resolution(cfg, l)
        assert N.dense_level(cfg, l) == (n <= 79)


def test_hash_uses_32_bit_wraparound_and_xor():
    cfg = N.NgpConfig()
    l = cfg.levels - 1
    assert not N.dense_level(cfg, l)
    v = np.array([[1, 2, 3], [0, 0, 0], [7, 0, 0], [0, 1, 0]])
    # 2 * 2654435761 = 5308871522 wraps to 1013904226; 3 * 805459861 = 2416379583 does not wrap
    expect = [(1 ^ 1013904226 ^ 2416379583) % (1 << 19), 0, 7, 2654435761 % (1 << 19)]
    assert list(N.vertex_index(cfg, l, v)) == expect


def test_dense_index_is_row_major_in_x_then_y_then_z():
    n = N.level_resolution(SMALL, 0) + 1
    assert N.dense_level(SMALL, 0)
    assert list(N.vertex_index(SMALL, 0, np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [2, 3, 1]]))) == \
        [1, n, n * n, 2 + 3 * n + n * n]


def _level(enc, l, F=2):
    return enc[:, l * F:(l + 1) * F]


def test_feature_at_a_grid_vertex_is_the_table_entry():
    import torch
    m = N.init_model(SMALL, seed=1)
    tables = torch.as_tensor(m["tables"], dtype=torch.float64)
    res = N.level_resolution(SMALL, 0)       # 4: vertices at multiples of 1/4
    v = np.array([[0, 0, 0], [1, 2, 3], [4, 4, 4], [3, 0, 2]])
    x = v / res
    enc = N.encode(SMALL, x, np.zeros(3), np.ones(3), tables).numpy()
    idx = N.vertex_index(SMALL, 0, v)
    np.testing.assert_array_equal(_level(enc, 0), m["tables"][0][idx].astype(np.float64))


def test_feature_is_trilinear_inside_a_cell_and_continuous_across_faces():
    import torch
    m = N.init_model(SMALL, seed=2)
    tables = torch.as_tensor(m["tables"], dtype=torch.float64)
    res = N.level_resolution(SMALL, 0)
    t = np.linspace(0.0, 1.0, 9)
    base = np.array([1.3, 2.6, 0.4]) / res     # inside cell (1, 2, 0)
    x = base[None, :] + np.outer(t * 0.5 / res, [1.0, 0.0, 0.0])
    f = _level(N.encode(SMALL, x, np.zeros(3), np.ones(3), tables).numpy(), 0)
    assert np.abs(f[2:] - 2 * f[1:-1] + f[:-2]).max() < 1e-15   # linear along an axis
    eps = 1e-9
    xa = np.array([[2.0 / res - eps, 0.31, 0.77], [2.0 / res + eps, 0.31, 0.77]])
    fa = N.encode(SMALL, xa, np.zeros(3), np.ones(3), tables).numpy()
    assert np.abs(fa[0] - fa[1]).max() < 1e-9


def test_zero_network_gives_the_head_offsets():
    m = N.init_model(SMALL, seed=3)
    for k in ("w1", "w2", "w3", "b1", "b2", "b3"):
        m[k] = np.zeros_like(m[k])
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(5, 3))
    p = N.params(SMALL, x, np.zeros(3), np.ones(3), m)
    np.testing.assert_array_equal(p["color"], 0.5)
    np.testing.assert_array_equal(p["opacity"], 0.5)
    np.testing.assert_array_equal(p["scale"], SMALL.scale_max / 2)
    np.testing.assert_array_equal(p["quat"], np.tile([[1.0], [0.0], [0.0], [0.0]], (1, 5)))


def test_gradients_match_central_differences():
    rng = np.random.default_rng(4)
    m = N.init_model(SMALL, seed=4)
    m["tables"] = rng.uniform(-0.5, 0.5, size=m["tables"].shape).astype(np.float32)  # away from ReLU ties
    x = rng.uniform(-2, 3, size=(40, 3))
    lo, hi = np.array([-2.0, -2.0, -2.0]), np.array([3.0, 3.0, 3.0])
    d = dict(quat=rng.normal(size=(4, 40)), scale=rng.normal(size=(3, 40)), opacity=rng.normal(size=40),
             color=rng.normal(size=(3, 40)))
    _, g = N.params_and_grads(SMALL, x, lo, hi, m, d)

    def f(mm):
        p = N.params(SMALL, x, lo, hi, mm)
        return sum(float((p[k] * d[k]).sum()) for k in p)

    h = 1e-6
    enc_rows = N.vertex_index(SMALL, 2, np.floor(np.clip((x - lo) / (hi - lo), 0, 1) *
                                                 N.level_resolution(SMALL, 2)).astype(np.int64))
    probes = [("tables", (2, int(enc_rows[0]), 1)), ("tables", (2, int(enc_rows[7]), 0)), ("w1", (3, 5)),
              ("b1", (2,)), ("w2", (1, 6)), ("b2", (7,)), ("w3", (9, 4)), ("b3", (3,)), ("w3", (0, 2))]
    for name, ix in probes:
        mp = {k: np.asarray(v, np.float64).copy() for k, v in m.items()}
        mm = {k: np.asarray(v, np.float64).copy() for k, v in m.items()}
        mp[name][ix] += h
        mm[name][ix] -= h
        fd = (f(mp) - f(mm)) / (2 * h)
        assert fd == pytest.approx(g[name][ix], rel=1e-6, abs=1e-9), (name, ix)
