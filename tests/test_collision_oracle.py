"""Pins of the reference collision check (Sec. II-A: agents that collide are
marked dead and excluded): hand-built geometric cases and agreement with a
library k-d tree away from the threshold."""
import numpy as np
import pytest
from scipy.spatial import cKDTree


def rows_of(points):
    return np.ascontiguousarray(np.asarray(points, dtype=np.float32).T)


def test_pair_inside_and_outside_the_radius_sum(oracle):
    r = np.float32(0.17)
    gap = np.float32(2 * r)
    inside = rows_of([[10, 10, 5], [10 + gap * np.float32(0.999), 10, 5]])
    outside = rows_of([[10, 10, 5], [10 + gap * np.float32(1.001), 10, 5]])
    a, died = oracle.detect_collisions(inside, [r], np.ones(2, np.uint8))
    assert died == 2 and not a.any()
    a, died = oracle.detect_collisions(outside, [r], np.ones(2, np.uint8))
    assert died == 0 and a.all()


def test_touching_exactly_is_not_a_collision(oracle):
    """Strict inequality: |d| = r_i + r_j (representable exactly) survives."""
    pts = rows_of([[0, 0, 0], [0.5, 0, 0]])
    a, died = oracle.detect_collisions(pts, [0.25], np.ones(2, np.uint8))
    assert died == 0


def test_dead_agents_are_excluded_and_decisions_are_simultaneous(oracle):
    # A-B and B-C overlap, A-C do not: all three die in one call
    pts = rows_of([[0, 0, 0], [0.3, 0, 0], [0.6, 0, 0], [5, 5, 5], [5.2, 5, 5]])
    alive = np.array([1, 1, 1, 1, 0], np.uint8)        # E is already dead
    a, died = oracle.detect_collisions(pts, [0.17], alive)
    assert a.tolist() == [0, 0, 0, 1, 0] and died == 3


def test_per_type_radii(oracle):
    pts = rows_of([[0, 0, 0], [0.5, 0, 0], [10, 0, 0], [10.5, 0, 0]])
    ti = np.array([0, 1, 0, 0], np.int32)
    a, _ = oracle.detect_collisions(pts, [0.1, 0.45], np.ones(4, np.uint8), type_idx=ti)
    assert a.tolist() == [0, 0, 1, 1]                 # 0.1 + 0.45 > 0.5 > 0.2


def test_lattice_spaced_beyond_the_threshold_survives(oracle):
    g = np.arange(6, dtype=np.float32) * np.float32(0.35)
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    a, died = oracle.detect_collisions(rows_of(pts), [0.17], np.ones(len(pts), np.uint8))
    assert died == 0


def test_matches_kd_tree_away_from_the_threshold(oracle):
    rng = np.random.default_rng(11)
    n, r = 3000, np.float32(0.17)
    pts = rng.uniform(0, [12, 12, 3], size=(n, 3)).astype(np.float32)
    thr = float(2 * r)
    d = cKDTree(pts.astype(np.float64))
    # pairs within a band around the threshold are decided by rounding; keep none
    near = d.query_pairs(thr * (1 + 1e-5))
    far = d.query_pairs(thr * (1 - 1e-5))
    band = near - far
    keep = np.ones(n, bool)
    for i, j in band:
        keep[i] = keep[j] = False
    pts = pts[keep]
    d = cKDTree(pts.astype(np.float64))
    expect = np.ones(len(pts), np.uint8)
    for i, j in d.query_pairs(thr):
        expect[i] = expect[j] = 0
    a, died = oracle.detect_collisions(rows_of(pts), [r], np.ones(len(pts), np.uint8))
    assert np.array_equal(a, expect) and died == int((expect == 0).sum()) > 0


def test_per_agent_query_matches_full_check(oracle):
    rng = np.random.default_rng(5)
    pts = rng.uniform(0, [6, 6, 2], size=(1500, 3)).astype(np.float32)
    alive = (rng.random(1500) > 0.1).astype(np.uint8)
    full, _ = oracle.detect_collisions(rows_of(pts), [0.17], alive)
    q = np.arange(1500)
    hit = oracle.collides(rows_of(pts), [0.17], alive, q)
    expect = (alive == 1) & (full == 0)
    assert np.array_equal(hit.astype(bool), expect)
