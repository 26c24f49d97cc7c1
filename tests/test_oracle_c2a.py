"""Pins for the oracle's alternative CCD (conservative advancement along the
closest direction, after the C2A reference the paper cites for its CCD):
the additive CCD's steps with its motion bound lp replaced, at each
iterate, by the closing speed along the closest direction.

Pinned by closed forms (a point or an edge approaching along the contact
normal while the other primitive slides in its own plane: the bound is
(1 - s) d0 / v whatever the sliding speed, where the additive bound
shrinks), separating motion (t_c), zero motion, and brute force: on random
pairs and random linear motions the sampled distance stays positive up to
the bound, which never exceeds the first sampled time of contact."""
import numpy as np
import pytest

import oracle as O

S = 0.1


def _dist(kind, x12):
    return np.sqrt(O.pair_eval(kind, x12, 1.0, 1.0)[2])


def _pt(h):
    return np.array([0.2, 0.25, h, 0, 0, 0, 1, 0, 0, 0, 1, 0], dtype=float)


def _ee(h):
    return np.array([-1, 0.1, h, 1, 0.1, h, 0.05, -1, 0, 0.05, 1, 0], dtype=float)


@pytest.mark.parametrize("w", [0.0, 0.05, 0.3])
@pytest.mark.parametrize("v,d0", [(2.0, 1.0), (1e-3, 2e-4)])
def test_point_approaching_a_sliding_triangle(w, v, d0):
    x = _pt(d0)
    p = np.zeros(12)
    p[2] = -v
    p[3::3] = -w * v  # the triangle slides along -x in its own plane; the point stays over it
    t, it = O.c2a_pair(0, x, p, s=S)
    assert t == pytest.approx((1 - S) * d0 / v, rel=1e-12)
    assert it == 2
    ta, _ = O.accd_pair(0, x, p, s=S)
    if w > 0:
        assert ta < t  # the additive bound counts the sliding as closing speed
    else:
        assert ta == pytest.approx(t, rel=1e-12)


@pytest.mark.parametrize("w", [0.0, 0.2])
def test_edge_approaching_a_sliding_edge(w):
    d0, v = 3e-3, 0.5
    x = _ee(d0)
    p = np.zeros(12)
    p[2] = p[5] = -v  # edge a moves down
    p[7] = p[10] = w  # edge b slides along its own direction (y)
    t, _ = O.c2a_pair(1, x, p, s=S)
    assert t == pytest.approx((1 - S) * d0 / v, rel=1e-12)


def test_separating_and_still():
    x = _pt(0.5)
    p = np.zeros(12)
    p[2] = 1.0  # the point moves away
    assert O.c2a_pair(0, x, p) == (1.0, 0)
    assert O.c2a_pair(0, x, np.zeros(12)) == (1.0, 0)
    t, _ = O.c2a_pair(0, x, -p, t_c=0.25)  # contact at 0.5 lies beyond t_c
    assert t == 0.25


@pytest.mark.parametrize("kind", [0, 1])
def test_conservative_against_sampled_motion(kind):
    rng = np.random.default_rng(40 + kind)
    for _ in range(80):
        x = rng.normal(size=12)
        p = rng.normal(size=12) * rng.uniform(0.5, 4.0)
        t, it = O.c2a_pair(kind, x, p, s=S)
        assert 0 < t <= 1.0 and it >= 0
        ts = np.linspace(0.0, 1.0, 2001)
        d = np.array([_dist(kind, x + tt * p) for tt in ts])
        # first sampled time of (near) contact
        hit = np.nonzero(d < 1e-9)[0]
        if len(hit):
            assert t <= ts[hit[0]]
        # positive all the way to the bound
        assert d[ts <= t].min() > 0
        # and at the bound itself
        assert _dist(kind, x + t * p) > 0


@pytest.mark.parametrize("kind", [0, 1])
def test_colliding_motions_stop_before_contact(kind):
    rng = np.random.default_rng(60 + kind)
    n_done = 0
    for _ in range(400):
        x0 = rng.normal(size=12)
        # aim the pair's first primitive at the second's
        c1 = x0[:3] if kind == 0 else 0.5 * (x0[:3] + x0[3:6])
        c2 = x0[3:].reshape(3, 3).mean(0) if kind == 0 else 0.5 * (x0[6:9] + x0[9:12])
        p = np.zeros(12)
        nf = 1 if kind == 0 else 2
        for a in range(4):
            p[3 * a:3 * a + 3] = (c2 - c1) * (1.5 if a < nf else 0.0) + rng.normal(size=3) * 0.05
        ts = np.linspace(0.0, 1.0, 2001)
        d = np.array([_dist(kind, x0 + tt * p) for tt in ts])
        hit = np.nonzero(d < 1e-3 * d[0])[0]
        if not len(hit):
            continue
        t, _ = O.c2a_pair(kind, x0, p, s=S)
        assert t <= ts[hit[0]]
        assert d[ts <= t].min() > 0
        n_done += 1
        if n_done >= 25:
            break
    assert n_done >= 10
