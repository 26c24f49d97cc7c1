"""Edge cases of the oracle: the barrier and its derivatives at distances
down to 1e-8 dhat against a 50-digit evaluation of Eq. 7 (decimal
arithmetic), and distances of degenerate primitives (zero-area triangles,
zero-length edges) against the type-free definition, with finite
derivatives."""
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle as O
from tests import _geom as G

getcontext().prec = 50


def _b_decimal(r):
    """b/dhat^2, b'/dhat, b'' at d = r dhat from b(d) = -(d - dhat)^2 ln(d/dhat),
    in 50-digit decimal arithmetic."""
    r = Decimal(r)
    one = Decimal(1)
    lr = r.ln()
    b = -((r - one) ** 2) * lr
    b1 = -2 * (r - one) * lr - (r - one) ** 2 / r
    b2 = -2 * lr - 4 * (r - one) / r + (r - one) ** 2 / (r * r)
    return float(b), float(b1), float(b2)


@pytest.mark.parametrize("r", [1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 0.5, 0.999999])
def test_barrier_near_zero_and_one(r):
    dhat = 2e-4
    b, b1, b2 = O.barrier(r * dhat, dhat)
    rb, rb1, rb2 = _b_decimal(r * dhat / dhat)
    assert b / dhat ** 2 == pytest.approx(rb, rel=1e-12)
    assert b1 / dhat == pytest.approx(rb1, rel=1e-12)
    assert b2 == pytest.approx(rb2, rel=1e-12)


def _degenerate_cases(rng):
    out = []
    for _ in range(50):
        base = rng.normal(size=3) * 1e-2
        t0 = base
        t1 = base + rng.normal(size=3) * 1e-2
        # collinear triangle (zero area) and a triangle with a repeated vertex
        s = rng.uniform(-0.5, 1.5)
        out.append((0, np.concatenate([rng.normal(size=3) * 1e-2, t0, t1, t0 + s * (t1 - t0)])))
        out.append((0, np.concatenate([rng.normal(size=3) * 1e-2, t0, t1, t1])))
        # zero-length edge against a segment, and two zero-length edges
        p = rng.normal(size=3) * 1e-2
        out.append((1, np.concatenate([p, p, t0, t1])))
        out.append((1, np.concatenate([p, p, t0, t0])))
    return out


def test_degenerate_primitives_distance():
    rng = np.random.default_rng(0)
    for kind, x12 in _degenerate_cases(rng):
        t = O.pt_type(*x12.reshape(4, 3)) if kind == 0 else O.ee_type(*x12.reshape(4, 3))
        s = O.pair_dist2(kind, t, x12)
        d = G.pair_distance(kind, x12)
        assert np.sqrt(s) == pytest.approx(d, rel=1e-12, abs=1e-15)
        if 0 < np.sqrt(s) < 1e-2:
            st, _, _, e, g, H = O.pair_eval(kind, x12, 1e-2, 1e3)
            assert st == O.OK and np.isfinite(e) and np.isfinite(g).all() and np.isfinite(H).all()
