"""The two-body input of the realignment study (the setup of the paper's
Fig. 2): two irregular bodies of unit radius; beyond a separation of 2 sqrt 3
each body lies in its own octant, so with n_leaf = bodies' size and a wide
acceptance angle the walk has exactly one far pair, the two bodies."""
import numpy as np
import pytest

import oracle
from paper_2107_07166_amd.generators import irregular_pair


@pytest.mark.parametrize("sep", [3.6, 8.0])
def test_bodies_are_unit_radius_and_apart(sep):
    pos, m = irregular_pair(1500, 3, sep)
    assert pos.shape == (3000, 3) and np.isclose(m.sum(), 1.0)
    c = sep / (2 * np.sqrt(3.0))
    for half, sign in ((pos[:1500], -1.0), (pos[1500:], 1.0)):
        ctr = half.mean(0)
        np.testing.assert_allclose(ctr, sign * c, atol=1e-12)
        assert np.isclose(np.sqrt(((half - ctr) ** 2).sum(1)).max(), 1.0)
        assert (sign * half > 0).all()


def test_one_far_pair_between_the_bodies():
    pos, m = irregular_pair(1500, 3, 4.0)
    t = oracle.Tree(pos, m, n_leaf=1500, theta=0.99)
    far, near = t.lists()
    nodes = t.nodes()
    assert len(far) == 1
    a, b = far[0]
    assert {int(nodes["count"][a]), int(nodes["count"][b])} == {1500}
