"""Host-side batch layout (no GPU): concatenation offsets, index shifts and
the per-vertex scene ids of a ragged batch."""
import numpy as np
import pytest

from scenes import scene as S

B = pytest.importorskip("paper_2409_16385_amd.batch")


@pytest.fixture(scope="module")
def scenes():
    return [S.grasp_scene(900 + i, 6 + 2 * i, 80 + 40 * i, 8, frac=0.5, rotate=True) for i in range(3)]


def test_offsets_and_shifts(scenes):
    hb = B.concat(scenes)
    assert hb.n_scene == 3
    assert list(hb.vert_off) == list(np.concatenate([[0], np.cumsum([s.n_vert for s in scenes])]))
    assert hb.n_node == sum(s.n_node for s in scenes)
    for i, s in enumerate(scenes):
        f = hb.faces[hb.face_off[i]:hb.face_off[i + 1]]
        assert np.array_equal(f - hb.vert_off[i], s.faces)
        e = hb.edges[hb.edge_off[i]:hb.edge_off[i + 1]]
        assert np.array_equal(e - hb.vert_off[i], s.edges)
        v0, v1 = hb.vert_off[i], hb.vert_off[i + 1]
        assert np.all(hb.vert_scene[v0:v1] == i)
        rp = hb.W_rowptr[v0:v1 + 1]
        assert np.array_equal(rp - rp[0], s.W_rowptr)
        cols = hb.W_col[rp[0]:rp[-1]]
        assert np.array_equal(cols - hb.node_off[i], s.W_col)
        assert np.array_equal(hb.q[3 * hb.node_off[i]:3 * hb.node_off[i + 1]], s.q)


def test_every_primitive_stays_in_one_scene(scenes):
    hb = B.concat(scenes)
    sf = hb.vert_scene[hb.faces]
    assert np.all(sf == sf[:, :1])
    se = hb.vert_scene[hb.edges]
    assert np.all(se[:, 0] == se[:, 1])


def test_mismatched_dhat_is_rejected(scenes):
    import copy
    other = copy.copy(scenes[1])
    other.dhat = scenes[0].dhat * 2
    with pytest.raises(ValueError):
        B.concat([scenes[0], other])
