"""The edge post-pass's filters and rounded normals as the library evaluates
them (host-side constants, no GPU) against the oracle's, bit for bit: the
coefficients, and with them every edge and orientation decision, can only
agree bit for bit if the taps do."""
import numpy as np

from oracle import edgepass as E


def test_filters_bit_identical():
    import paper_2303_09523_amd as P
    taps, normals = P.edge_filters()
    ref = E.shearlet_filters()
    assert taps.shape == ref.shape == (8, 9, 9)
    assert np.array_equal(taps.view(np.uint64), ref.view(np.uint64))


def test_normals_match_the_oracle():
    import paper_2303_09523_amd as P
    _, normals = P.edge_filters()
    for k in range(8):
        assert tuple(int(v) for v in normals[k]) == E.normal_step(k)
