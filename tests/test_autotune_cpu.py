"""Host logic of the tile autotuner: every candidate shape is one the library
instantiates for the kind (the blocked kinds vary only their z chunk), and no
z chunk exceeds the grid's planes."""
import pytest

import paper_1207_1746_amd as G
from paper_1207_1746_amd import autotune as AT


@pytest.mark.parametrize("kind", [G.K_WJACOBI, G.K_VARCOEF7, G.K_LINEAR, G.K_VC13_APPLY, G.K_RBGS,
                                  G.K_IMG_BOX5_LAP, G.K_WJACOBI_TB, G.K_RBGS_TB])
@pytest.mark.parametrize("dtype", [G.F64, G.F32])
@pytest.mark.parametrize("nz", [1, 7, 512])
def test_candidates_are_instantiated_shapes(kind, dtype, nz):
    cands = AT.candidates(kind, dtype, nz)
    assert cands and len(set(cands)) == len(cands)
    for v, nw, cz in cands:
        if kind in AT.BLOCKED:
            assert (v, nw) == (1, 16)
        elif kind == G.K_IMG_BOX5_LAP:
            assert (v, nw) == (4, 4)
        else:
            assert v in (1, 2, 4) and nw in (4, 6, 8)
            if kind in AT.RADIUS2 and dtype == G.F64:
                assert v == 1
            if kind not in AT.RADIUS2:
                assert nw in (4, 8)
        if kind != G.K_IMG_BOX5_LAP:
            assert 1 <= cz <= max(nz, 1)
