"""The per-call tile choice of the rank-K kernels (no tile fixed or tuned):
a cost model of the padded lower-triangle tile area, evaluated on the host
(chi0_tile_choice needs no device).  The expected choices are the fastest
configurations measured on the MI355X for these shapes: for BF16x3 and
FP32 the frequency-group kernels whenever there are several frequencies
(npb 2048 and 384) and 64^2 tiles for one frequency at npb 287; FP64 its
large tiles at npb 2048 and smaller square ones at npb 287-384."""
import pytest

from paper_2506_03477_amd import Chi0Error, tile_choice

HEADLINE = [(2048, 12, [(200, 1200)] * 16)]          # npb 2048, 16 k-points, 12 frequencies
BATCH = [(384, 12, [(32, 250)] * 2)] * 32             # 32 q-points at npb 384
SIGX = [(287, 1, [(92, 2097)] * 16)]                  # exchange self-energy, nqp 287

CASES = [
    (HEADLINE, {"bf16x3": 20, "fp32": 2, "fp64": 3}),
    (BATCH, {"bf16x3": 20, "fp32": 2, "fp64": 3}),
    (SIGX, {"bf16x3": 2, "fp32": 1, "fp64": 2}),
]


@pytest.mark.parametrize("shapes,expected", CASES)
def test_choice_matches_measured_best(shapes, expected):
    for prec, tile in expected.items():
        assert tile_choice(prec, shapes) == tile, prec


def test_choice_is_size_driven_not_row_driven():
    # the model scales every candidate by the same rows: doubling the rows,
    # or the frequencies between whole frequency groups, does not change the
    # choice; one frequency makes a four-frequency group cost four
    for prec in ("bf16x3", "fp32", "fp64"):
        a = tile_choice(prec, SIGX)
        assert tile_choice(prec, [(287, 1, [(184, 2097)] * 16)]) == a
        b = tile_choice(prec, [(287, 4, [(92, 2097)] * 16)])
        assert tile_choice(prec, [(287, 8, [(92, 2097)] * 16)]) == b
    assert tile_choice("bf16x3", SIGX) != tile_choice("bf16x3", [(287, 4, [(92, 2097)] * 16)])


def test_choice_rejects_bad_input():
    with pytest.raises(Chi0Error):
        tile_choice("bf16x3", [(0, 1, [(1, 1)])])
    with pytest.raises(Chi0Error):
        tile_choice("fp64", [(16, 1, [(-1, 1)])])
    assert tile_choice("fp64", [(16, 1, [])]) >= 0       # no blocks: any tile, no error
