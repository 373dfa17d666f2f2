"""Host logic of the autotuner (no GPU): the launch shapes it tries."""
import pytest

from paper_2208_13769_amd.autotune import GENERAL, candidates, strips


class FakeSolver:
    """Stands in for a solver: blocks resident per device for a shape, 0 for
    a shape the library cannot launch (here: two steps with 512 threads)."""

    def __init__(self, per_cu=4, cus=256):
        self.per_cu, self.cus = per_cu, cus

    def resident_blocks(self, block, spl):
        if spl == 2 and block == 512:
            return 0
        return self.per_cu * self.cus


def test_strips_are_multiples_of_32_columns():
    # 256 threads, two PC steps: halo 10 each side, 236 columns -> 224
    assert strips(4096, 256, "fp32u64", "pc", 2) == 19
    # 16-bit storage takes the same 32-column rule (two blocks may share a
    # line) with one more halo column: 256 - 2 * 6 = 244 -> 224, 512 -> 480
    assert strips(4096, 256, "fp16", "pc", 1) == 19
    assert strips(4096, 512, "fp16", "pc", 1) == 9
    assert strips(4096, 128, "fp16", "pc", 1) == 43  # 128 - 12 = 116 -> 96 columns
    assert strips(100, 128, "fp16", "pc", 1) == 1 and strips(117, 128, "fp16", "pc", 1) == 2
    # a plate narrower than one block's reach is one strip
    assert strips(100, 128, "fp32", "pc", 1) == 1


def test_large_plate_segments_fill_whole_waves():
    s = FakeSolver()
    c = candidates(s, 4096, 4096, "fp32u64", "pc")
    assert c[-1] == GENERAL  # the general step is always a candidate
    c = c[:-1]
    assert c and all(spl in (1, 2) for _, _, spl in c)
    assert not any(b == 512 and spl == 2 for b, _, spl in c)  # not launchable here
    for block, segs, spl in c:
        n_str = strips(4096, block, "fp32u64", "pc", spl)
        # no short-segment candidates on a plate whose grid fills the device
        assert 4096 // segs >= 8
        assert n_str * segs <= 4 * s.resident_blocks(block, spl)


def test_small_plate_tries_short_segments():
    c = candidates(FakeSolver(), 64, 64, "fp64", "pc")
    segs_64 = {segs for b, segs, spl in c if b == 64 and spl == 1}
    # one-, two- and four-row segments besides the 8-row floor of the wave rule
    assert {64, 32, 16, 8} <= segs_64


@pytest.mark.parametrize("scheme", ["pc", "explicit"])
def test_explicit_scheme_has_one_step_per_launch(scheme):
    c = candidates(FakeSolver(), 300, 90, "fp32", scheme)
    spls = {spl for b, _, spl in c if b}
    assert spls == ({1, 2} if scheme == "pc" else {1})
