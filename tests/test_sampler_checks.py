"""Host-side argument checks of the Python binding (no GPU needed): a stats
tensor of the wrong dtype, device, layout or shape is refused before its
pointer reaches the library."""
import pytest

torch = pytest.importorskip("torch")

from paper_2304_01772_amd.sampler import Sampler  # noqa: E402


def _bare(R=3, width=8):
    # a Sampler without a context: only the fields the checks read
    s = Sampler.__new__(Sampler)
    s.device = torch.device("cpu")
    s.R, s.width, s.ctx = R, width, None
    return s


def test_stats_checks_accept_a_matching_tensor():
    s = _bare()
    s._check_stats(torch.zeros((5, 3, 8), dtype=torch.int32), 5, "sweep")


@pytest.mark.parametrize("bad,rows", [
    (torch.zeros((5, 3, 8), dtype=torch.int64), 5),          # dtype
    (torch.zeros((5, 3, 8), dtype=torch.float32), 5),
    (torch.zeros((4, 3, 8), dtype=torch.int32), 5),          # too few rows
    (torch.zeros((5, 2, 8), dtype=torch.int32), 5),          # another R
    (torch.zeros((5, 3, 16), dtype=torch.int32), 5),         # another width
    (torch.zeros((5, 24), dtype=torch.int32), 5),            # flattened
    (torch.zeros((5, 8, 3), dtype=torch.int32).transpose(1, 2), 5),  # not contiguous
    (None, 1),
])
def test_stats_checks_refuse_mismatches(bad, rows):
    s = _bare()
    with pytest.raises(ValueError):
        s._check_stats(bad, rows, "sweep")


def test_stats_checks_refuse_another_device():
    s = _bare()
    s.device = torch.device("meta")
    with pytest.raises(ValueError):
        s._check_stats(torch.zeros((5, 3, 8), dtype=torch.int32), 5, "grad")
