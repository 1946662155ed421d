"""Host-side logic that needs no GPU: serving pool sizing."""
import pytest

from paper_1812_01502_amd.serving import slot_footprint, slots_for_budget


def test_slot_footprint_counts_every_buffer():
    # states (2 buffers x d planes) + log-weights (2 buffers) + partial records
    # + control block + model parameters + record
    assert slot_footprint(1, 4096) == 2 * 4096 * 4 + 2 * 4096 * 4 + 8 * 7 * 4 + 12800 + 5632 + 304
    assert slot_footprint(16, 1 << 20) > slot_footprint(4, 1 << 20) > slot_footprint(1, 1 << 20)


@pytest.mark.parametrize("budget", [1 << 26, 1 << 30, 24 << 30])
def test_slots_for_budget_fits(budget):
    dims = {"sv": 1, "lg4": 4}
    shapes = {("sv", 4096): 1.0, ("lg4", 1 << 16): 1.0, ("lg4", 1 << 20): 2.0}
    cnt = slots_for_budget(shapes, dims, budget)
    used = sum(slot_footprint(dims[m], n) * c for (m, n), c in cnt.items())
    assert all(c >= 1 for c in cnt.values())
    # each pool stays within its share (pools of one slot may exceed a tiny budget)
    for (m, n), c in cnt.items():
        share = budget * shapes[(m, n)] / sum(shapes.values())
        assert c == 1 or c * slot_footprint(dims[m], n) <= share
    assert used <= budget or min(cnt.values()) == 1
