"""Admission logic of the serving loop on the CPU (no device): footprints
within the budget, least-recently-used eviction of idle slots, busy slots
never evicted, systems that cannot fit rejected up front."""
import pytest

import paper_2009_12617_amd.serve as S


class FakeSlot:
    def __init__(self, system_id, sysd, precision, device):
        self.system_id = system_id
        self.footprint = 100
        self.busy = False
        self.last_used = 0.0
        self.released = False

    def release(self):
        self.released = True


@pytest.fixture
def srv(monkeypatch):
    monkeypatch.setattr(S, "Slot", FakeSlot)
    monkeypatch.setattr(S, "slot_footprint", lambda sysd, precision: 100)
    s = S.Server.__new__(S.Server)
    s.pool = [object()] * 5
    s.budget = 250
    s.precision = "fp32_fixed"
    s.slots_per_system = 2
    s.device = None
    s.slots = {i: [] for i in range(5)}
    s.resident = 0
    s.stats = S.ServeStats()
    return s


def test_budget_eviction_and_reuse(srv):
    a = srv._free_slot(0, 0.0)
    a.busy = True
    b = srv._free_slot(1, 0.1)
    b.busy = True
    assert srv.resident == 200
    assert srv._free_slot(2, 0.2) is None          # full and nothing idle
    assert srv.stats.rejected_for_budget == 1
    b.busy, b.last_used = False, 0.3
    assert srv._free_slot(1, 0.35) is b             # an idle slot of the system is reused
    c = srv._free_slot(2, 0.4)                      # evicts the idle slot of system 1
    assert c.system_id == 2 and b.released and not a.released
    assert srv.stats.evictions == 1 and srv.resident == 200
    assert srv.stats.peak_resident_bytes <= srv.budget


def test_slots_per_system_cap(srv):
    srv.budget = 10 ** 6
    x = srv._free_slot(3, 0.0)
    x.busy = True
    y = srv._free_slot(3, 0.0)
    y.busy = True
    assert srv._free_slot(3, 0.0) is None


def test_system_larger_than_budget_is_rejected(monkeypatch):
    monkeypatch.setattr(S, "slot_footprint", lambda sysd, precision: 10 ** 9)
    with pytest.raises(ValueError):
        S.Server([object()], hbm_budget_bytes=10 ** 6, device="cpu")
