"""Admission logic on the CPU (no device).

The arena allocator and slot accounting of the C batch API are exercised
through the ABI wherever they answer before touching a device (footprints,
systems that cannot fit, bad arguments, an empty launch), and the serving
loop's policy (reuse of a system's idle slot, least-recently-used eviction
of idle slots of other systems, busy slots never evicted, the per-system
slot cap) against a stand-in arena with the same first-fit contract."""
import ctypes

import pytest

import paper_2009_12617_amd.serve as S
from paper_2009_12617_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def desc(K=32, order=4, max_atoms=1000, prec=1, own=True):
    d = _lib.SystemDesc()
    d.K1 = d.K2 = d.K3 = K
    d.order, d.beta, d.precision, d.max_atoms, d.N = order, 0.34, prec, max_atoms, max_atoms
    d.box[:] = [30.0, 0, 0, 0, 30.0, 0, 0, 0, 30.0]
    if not own:
        d.pos = d.q = d.forces = 0x7f0000000000  # never dereferenced here
    return d


def test_footprint_is_workspace_plus_io(lib):
    own = lib.pme_batch_footprint(ctypes.byref(desc()))
    ext = lib.pme_batch_footprint(ctypes.byref(desc(own=False)))
    ws = lib.pme_workspace_bytes(32, 32, 32, 4, 1000, 1)
    assert ext == (ws + 255) // 256 * 256
    # positions, charges, forces (56 B per atom) and the energy/virial row,
    # each rounded up to 256 bytes
    assert own - ext == 24000 // 256 * 256 + 256 + 8192 + 24000 // 256 * 256 + 256 + 256
    assert lib.pme_batch_footprint(ctypes.byref(desc(K=50))) == 0
    assert lib.pme_batch_footprint(None) == 0


def test_batch_admission_answers_without_a_device(lib):
    fake = 0x7f0000000000  # never dereferenced: every call below answers first
    h = ctypes.c_void_p()
    assert lib.pme_batch_create(ctypes.byref(h), 0, fake, 1 << 20, None) == 1
    assert lib.pme_batch_create(ctypes.byref(h), 4, fake + 8, 1 << 20, None) == 3
    assert lib.pme_batch_create(ctypes.byref(h), 4, fake, 1 << 20, None) == 0
    slot = ctypes.c_int(7)
    big = desc(K=64, max_atoms=65535)
    assert lib.pme_batch_footprint(ctypes.byref(big)) > (1 << 20)
    assert lib.pme_batch_admit(h, ctypes.byref(big), ctypes.byref(slot)) == 8  # PME_EBUSY
    assert slot.value == -1
    assert lib.pme_batch_admit(h, ctypes.byref(desc(K=50)), ctypes.byref(slot)) == 2
    bad = desc(max_atoms=-1)
    assert lib.pme_batch_admit(h, ctypes.byref(bad), ctypes.byref(slot)) == 1
    assert lib.pme_batch_retire(h, 0) == 1          # nothing admitted
    assert lib.pme_batch_retire(h, -3) == 1
    assert lib.pme_batch_plan(h, 0) is None
    assert lib.pme_batch_launch(h, None, 0) == 0    # nothing to run
    two = (ctypes.c_int * 2)(0, 1)
    assert lib.pme_batch_launch(h, two, 2) == 1     # slots not admitted
    n, used, lf = ctypes.c_int(-1), ctypes.c_size_t(1), ctypes.c_size_t(0)
    assert lib.pme_batch_stats(h, ctypes.byref(n), ctypes.byref(used), ctypes.byref(lf)) == 0
    assert n.value == 0 and used.value == 0 and lf.value == 1 << 20
    assert lib.pme_batch_destroy(h) == 0
    assert lib.pme_batch_destroy(None) == 1


def test_tuning_queries_without_a_device(lib):
    v = lib.pme_tuning_variants(64, 64, 64, 4, 1)
    assert v == 31                                   # every variant at 64^3
    assert lib.pme_tuning_variants(64, 64, 64, 4, 0) == 31   # FP64 too (152 KB of LDS per column)
    assert lib.pme_tuning_variants(48, 48, 48, 4, 1) & 16 == 0  # 48-point pencils: no
    assert lib.pme_tuning_variants(16, 16, 16, 4, 1) == 1 | 4 | 8   # no split column passes
    assert lib.pme_tuning_variants(50, 50, 50, 4, 1) == 0
    t = _lib.Tuning()
    assert lib.pme_default_tuning(64, 64, 64, 4, 1, ctypes.byref(t)) == 0
    assert t.as_dict() == {"conv": 2, "interp": 0, "bin_chunk": 1024}
    assert lib.pme_default_tuning(64, 64, 64, 4, 0, ctypes.byref(t)) == 0
    assert t.as_dict() == {"conv": 2, "interp": 0, "bin_chunk": 1024}
    assert lib.pme_default_tuning(48, 48, 48, 4, 1, ctypes.byref(t)) == 0
    assert t.as_dict() == {"conv": 0, "interp": 0, "bin_chunk": 1024}
    assert lib.pme_default_tuning(128, 128, 128, 6, 1, ctypes.byref(t)) == 0
    assert t.as_dict() == {"conv": 1, "interp": 1, "bin_chunk": 1024}
    assert lib.pme_default_tuning(64, 64, 128, 4, 1, ctypes.byref(t)) == 0
    assert t.as_dict() == {"conv": 1, "interp": 0, "bin_chunk": 1024}
    assert lib.pme_default_tuning(50, 50, 50, 4, 1, ctypes.byref(t)) == 2
    assert lib.pme_set_tuning(None, ctypes.byref(t)) == 1
    assert lib.pme_get_tuning(None, ctypes.byref(t)) == 1
    assert lib.pme_autotune(None, None, None, 0, None, None, None, 5, None, None, None, 0) == 1


class FakeSlot:
    def __init__(self, system_id, slot):
        self.system_id = system_id
        self.slot = slot
        self.footprint = 100
        self.busy = False
        self.last_used = 0.0


class FakePool:
    """First-fit stand-in: fixed-size systems of 100 bytes in `budget`."""

    def __init__(self, budget):
        self.budget, self.used, self.next, self.retired = budget, 0, 0, []

    def admit(self, *a, **k):
        if self.used + 100 > self.budget:
            return None
        self.used += 100
        self.next += 1
        return self.next

    def retire(self, slot):
        self.used -= 100
        self.retired.append(slot)


@pytest.fixture
def srv(monkeypatch):
    monkeypatch.setattr(S, "Slot", lambda system_id, slot, pool, sysd, fp, bufs: FakeSlot(system_id, slot))
    monkeypatch.setattr(S.Server, "_host_bufs", lambda self, system_id: None)
    s = S.Server.__new__(S.Server)
    s.pool = [S.PoolSystem(None, [0.0], None, 32)] * 5
    s.budget = 250
    s.precision = "fp32_fixed"
    s.slots_per_system = 2
    s.device = None
    s.compute = None
    s.batch = FakePool(250)
    s.fp = [100] * 5
    s.slots = {i: [] for i in range(5)}
    s.resident = 0
    s.stats = S.ServeStats()
    monkeypatch.setattr(S.torch.cuda, "stream", lambda st: _Null())
    return s


class _Null:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def test_budget_eviction_and_reuse(srv):
    a = srv._free_slot(0)
    a.busy = True
    b = srv._free_slot(1)
    b.busy = True
    assert srv.resident == 200
    assert srv._free_slot(2) is None               # full and nothing idle
    assert srv.stats.rejected_for_budget == 1
    b.busy, b.last_used = False, 0.3
    assert srv._free_slot(1) is b                  # an idle slot of the system is reused
    c = srv._free_slot(2)                          # evicts the idle slot of system 1
    assert c.system_id == 2 and srv.batch.retired == [b.slot]
    assert srv.stats.evictions == 1 and srv.resident == 200
    assert srv.stats.peak_resident_bytes <= srv.budget


def test_slots_per_system_cap(srv):
    srv.batch = FakePool(10 ** 6)
    x = srv._free_slot(3)
    x.busy = True
    y = srv._free_slot(3)
    y.busy = True
    assert srv._free_slot(3) is None


def test_kept_forces_copied_out_in_chunks():
    # the serving loop copies a kept request's forces out of the slot's
    # pinned buffer a chunk per loop turn, releasing the slot only after the
    # last chunk; two requests queue in completion order
    import numpy as np
    import torch

    class Slot:
        busy = True

    class Req:
        pass

    class Stub:
        COPY_CHUNK = S.Server.COPY_CHUNK

    rng = np.random.default_rng(7)
    reqs = []
    for n in (S.Server.COPY_CHUNK * 2 + 5, 17):
        r = Req()
        r.slot = Slot()
        r.slot.host_f = torch.from_numpy(rng.standard_normal((n, 3)))
        r.forces = np.empty((n, 3))
        r.copied = 0
        reqs.append(r)
    pending = list(reqs)
    turns = 0
    while pending:
        S.Server._copy_kept(Stub(), pending)
        turns += 1
        if reqs[0] in pending:
            assert reqs[0].slot.busy and reqs[1].slot.busy
    assert turns == 4  # three chunks, then the small request
    for r in reqs:
        assert not r.slot.busy
        assert np.array_equal(r.forces, r.slot.host_f.numpy())
