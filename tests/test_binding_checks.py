"""Host checks of the Python binding: keys of the wrong width, bound arrays
of different lengths and malformed batch offsets are rejected before any call
crosses the C ABI (whose kernels would otherwise read past the caller's
buffers).  No GPU is used: the library is replaced by a stub that fails the
test if it is called, and CPU tensors stand in for device tensors."""
import pytest
import torch

binding = pytest.importorskip("paper_2506_01576_amd._binding")


class _NoCalls:
    def __getattr__(self, name):
        raise AssertionError(f"{name} reached the C ABI")


@pytest.fixture
def host_binding(monkeypatch):
    monkeypatch.setattr(binding, "lib", lambda: _NoCalls())
    monkeypatch.setattr(binding, "_dev", lambda t, name: None)
    monkeypatch.setattr(binding, "_stream", lambda s: 0)
    return binding


def _index(b, bits):
    return b.Index._wrap(b.ctypes.c_void_p(1), 100, 9, "eks", bits, torch.int64 if bits == 64 else torch.int32)


def _batch(b, bits, count):
    bt = b.Batch.__new__(b.Batch)
    bt._indexes = []
    bt.key_bits, bt.count, bt._total_seen = bits, count, {}
    bt._h = b.ctypes.c_void_p(1)
    return bt


def test_index_rejects_wrong_width(host_binding):
    ix = _index(host_binding, 64)
    for bad in (torch.zeros(4, dtype=torch.int32), torch.zeros(4, dtype=torch.float64)):
        with pytest.raises(ValueError):
            ix.point(bad)
        with pytest.raises(ValueError):
            ix.range(bad, bad)
    q = torch.zeros(4, dtype=torch.int64)
    with pytest.raises(ValueError):
        ix.point(q, out=torch.empty(3, dtype=torch.int32))  # output too short
    with pytest.raises(ValueError):
        ix.point(q, out=torch.empty(4, dtype=torch.int64))  # output not 32-bit
    ix._h = None


def test_index_range_rejects_unequal_bounds(host_binding):
    ix = _index(host_binding, 32)
    with pytest.raises(ValueError):
        ix.range(torch.zeros(5, dtype=torch.int32), torch.zeros(4, dtype=torch.int32))
    ix._h = None


def test_batch_point_checks(host_binding):
    bt = _batch(host_binding, 64, 3)
    q = torch.zeros(10, dtype=torch.int64)
    good = torch.tensor([0, 4, 4, 10], dtype=torch.int64)
    for bad_q in (torch.zeros(10, dtype=torch.int32),):
        with pytest.raises(ValueError):
            bt.point(bad_q, good)
    for bad_off in (torch.tensor([0, 4, 10], dtype=torch.int64),       # count + 1 entries expected
                    torch.tensor([0, 4, 4, 10], dtype=torch.int32),    # not 64-bit
                    torch.tensor([0, 4, 4, 11], dtype=torch.int64)):   # more queries than given
        with pytest.raises(ValueError):
            bt.point(q, bad_off)
    with pytest.raises(ValueError):
        bt.point(q, good, out=torch.empty(9, dtype=torch.int32))
    bt._h = None


def test_batch_mixed_checks(host_binding):
    bt = _batch(host_binding, 32, 2)
    lo = torch.zeros(6, dtype=torch.int32)
    off = torch.tensor([0, 2, 6], dtype=torch.int64)
    kind = torch.zeros(6, dtype=torch.uint8)
    with pytest.raises(ValueError):
        bt.mixed(lo, torch.zeros(5, dtype=torch.int32), kind, off)
    with pytest.raises(ValueError):
        bt.mixed(lo, lo, torch.zeros(5, dtype=torch.uint8), off)
    with pytest.raises(TypeError):
        bt.mixed(lo, lo, torch.zeros(6, dtype=torch.int32), off)
    with pytest.raises(ValueError):
        bt.mixed(torch.zeros(6, dtype=torch.int64), torch.zeros(6, dtype=torch.int64), kind, off)
    with pytest.raises(ValueError):
        bt.mixed(lo, lo, kind, torch.tensor([0, 2, 5], dtype=torch.int64))  # must cover all 6 queries
    bt._h = None
