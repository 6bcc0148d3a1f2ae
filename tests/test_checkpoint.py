"""Checkpoint/resume of the texture fit (CPU): the state round-trips bit for bit through save_state /
load_state, is written in place (tensor addresses kept, as a captured graph needs), and a file that does
not match the run (names, counts, shapes, dtypes, settings) is refused before anything is overwritten."""
import pytest
import torch

from paper_2409_02482_amd.fit import load_state, save_state


def _state(seed, shape=(8, 6, 4)):
    g = torch.Generator().manual_seed(seed)
    return {"params": [torch.rand(shape, generator=g) for _ in range(3)],
            "m": [torch.randn(shape, generator=g) for _ in range(3)],
            "v": [torch.rand(shape, generator=g) for _ in range(3)],
            "step": torch.tensor([17], dtype=torch.int32),
            "history": torch.rand(32, generator=g, dtype=torch.float64)}


def _flat(st):
    out = []
    for v in st.values():
        out += list(v) if isinstance(v, list) else [v]
    return out


def test_round_trip_bit_for_bit_in_place(tmp_path):
    a, b = _state(1), _state(2)
    path = str(tmp_path / "fit.pt")
    save_state(path, a, {"k": 3, "loss": "l2"})
    ptrs = [t.data_ptr() for t in _flat(b)]
    load_state(path, b, {"k": 3, "loss": "l2"})
    assert [t.data_ptr() for t in _flat(b)] == ptrs
    for x, y in zip(_flat(a), _flat(b)):
        assert x.dtype == y.dtype and torch.equal(x.view(torch.uint8), y.view(torch.uint8))


@pytest.mark.parametrize("what", ["meta", "shape", "count", "dtype", "name"])
def test_mismatch_refused_without_writing(tmp_path, what):
    a = _state(1)
    path = str(tmp_path / "fit.pt")
    save_state(path, a, {"k": 3, "loss": "l2"})
    b = _state(2)
    meta = {"k": 3, "loss": "l2"}
    if what == "meta":
        meta = {"k": 3, "loss": "l1"}
    elif what == "shape":
        b["v"][2] = torch.zeros(8, 6, 3)
    elif what == "count":
        b["m"] = b["m"][:2]
    elif what == "dtype":
        b["history"] = torch.zeros(32, dtype=torch.float32)
    elif what == "name":
        b["extra"] = torch.zeros(1)
    before = [t.clone() for t in _flat(b)]
    with pytest.raises(ValueError):
        load_state(path, b, meta)
    for x, y in zip(before, _flat(b)):
        assert torch.equal(x, y)
