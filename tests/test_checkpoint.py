"""Checkpoint files of a BDF2 march (q^n, q^{n-1}, t, dt, step): exact round trip on the host.
The resume-equals-continuous check on the GPU path is in test_gpu_checkpoint.py."""
import numpy as np
import pytest
import torch

from paper_1903_06304_amd import lmfr


def _state(seed, shape=(4, 37)):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(shape, generator=g, dtype=torch.float64) * 10.0 ** torch.randint(-30, 30, shape, generator=g)


def test_single_state_round_trip_is_exact(tmp_path):
    q, qm = _state(1), _state(2)
    t, dt = 0.1 + 0.2, 1.0 / 3.0   # values without a short decimal form
    lmfr.save_checkpoint(tmp_path / "c.safetensors", q, qm, t, dt, step=17)
    ck = lmfr.load_checkpoint(tmp_path / "c.safetensors", device="cpu")
    assert torch.equal(ck["q"], q) and torch.equal(ck["q_nm1"], qm)
    assert ck["t"] == t and ck["dt"] == dt and ck["step"] == 17


def test_batch_and_bdf1_start_round_trip(tmp_path):
    qs = [_state(3, (4, 5)), _state(4, (4, 11))]
    lmfr.save_checkpoint(tmp_path / "b.safetensors", qs, None, 2.5, 1e-3, step=0)
    ck = lmfr.load_checkpoint(tmp_path / "b.safetensors", device="cpu")
    assert ck["q_nm1"] is None and len(ck["q"]) == 2
    assert all(torch.equal(a, b) for a, b in zip(ck["q"], qs))
    with pytest.raises(ValueError):
        lmfr.save_checkpoint(tmp_path / "x.safetensors", qs, qs[:1], 0.0, 1.0)


def test_foreign_file_is_rejected(tmp_path):
    from safetensors.torch import save_file
    save_file({"q.0": torch.zeros(3, dtype=torch.float64)}, str(tmp_path / "f.safetensors"), metadata={"count": "1"})
    with pytest.raises(ValueError):
        lmfr.load_checkpoint(tmp_path / "f.safetensors", device="cpu")
