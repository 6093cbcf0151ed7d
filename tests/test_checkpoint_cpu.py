"""Checkpoint files: round trip of every dtype the reconstruction state uses,
atomic replace, and refusal of foreign files (no GPU)."""
import numpy as np
import pytest
import torch

from paper_2008_11511_amd import checkpoint


def test_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    state = dict(obj=torch.from_numpy((rng.standard_normal((5, 7)) + 1j * rng.standard_normal((5, 7)))
                                      .astype(np.complex64)),
                 ml_state=torch.from_numpy(rng.integers(0, 255, 4096, dtype=np.uint8)),
                 positions=rng.standard_normal((9, 2)),
                 background=torch.ones((4, 4), dtype=torch.float32), psi=None)
    path = str(tmp_path / "ck.npz")
    checkpoint.save(path, **state)
    got = checkpoint.load(path)
    assert set(got) == {"obj", "ml_state", "positions", "background"}
    for k in got:
        ref = state[k] if isinstance(state[k], torch.Tensor) else torch.from_numpy(state[k])
        assert got[k].dtype == ref.dtype and torch.equal(got[k], ref)
    assert not (tmp_path / "ck.npz.tmp").exists()


def test_refuses_other_files(tmp_path):
    path = str(tmp_path / "other.npz")
    np.savez(path, obj=np.zeros(3))
    with pytest.raises(ValueError):
        checkpoint.load(path)
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x.npz"), __format__=np.zeros(1))
