"""Durable checkpoint files (host side, no GPU): the arrays come back bit for
bit, and a damaged, truncated or foreign file is refused before anything is
resumed from it."""
import os

import numpy as np
import pytest

from paper_1904_08553_amd import dc


def _state(seed, n=500, nnz=3000):
    rng = np.random.default_rng(seed)
    deg = rng.multinomial(nnz, np.ones(n) / n)
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    col = rng.integers(0, n, nnz).astype(np.int32)
    w = rng.integers(1, 9, nnz).astype(np.int32)
    C = rng.integers(0, n, n).astype(np.int32)
    return n, off, col, w, C


def test_round_trip(tmp_path):
    st = _state(0)
    p = tmp_path / "g.npz"
    dc.write_checkpoint(p, *st)
    back = dc.read_checkpoint(p)
    assert back[0] == st[0]
    for a, b in zip(st[1:], back[1:]):
        assert a.dtype == b.dtype and np.array_equal(a, b)
    # no temporary file is left beside it
    assert sorted(os.listdir(tmp_path)) == ["g.npz"]


def test_replace_is_whole(tmp_path):
    p = tmp_path / "g.npz"
    dc.write_checkpoint(p, *_state(1))
    st2 = _state(2, n=700)
    dc.write_checkpoint(p, *st2)
    assert dc.read_checkpoint(p)[0] == 700


def test_flipped_byte_is_refused(tmp_path):
    n, off, col, w, C = _state(3)
    p = tmp_path / "g.npz"
    dc.write_checkpoint(p, n, off, col, w, C)
    # the same arrays with one label changed, under the stored digest
    with np.load(p, allow_pickle=False) as z:
        arrs = {k: z[k].copy() for k in z.files}
    arrs["C"][7] ^= 1
    with open(p, "wb") as f:
        np.savez(f, **arrs)
    with pytest.raises(dc.CheckpointError, match="digest"):
        dc.read_checkpoint(p)


def test_truncated_file_is_refused(tmp_path):
    p = tmp_path / "g.npz"
    dc.write_checkpoint(p, *_state(4))
    data = p.read_bytes()
    p.write_bytes(data[: len(data) // 2])
    with pytest.raises(dc.CheckpointError):
        dc.read_checkpoint(p)


def test_other_version_and_shapes_are_refused(tmp_path):
    n, off, col, w, C = _state(5)
    p = tmp_path / "g.npz"
    dc.write_checkpoint(p, n, off, col, w, C)
    with np.load(p, allow_pickle=False) as z:
        arrs = {k: z[k].copy() for k in z.files}
    bad = dict(arrs, version=np.array([dc.CKPT_VERSION + 1], np.int64))
    with open(p, "wb") as f:
        np.savez(f, **bad)
    with pytest.raises(dc.CheckpointError, match="version"):
        dc.read_checkpoint(p)
    bad = dict(arrs, n=np.array([n + 1], np.int64))
    with open(p, "wb") as f:
        np.savez(f, **bad)
    with pytest.raises(dc.CheckpointError, match="shapes"):
        dc.read_checkpoint(p)
    bad = {k: v for k, v in arrs.items() if k != "digest"}
    with open(p, "wb") as f:
        np.savez(f, **bad)
    with pytest.raises(dc.CheckpointError, match="missing"):
        dc.read_checkpoint(p)
