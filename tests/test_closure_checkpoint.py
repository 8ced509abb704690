"""Host checks of the closure checkpoint file: layout written by
save_checkpoint, and load_checkpoint refusing foreign or truncated files before
any device work."""
import json
import struct

import numpy as np
import pytest
import torch

from paper_2003_01282_amd import closure as C


class FakeNet:
    """Stands in for S.Closure: the attributes and calls save_checkpoint uses."""
    d_in, hidden, nt = 10, 16, 8
    dims = [32, 16, 16, 16, 8]

    def __init__(self):
        self.offsets = [0, 512, 528, 784, 800, 1056, 1072, 1200]
        self.n_params = 1208
        rng = np.random.default_rng(0)
        self.vecs = {w: torch.from_numpy(rng.standard_normal(self.n_params).astype(np.float32)) for w in (0, 2, 3)}

    def step(self):
        return 17

    def get(self, which):
        return self.vecs[which]


def test_checkpoint_layout(tmp_path):
    net = FakeNet()
    path = tmp_path / "c.ckpt"
    C.save_checkpoint(net, str(path), epoch=3, seed=9)
    raw = path.read_bytes()
    (hl,) = struct.unpack("<Q", raw[:8])
    head = json.loads(raw[8:8 + hl])
    assert head["format"] == C.CHECKPOINT_FORMAT
    assert (head["epoch"], head["seed"], head["adam_step"], head["n_params"]) == (3, 9, 17, net.n_params)
    assert head["arrays"] == ["weights", "adam_m1", "adam_m2"] and head["offsets"] == net.offsets
    body = np.frombuffer(raw[8 + hl:], dtype="<f4")
    assert body.size == 3 * net.n_params
    for k, which in enumerate((0, 2, 3)):
        assert np.array_equal(body[k * net.n_params:(k + 1) * net.n_params], net.vecs[which].numpy())


def test_load_refuses_foreign_and_truncated_files(tmp_path):
    bad = tmp_path / "bad.ckpt"
    head = json.dumps({"format": "something-else"}).encode()
    bad.write_bytes(struct.pack("<Q", len(head)) + head)
    with pytest.raises(ValueError, match="not a closure checkpoint"):
        C.load_checkpoint(str(bad))
    good = tmp_path / "good.ckpt"
    C.save_checkpoint(FakeNet(), str(good))
    cut = tmp_path / "cut.ckpt"
    cut.write_bytes(good.read_bytes()[:-4])
    with pytest.raises(ValueError, match="truncated"):
        C.load_checkpoint(str(cut))
