"""Helpers for the GPU parity tests (device placement and result comparison)."""
import numpy as np
import torch

DEV = torch.device("cuda:0")


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def same_tmfg(got: dict, ref: dict) -> None:
    for k in ("order", "edges", "steps", "faces"):
        a, b = np.asarray(got[k]), np.asarray(ref[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)[:5]
            raise AssertionError(f"{k} differs at {bad.tolist()}")
    ga = np.asarray(got["step_gain"], dtype=np.float32)
    gb = np.asarray(ref["step_gain"], dtype=np.float32)
    assert ga.tobytes() == gb.tobytes(), "step gains differ"


def uint16_rows(idx: torch.Tensor, n: int) -> np.ndarray:
    return idx.cpu().numpy().view(np.uint16)[:, : n - 1].astype(np.int64)
