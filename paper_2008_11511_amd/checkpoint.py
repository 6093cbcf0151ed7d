"""Checkpoint and resume of a reconstruction.

A reconstruction's state is all caller-owned: object, probe, exit waves (DM,
AP with probe update), the CG state buffer of ML cycles, scan positions and
the background.  A checkpoint copies the named tensors to the host (after
the current stream's work) and writes them to one `.npz` file with no
pickled objects; `load` reads them back onto a device.  Kernels reduce in a
fixed order, so a run resumed from a checkpoint gives bitwise the result of
the uninterrupted run.
"""
from __future__ import annotations

import os
from typing import Dict, Optional

import numpy as np
import torch

FORMAT = 1


def save(path: str, **state) -> None:
    """Write tensors (any device) and numpy arrays under their keyword names.
    The file is written to `path` + ".tmp" and then renamed, so an
    interrupted save never leaves a partial checkpoint under `path`."""
    arrays = {"__format__": np.array(FORMAT, np.int64)}
    for name, value in state.items():
        if name.startswith("__"):
            raise ValueError(f"reserved name {name!r}")
        if value is None:
            continue
        if isinstance(value, torch.Tensor):
            arrays[name] = value.detach().cpu().numpy()        # waits for the stream's work
        else:
            arrays[name] = np.asarray(value)
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, **arrays)
    os.replace(tmp, path)


def load(path: str, device: Optional[torch.device] = None) -> Dict[str, torch.Tensor]:
    """Read a checkpoint: {name: tensor on `device`} (host if None)."""
    with np.load(path, allow_pickle=False) as z:
        fmt = int(z["__format__"]) if "__format__" in z.files else -1
        if fmt != FORMAT:
            raise ValueError(f"{path}: checkpoint format {fmt}, expected {FORMAT}")
        out = {}
        for name in z.files:
            if name == "__format__":
                continue
            t = torch.from_numpy(np.array(z[name]))
            out[name] = t.to(device) if device is not None else t
    return out
