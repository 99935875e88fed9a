"""Reader for the hand-worked fixtures under tests/golden/ (plain text:
'#' comments, '[name]' headers, rows of integers)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str) -> dict:
    out, cur, rows = {}, None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                if cur is not None:
                    out[cur] = np.array(rows, dtype=np.int64)
                cur, rows = line.strip("[]"), []
                continue
            rows.append([int(t) for t in line.split()])
    if cur is not None:
        out[cur] = np.array(rows, dtype=np.int64)
    return out


def as_volume(a: np.ndarray) -> np.ndarray:
    """2D fixture (Y, Z) -> (1, Y, Z); 1-row fixture (1, Z) -> (1, 1, Z)."""
    return a.reshape((1,) + a.shape)
