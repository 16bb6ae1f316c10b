"""Small helpers shared by the tests (no method arithmetic)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def grid_to_xy(pts) -> np.ndarray:
    """Grid integers (kx, ky) -> float32 (n, 2) coordinates k * 2^-20."""
    a = np.asarray(pts, dtype=np.int64).reshape(-1, 2)
    return (a.astype(np.float32) * np.float32(2.0 ** -20)).astype(np.float32)


def load_golden(name: str) -> dict:
    """Parse a hand-worked fixture from tests/golden/."""
    out: dict = {"points": []}
    section = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line == "points:":
                section = "points"
                continue
            if ":" in line:
                key, val = line.split(":", 1)
                out[key.strip()] = [int(v) for v in val.split()]
                section = None
                continue
            if section == "points":
                x, y = line.split()
                out["points"].append((int(x), int(y)))
    return out


def golden_names():
    return sorted(n for n in os.listdir(GOLDEN) if n.endswith(".txt"))
