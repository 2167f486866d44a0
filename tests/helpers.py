"""Shared test helpers (no stitching arithmetic here)."""
from __future__ import annotations

import numpy as np
import torch


def gpu_available() -> bool:
    return torch.cuda.is_available()


def u8_report(got: np.ndarray, want: np.ndarray) -> tuple[int, float]:
    d = np.abs(got.astype(np.int64) - want.astype(np.int64))
    return int(d.max()) if d.size else 0, float((d == 1).mean()) if d.size else 0.0


def assert_u8_parity(got: np.ndarray, want: np.ndarray, max_frac: float = 1e-4) -> None:
    """No sample differs by more than 1; at most max_frac of the samples differ by 1."""
    assert got.shape == want.shape, (got.shape, want.shape)
    dmax, frac = u8_report(got, want)
    assert dmax <= 1, f"uint8 sample differs by {dmax}"
    assert frac <= max_frac, f"{frac:.3%} of uint8 samples differ by 1 (limit {max_frac:.3%})"


def assert_float_parity(got, want, tol: float = 1e-4, what: str = "") -> float:
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    err = float(np.max(np.abs(got - want))) if got.size else 0.0
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    assert err <= tol, f"{what}: max |delta| = {err:.3g} > {tol}"
    return err


def random_partition(rng, n: int, h: int, w: int, kind: str = "noise") -> list[np.ndarray]:
    """n uint8 weight maps summing to 255 at every pixel."""
    if n == 1:
        return [np.full((h, w), 255, np.uint8)]
    if kind == "cuts":
        cuts = np.sort(rng.choice(np.arange(1, w), size=n - 1, replace=False))
        bounds = [0, *cuts.tolist(), w]
        out = []
        for i in range(n):
            m = np.zeros((h, w), np.uint8)
            m[:, bounds[i]:bounds[i + 1]] = 255
            out.append(m)
        return out
    raw = rng.random((n, h, w))
    raw = raw / raw.sum(0, keepdims=True) * 255.0
    q = np.floor(raw).astype(np.int64)
    rem = 255 - q.sum(0)
    order = np.argsort(-(raw - q), axis=0)
    for r in range(n):
        sel = rem > r
        idx = order[r]
        np.put_along_axis(q, idx[None], np.take_along_axis(q, idx[None], 0) + sel[None], 0)
    assert np.all(q.sum(0) == 255)
    return [q[i].astype(np.uint8) for i in range(n)]


def rig_areas(rig, margin: int = 24) -> list:
    """The rig's feature detection areas (Alg. 2 step 1) from the library's host call,
    checked equal to the oracle's before use (so GPU and oracle work on the same areas)."""
    import oracle
    import paper_1810_03988_amd as P
    got = P.detection_areas(rig.frame_sizes, rig.H, rig.canvas_w, rig.canvas_h, margin)
    assert got == oracle.detection_areas(rig.frame_sizes, rig.H, rig.canvas_w, rig.canvas_h, margin)
    return got
