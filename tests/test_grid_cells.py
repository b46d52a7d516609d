"""The cell block a hit point's disc can reach (device function disc_cells),
modelled in float32 on the CPU: every photon cell within the disc must lie in
the block, and the fine grid's block must span at most 3 cells per axis.

The model repeats the device arithmetic step by step: cell coordinates
(x - lo) * inv_h in float32, the widened radius rc (1 + 2^-8) + (|cc| + 1) 2^-s,
and the photon's cell floor((p - lo) * inv_h).  Photons are drawn inside the
disc (float32 squared distance, compared in double, as the range query does)
and right at its rim, where rounding matters most.
"""
import numpy as np
import pytest

f32 = np.float32


def _grid(r_max, fine):
    h = (r_max * (1.0 + 1.0 / 32.0)) if fine else (2.0 * r_max * (1.0 + 1.0 / 1024.0))
    return f32(1.0 / h)


def _block(cc, rc, fine):
    """Per axis: first cell and number of cells (the device's disc_cells)."""
    if fine:
        rr = rc * f32(1.0 + 2.0 ** -8) + (np.abs(cc) + f32(1.0)) * f32(2.0 ** -20)
        c0 = np.floor(cc - rr).astype(np.int64)
        n = np.minimum(np.floor(cc + rr).astype(np.int64) - c0 + 1, 3)
        return c0, n, np.floor(cc + rr).astype(np.int64) - c0 + 1
    rr = rc * f32(1.0 + 2.0 ** -8) + (np.abs(cc) + f32(1.0)) * f32(2.0 ** -16)
    bb = np.floor(cc - f32(0.5)).astype(np.int64)
    mid = (bb + 1).astype(f32)
    lower = (cc - rr) < mid
    upper = (cc + rr) >= mid
    c0 = np.where(lower, bb, bb + 1)
    n = lower.astype(np.int64) + upper.astype(np.int64)
    return c0, n, n


@pytest.mark.parametrize("fine", [True, False])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_disc_cells_cover_the_disc(fine, seed):
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-3.0, 3.0, 3).astype(f32)
    for _ in range(40):
        ext = f32(rng.uniform(0.5, 20.0))
        # radii from a few cells across the scene down to the 4096-cell limit of the fine grid
        r_max = float(ext) / float(rng.choice([4.0, 64.0, 1000.0, 4000.0])) / (1.0 + 1.0 / 32.0)
        inv_h = _grid(r_max, fine)
        m = 4000
        x = (lo + rng.uniform(0.0, 1.0, (m, 3)).astype(f32) * ext).astype(f32)
        r = (r_max * rng.uniform(0.0, 1.0, m) ** 0.25).astype(np.float64)
        r[:50] = r_max
        # half the hit points sit where the disc's rim meets a cell boundary
        # along a random axis (within a few float32 steps)
        k = m // 2
        ax = rng.integers(0, 3, k)
        sgn = np.where(rng.uniform(size=k) < 0.5, -1.0, 1.0)
        cell_edge = 1.0 / float(inv_h)
        cc0 = np.floor((x[:k, ax[0]] - lo[ax[0]]) / cell_edge)   # any cell index near the old point
        target = (cc0 + 0.5 + sgn * 0.5) * cell_edge - sgn * r[:k] * rng.uniform(1 - 1e-6, 1 + 1e-6, k)
        x[np.arange(k), ax] = (lo[ax] + target).astype(f32)
        r2 = r * r
        cc = ((x - lo) * inv_h).astype(f32)
        rc = (np.sqrt(r2).astype(f32) * inv_h).astype(f32)
        c0, n, n_raw = _block(cc, rc[:, None], fine)
        if fine:
            assert n_raw.max() <= 3          # the clamp in the device code never bites
        assert n.min() >= 1 and n.max() <= (3 if fine else 2)
        # photons inside the disc, many right at its rim
        d = rng.normal(size=(m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        d[np.arange(k)] = 0.0                                     # boundary cases: along the axis, towards the rim
        d[np.arange(k), ax] = sgn
        s = np.where(rng.uniform(size=m) < 0.5, 1.0 - 1e-7, rng.uniform(size=m) ** (1 / 3))
        p = (x.astype(np.float64) + d * (r * s)[:, None]).astype(f32)
        diff = (p - x).astype(f32)
        d2 = ((diff[:, 0] * diff[:, 0] + diff[:, 1] * diff[:, 1]).astype(f32) + diff[:, 2] * diff[:, 2]).astype(f32)
        inside = d2.astype(np.float64) < r2
        pc = np.floor(((p - lo) * inv_h).astype(f32)).astype(np.int64)
        ok = (pc >= c0) & (pc < c0 + n)
        assert ok[inside].all()
        assert inside.mean() > 0.3
