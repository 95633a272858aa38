"""Host pin of the error bounds behind the screened FP64 walk (paper, "Tree
walk": the FP64 walk's prune / open / cutoff decisions).  The screened walk
forms each node test's quantity in FP32 (node centre exact in half-cells,
the target's offset from its level-21 cell centre rounded once, the
centre-of-mass offset rounded once) and trusts the FP32 outcome only outside
a band around the threshold.  Here that FP32 arithmetic is emulated with
numpy (every operation rounded to float32; products and fused forms both
tried) on random boxes, levels, nodes and targets, and the FP32 values are
compared with the FP64 ones computed as the FP64 walk computes them:

  max|dc|:  |FP32 - FP64| <= 2^-22.4 (max|dc| + h) + 2^-51 (|lo| + L)
  r^2:      |FP32 - FP64| <= 2^-18.5 r^2   when side <= r (theta <= 1),
            |offset| <= side/2 per axis and h <= r/2

(h: half a level-21 cell, L the root side, lo the root corner, |lo| <= 64 L),
and the bands the kernel uses (64 and 1024 ulps of the FP32 value) cover
them with the thresholds' own FP32 rounding.  No GPU code runs here."""
import numpy as np

F32 = np.float32


def _r32(x):
    return np.asarray(x, dtype=np.float64).astype(F32)


def _fma32(a, b, c):
    # fused multiply-add on float32 operands: the float64 product of two
    # float32 values is exact, so one float64 add then one float32 rounding
    return _r32(np.float64(a) * np.float64(b) + np.float64(c))


def _sample(rng, n):
    L = rng.choice([1.0, 3.7, 1000.0, 0.013], n)
    lo = np.where(rng.random(n) < 0.5, 0.0, rng.uniform(-64.0, 64.0, n) * L)
    lev = rng.integers(2, 22, n)
    h = L * 2.0 ** -22                      # half a level-21 cell
    cells = 2 ** lev                        # cells per axis at the node's level
    corner = (rng.random((n, 3)) * cells[:, None]).astype(np.int64)
    side = L / cells
    # node centre in half-cells of the level-21 grid: exact integers
    C = (corner * (2 ** (21 - lev))[:, None] * 2 + (2 ** (21 - lev))[:, None]).astype(np.int64)
    return L, lo, lev, h, corner, side, C


def _target_near(rng, lo, L, centre, radius):
    x = centre + rng.uniform(-1.0, 1.0, centre.shape) * radius[:, None]
    return np.clip(x, lo[:, None], (lo + L * (1 - 2.0 ** -30))[:, None])


def _fp32_offsets(x, lo, L, C):
    """The screened walk's FP32 centre offsets dc (per axis)."""
    h64 = L * 2.0 ** -22
    cell = np.floor((x - lo[:, None]) * (2.0 ** 21 / L)[:, None]).astype(np.int64)
    cell = np.clip(cell, 0, 2 ** 21 - 1)
    o = 2 * cell + 1                                         # origin, half-cells
    xr = _r32(x - (lo[:, None] + o * h64[:, None]))          # FP64 then one rounding
    h22f = _r32(h64)
    f = (C - o).astype(F32)                                  # exact integer difference
    unfused = _r32(_r32(np.float64(f) * np.float64(h22f[:, None])) - np.float64(xr))
    fused = _fma32(f, h22f[:, None], -xr)
    return unfused, fused


def _fp64_centre(lo, L, corner, lev):
    """The FP64 walk's cube centre: corner in level-21 cells plus half a side."""
    hh = L * 2.0 ** -21
    half = 2.0 ** (20 - lev)
    corner21 = corner * (2 ** (21 - lev))[:, None]
    return lo[:, None] + (corner21 + half[:, None]) * hh[:, None]


def test_centre_offset_bound():
    rng = np.random.default_rng(20261203)
    worst = 0.0
    for _ in range(8):
        n = 50000
        L, lo, lev, h, corner, side, C = _sample(rng, n)
        c64 = _fp64_centre(lo, L, corner, lev)
        # targets from a few cells to a few node sides away from the centre
        x = _target_near(rng, lo, L, c64, np.maximum(side * rng.uniform(0.0, 3.0, n), 4 * h))
        dc64 = c64 - x
        mdc64 = np.abs(dc64).max(axis=1)
        for dc32 in _fp32_offsets(x, lo, L, C):
            mdc32 = np.abs(dc32.astype(np.float64)).max(axis=1)
            bound = 2.0 ** -22.4 * (mdc64 + h) + 2.0 ** -51 * (np.abs(lo) + L)
            err = np.abs(mdc32 - mdc64)
            assert np.all(err <= bound), (err / bound).max()
            worst = max(worst, (err / bound).max())
    assert worst > 0.05  # the samples reach the bound's scale


def test_r2_bound_near_thresholds():
    rng = np.random.default_rng(7)
    for _ in range(8):
        n = 50000
        L, lo, lev, h, corner, side, C = _sample(rng, n)
        c64 = _fp64_centre(lo, L, corner, lev)
        # centre of mass anywhere in the node; its FP32 offset from the centre
        com = c64 + rng.uniform(-0.5, 0.5, (n, 3)) * side[:, None]
        wo = _r32(com - c64)
        # targets at distance r in [side, 3 side] from the centre of mass
        # (theta <= 1 near the open threshold; the same holds at the cutoff
        # threshold for nodes that are not opened)
        d = rng.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        r = side * rng.uniform(1.0, 3.0, n)
        x = com - d * r[:, None]
        inside = np.all((x >= lo[:, None]) & (x < (lo + L)[:, None]), axis=1)
        keep = inside & (h <= r / 2)
        dx64 = com - x
        r2_64 = (dx64[:, 0] * dx64[:, 0] + dx64[:, 1] * dx64[:, 1]) + dx64[:, 2] * dx64[:, 2]
        for dc32 in _fp32_offsets(x, lo, L, C):
            dx32 = _r32(np.float64(dc32) + np.float64(wo))
            r2_32 = _fma32(dx32[:, 2], dx32[:, 2], _fma32(dx32[:, 0], dx32[:, 0], _r32(np.float64(dx32[:, 1]) ** 2)))
            err = np.abs(r2_32.astype(np.float64) - r2_64)
            assert np.all(err[keep] <= 2.0 ** -18.5 * r2_64[keep]), (err[keep] / r2_64[keep]).max()


def test_bands_cover_the_bounds():
    # a band of K ulps of a float32 value v is at least K 2^-24 v
    for v in (1.0, 1.5, 1.9999999, 3.0e-7, 6.0e5):
        u = np.spacing(F32(v)).astype(np.float64)
        assert 64 * u >= 64 * 2.0 ** -24 * v and 1024 * u >= 1024 * 2.0 ** -24 * v
    # distance tests: 2^-22.4 (max|dc| + h) with max|dc| >= 1.2 h near a
    # threshold, the 2^-51 (|lo| + L) term with |lo| <= 64 L and h = L 2^-22,
    # and the thresholds' own FP32 rounding (5 x 2^-24)
    need_c = 2.0 ** -22.4 * (1.0 + 1.0 / 1.2) + 2.0 ** -51 * 65.0 * 2.0 ** 22 / 1.2 + 5 * 2.0 ** -24
    assert need_c <= 2.0 ** -20.3 and 64 * 2.0 ** -24 >= 4 * need_c
    # r^2 tests: 2^-18.5 and the thresholds' rounding
    need_r = 2.0 ** -18.5 + 5 * 2.0 ** -24
    assert 1024 * 2.0 ** -24 >= 8 * need_r
