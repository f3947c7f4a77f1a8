"""Seeded synthetic datasets.

X is drawn in float64 and rounded to float32; y is computed in float64 from the
rounded X (plus noise) and then rounded to float32, so that both evaluation
sides see exactly the same float32 inputs.  X is returned feature-major
([F, N], one contiguous row of N values per feature).
"""
import numpy as np

from .configs import Config

STREAM_X, STREAM_NOISE, STREAM_POP, STREAM_GOM, STREAM_REDRAW = 0, 1, 2, 3, 4
F32_MAX = float(np.finfo(np.float32).max)


def rng_for(cid: int, stream: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(cid), int(stream), int(salt)])


def make_dataset(cfg: Config, N: int = None, salt: int = 0):
    """Return (X32 [F, N] float32, y32 [N] float32) for a workload.

    ``N`` overrides the row count (same distribution); ``salt`` selects an
    independent draw.
    """
    N = cfg.N if N is None else int(N)
    rng = rng_for(cfg.cid, STREAM_X, salt)
    if cfg.x_dist == "N":
        x64 = rng.standard_normal((cfg.F, N))
    else:
        x64 = rng.uniform(cfg.x_lo, cfg.x_hi, (cfg.F, N))
    X32 = np.ascontiguousarray(x64.astype(np.float32))
    del x64
    xr = X32.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        y64 = cfg.target(xr)
    # a row whose target is not a finite float32 (e.g. a division by an exact
    # zero of the rounded inputs), or whose denominator is closer to zero than
    # the workload allows, is redrawn from its own stream; other rows keep
    # their values
    redraw = rng_for(cfg.cid, STREAM_REDRAW, salt)

    def rejected(xs, ys):
        out = ~(np.abs(ys) <= F32_MAX)
        if cfg.den is not None:
            out |= ~(np.abs(cfg.den(xs)) >= cfg.den_min)
        return out

    bad = rejected(xr, y64)
    while np.any(bad):
        cols = np.nonzero(bad)[0]
        if cfg.x_dist == "N":
            xn = redraw.standard_normal((cfg.F, cols.size))
        else:
            xn = redraw.uniform(cfg.x_lo, cfg.x_hi, (cfg.F, cols.size))
        X32[:, cols] = xn.astype(np.float32)
        xr[:, cols] = X32[:, cols].astype(np.float64)
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            y64[cols] = cfg.target(xr[:, cols])
        bad = np.zeros(N, dtype=bool)
        bad[cols] = rejected(xr[:, cols], y64[cols])
    if cfg.noise:
        y64 = y64 + cfg.noise * rng_for(cfg.cid, STREAM_NOISE, salt).standard_normal(N)
    y32 = y64.astype(np.float32)
    assert np.all(np.isfinite(y32))
    return X32, y32
