"""Launch-configuration space of the product kernels and a timing autotuner.

The paper picks, per matrix, the fastest of its implementations and thread
counts (Sec. 4.1).  The GPU counterpart is the choice of kernel variant and
launch shape; `autotune` times every candidate on the device with HIP events
(through torch's stream) and keeps the fastest.
"""

from __future__ import annotations

VECTOR, STREAM = 0, 1

LANES = (1, 2, 4, 8, 16, 32, 64)
UNROLLS = (1, 2, 4)
TILES = (1024, 2048, 4096)


def candidates():
    """All (variant, lanes, unroll, tile) the library accepts and the tuner
    tries.  The stream variant's tile is the cap on entries per workgroup."""
    out = [(VECTOR, l, u, 2048) for l in LANES for u in UNROLLS]
    out += [(STREAM, g, 1, t) for g in LANES for t in TILES]
    return out


def config_name(c):
    v, l, u, t = c
    return f"vector_l{l}_u{u}" if v == VECTOR else f"stream_g{l}_t{t}"


def time_config(mat, cfg, x, y, reps=20, beta=0.0):
    """Mean device time (seconds) of one product with configuration cfg."""
    import torch

    mat.set_config(*cfg)
    mat.apply(x, y, 1.0, beta)  # warm
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        mat.apply(x, y, 1.0, beta)
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) * 1e-3 / reps


def autotune(mat, x, y, configs=None, reps=20):
    """Time every configuration; set and return the fastest with all timings."""
    configs = candidates() if configs is None else configs
    times = {}
    for c in configs:
        times[c] = time_config(mat, c, x, y, reps)
    best = min(times, key=times.get)
    mat.set_config(*best)
    return best, times
