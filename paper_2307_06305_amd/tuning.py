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
GATHERS = (1, 2)  # stream variant: x values per gather load (interleaved, paired)


def candidates(paired=True):
    """All (variant, lanes, unroll, tile) the library accepts and the tuner
    tries.  The stream variant's tile is the cap on entries per workgroup and
    its unroll the number of x values per gather load (2: paired gathers,
    for the scalar storage cells)."""
    out = [(VECTOR, l, u, 2048) for l in LANES for u in UNROLLS]
    out += [(STREAM, g, x, t) for x in (GATHERS if paired else (1,)) for g in LANES for t in TILES]
    return out


def candidates_for(mat):
    """The candidates that apply to a handle: paired gathers only where the
    handle takes them."""
    return candidates(paired=mat.takes_paired)


def config_name(c):
    v, l, u, t = c
    if v == VECTOR:
        return f"vector_l{l}_u{u}"
    return f"{'paired' if u == 2 else 'stream'}_g{l}_t{t}"


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


def autotune(mat, x, y, configs=None, reps=20, finalists=3, sustained_s=0.02):
    """Time every configuration over `reps` products, then time the
    `finalists` fastest again over a sustained run of about `sustained_s`
    seconds each and keep the fastest of those.  The first pass ranks the
    candidates; the second compares the leaders where the GPU's clocks have
    settled (the first few hundred products after a change of kernel run
    several percent slower while its power management adapts, which a
    20-product timing does not average out).  Sets the winner, leaves the
    GPU in a sustained run of it, and returns it with every candidate's time
    (the finalists' from the sustained run)."""
    configs = candidates_for(mat) if configs is None else configs
    times = {}
    for c in configs:
        times[c] = time_config(mat, c, x, y, reps)
    def sustained(c):  # products in about sustained_s, within [reps, 10 reps]
        return min(10 * reps, max(reps, int(sustained_s / max(times[c], 1e-9))))

    ranked = sorted(times, key=times.get)[:max(1, finalists)]
    for c in ranked:
        n = sustained(c)
        time_config(mat, c, x, y, n)  # settle
        times[c] = time_config(mat, c, x, y, n)
    best = min(ranked, key=times.get)
    time_config(mat, best, x, y, sustained(best))  # sets it and leaves it running
    return best, times
