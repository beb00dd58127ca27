"""The five named workloads, with their seeds.

Matrix seed 1000+k and vector seed 2000+k for workload k:

0. 2D 5-point Laplacian, 64 x 64, natural order (n 4096, nnz 20224).
1. 3D 27-point stencil, 128^3, natural order (n 2,097,152, nnz 55,742,968).
2. Random banded, n 4,000,000, lognormal row lengths (mean 12, sigma 0.8,
   max 200), columns within +-20000 of the diagonal; plus a symmetrically
   scrambled copy (seed 3002) whose bandwidth is near n.
3. 3D 7-point Poisson operator on a 128 x 128 x 1024 box (n 16,777,216), the
   same size as a 256^3 cube but with grid bandwidth 128*128 = 16384, which
   fits a 16-bit offset; the 256^3 cube itself (bandwidth 65536) does not.
4. Batched family: 512 matrices, n log-uniform on [1e3, 2e5], mixed kinds,
   1-8 right-hand sides (seed 1004; selector training uses seed 5004).
"""

from __future__ import annotations

from . import matrices as M

CONFIG_SEEDS = {k: (1000 + k, 2000 + k) for k in range(5)}
SCRAMBLE_SEED = 3002
BATCH_COUNT = 512
TRAIN_SEED = 5004

_DESCRIPTIONS = {
    0: "laplace2d_5pt_64x64",
    1: "stencil3d_27pt_128^3",
    2: "banded_n4M_hb20000",
    3: "poisson3d_7pt_128x128x1024",
    4: "batch512_mixed",
}


def config_description(k: int, scrambled: bool = False) -> str:
    d = _DESCRIPTIONS[k]
    return d + ("_scrambled" if scrambled else "")


def config_matrix(k: int, scrambled: bool = False, scale: float = 1.0) -> M.CSR:
    """Matrix of workload k (0..3).  scale < 1 gives a smaller instance of the
    same family for quick tests (grid edges and n scaled accordingly)."""
    mseed, _ = CONFIG_SEEDS[k]
    if k == 0:
        return M.laplace_2d_5pt(max(3, int(round(64 * scale))))
    if k == 1:
        return M.stencil_3d_27pt(max(3, int(round(128 * scale))), mseed)
    if k == 2:
        n = max(16, int(round(4_000_000 * scale)))
        A = M.random_banded(n, mseed, half_band=min(20000, n - 1))
        return M.scramble_symmetric(A, SCRAMBLE_SEED) if scrambled else A
    if k == 3:
        e = max(3, int(round(128 * scale)))
        return M.poisson_3d_7pt(e, e, max(3, int(round(1024 * scale))))
    raise ValueError(f"no single matrix for workload {k}")


def config_vector(k: int, n: int, nrhs: int | None = None, salt: int = 0):
    _, vseed = CONFIG_SEEDS[k]
    return M.uniform_vector(n, vseed + 100_000 * salt, nrhs)
