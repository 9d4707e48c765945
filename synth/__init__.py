"""Seeded synthetic inputs for the 7-point stencil systems.

This module is the one place where the inputs are defined. It draws random
numbers and lays them out; it holds none of the solver's arithmetic (no
operator application, no right-hand side, no Krylov step). Both the FP64 CPU
oracle (through the tests) and the GPU library's own device-side generator
follow the same published recipe, so the same seed gives the same problem on
either side, bit for bit.

Counter-based generator
-----------------------
SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the golden-ratio increment
0x9E3779B97F4A7C15 and the output is the Stafford "Mix13" finaliser
(xor-shift 30, multiply 0xBF58476D1CE4E5B9, xor-shift 27, multiply
0x94D049BB133111EB, xor-shift 31).  Used here statelessly:

    key(seed, aid) = splitmix64(seed XOR (aid << 56))
    h(seed, aid, c) = splitmix64(key(seed, aid) XOR c)

where ``aid`` names the array and ``c`` is the linear cell index
``i + nx*(j + ny*k)`` (x fastest).

Problem recipe (the stand-in for the paper's 600x595x1536 test system, whose
matrix is not published)
-----------------------------------------------------------------------------
* Off-diagonal coefficient of direction a (aid 1..6 = xm, xp, ym, yp, zm, zp):
  ``-(0.5 + m * 2**-24)`` with ``m = h >> 41`` (23 bits); exact in FP32,
  range [-1, -0.5).  Drawn independently per cell and direction, so the
  operator is nonsymmetric.
* Recipe "zslab" additionally multiplies zm and zp by
  ``f(k) = 1 + 9 s(k)``: s is 1 on the centred slab ``nz//4 <= k < 3*nz//4``,
  0 far outside, joined on each side by a smoothstep ramp 4 cells wide.  The
  product is formed in FP64 (exact) and rounded once to FP32.
* Diagonal (aid 0, not drawn): ``fl32(sum |off| + 0.1)``, the six magnitudes
  summed in FP64 in the order xm, xp, ym, yp, zm, zp (exact), then 0.1 added
  in FP64 and the result rounded to FP32 (round to nearest even).  Boundary
  faces draw and count their outward coefficients too; those multiply the
  zero Dirichlet ghosts.
* Manufactured solution x* (aid 7): ``-1 + m' * 2**-23`` with
  ``m' = h >> 40`` (24 bits); exact in FP32 and FP64, range [-1, 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)

# array ids
AID_DIAG, AID_XM, AID_XP, AID_YM, AID_YP, AID_ZM, AID_ZP, AID_XSTAR = range(8)
AID_BATCH_SIDES = 16
AID_SERVE_GAP = 17
AID_SERVE_SIDE = 18
AID_SERVE_MODE = 19

COEF_NAMES = ("diag", "xm", "xp", "ym", "yp", "zm", "zp")

RECIPE_IID = 0
RECIPE_ZSLAB = 1


def splitmix64(x):
    """SplitMix64 output for state ``x`` (uint64 scalar or array), wrapping."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + GAMMA
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        return z ^ (z >> np.uint64(31))


def key(seed: int, aid: int) -> np.uint64:
    s = np.uint64(seed & MASK64) ^ (np.uint64(aid) << np.uint64(56))
    return np.uint64(splitmix64(s))


def cell_hash(seed: int, aid: int, cells) -> np.ndarray:
    cells = np.asarray(cells, dtype=np.uint64)
    return splitmix64(key(seed, aid) ^ cells)


def uniform01(seed: int, aid: int, idx) -> np.ndarray:
    """U[0,1) doubles from the top 53 bits of the hash."""
    h = cell_hash(seed, aid, idx)
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def offdiag_base(seed: int, aid: int, cells) -> np.ndarray:
    """-(0.5 + m 2^-24), m = top 23 bits; float32, exact."""
    m = (cell_hash(seed, aid, cells) >> np.uint64(41)).astype(np.float64)
    return (-(0.5 + m * 2.0 ** -24)).astype(np.float32)


def xstar_values(seed: int, cells) -> np.ndarray:
    m = (cell_hash(seed, AID_XSTAR, cells) >> np.uint64(40)).astype(np.float64)
    return -1.0 + m * 2.0 ** -23


def zslab_factor(k, nz: int) -> np.ndarray:
    """f(k) = 1 + 9 s(k) of the "zslab" recipe (FP64, exact dyadic values)."""
    k = np.asarray(k, dtype=np.float64)
    lo, hi, w = nz // 4, (3 * nz) // 4, 4.0

    def smooth(t):
        t = np.clip(t, 0.0, 1.0)
        return t * t * (3.0 - 2.0 * t)

    s = smooth((k - (lo - w)) / w) * smooth(((hi - 1 + w) - k) / w)
    return 1.0 + 9.0 * s


@dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    coef: list  # 7 float32 arrays, order diag, xm, xp, ym, yp, zm, zp (length = cells)
    xstar: np.ndarray  # float64
    cells: np.ndarray  # linear indices the arrays cover


def _cells_of_planes(nx, ny, planes) -> np.ndarray:
    plane = np.arange(nx * ny, dtype=np.int64)
    return np.concatenate([plane + nx * ny * int(k) for k in planes]) if len(planes) else \
        np.zeros(0, dtype=np.int64)


def make_problem(nx: int, ny: int, nz: int, seed: int = 0, recipe: int = RECIPE_IID,
                 planes=None) -> Problem:
    """Coefficients and x* of the recipe, on the whole mesh or on the z-planes listed."""
    if planes is None:
        cells = np.arange(nx * ny * nz, dtype=np.int64)
    else:
        cells = _cells_of_planes(nx, ny, planes)
    k = cells // (nx * ny)
    offs = []
    for aid in (AID_XM, AID_XP, AID_YM, AID_YP, AID_ZM, AID_ZP):
        c = offdiag_base(seed, aid, cells)
        if recipe == RECIPE_ZSLAB and aid in (AID_ZM, AID_ZP):
            c = (c.astype(np.float64) * zslab_factor(k, nz)).astype(np.float32)
        offs.append(c)
    acc = np.zeros(cells.shape, dtype=np.float64)
    for c in offs:
        acc = acc + np.abs(c.astype(np.float64))
    diag = (acc + 0.1).astype(np.float32)
    return Problem(nx, ny, nz, [diag] + offs, xstar_values(seed, cells), cells)


# ---------------------------------------------------------------------------
# The 2D 9-point operator (section IV, "SpMV (2D)")
# ---------------------------------------------------------------------------
# Off-diagonal ids 20..27 = w, e, s, n, sw, se, nw, ne; each drawn as the 3D
# off-diagonals are, -(0.5 + m 2^-24) per cell.  Diagonal: fl32(sum |off| +
# 0.1), the eight magnitudes summed in FP64 in that order (exact), outward
# links included.  x* as in 3D (aid 7), over the cells i + nx*j.
AID_2D9 = tuple(range(20, 28))
COEF_NAMES_2D9 = ("diag", "w", "e", "s", "n", "sw", "se", "nw", "ne")
PAPER_MESHES_2D9 = ((4800, 4800), (22800, 22800))  # the sizes section IV names


def make_problem_2d9(nx: int, ny: int, seed: int = 0, rows=None) -> Problem:
    """Coefficients (diag, w, e, s, n, sw, se, nw, ne) and x* of the 2D 9-point recipe, on the
    whole mesh or on the y-rows listed (every value depends only on its cell's global index)."""
    if rows is None:
        cells = np.arange(nx * ny, dtype=np.int64)
    else:
        cells = np.concatenate([np.arange(nx, dtype=np.int64) + nx * int(j) for j in rows]) if len(rows) else \
            np.zeros(0, dtype=np.int64)
    offs = [offdiag_base(seed, aid, cells) for aid in AID_2D9]
    acc = np.zeros(cells.shape, dtype=np.float64)
    for c in offs:
        acc = acc + np.abs(c.astype(np.float64))
    diag = (acc + 0.1).astype(np.float32)
    return Problem(nx, ny, 1, [diag] + offs, xstar_values(seed, cells), cells)


# ---------------------------------------------------------------------------
# Workload shapes (the paper's mesh and the stand-ins around it)
# ---------------------------------------------------------------------------
PAPER_MESH = (600, 595, 1536)  # the CS-1 run's mesh

WORKLOADS = {
    "cube32": dict(dims=(32, 32, 32), recipe=RECIPE_IID, seed=0, rtol=1e-8, max_iter=500),
    "cube256_zslab": dict(dims=(256, 256, 256), recipe=RECIPE_ZSLAB, seed=0, rtol=1e-6,
                          max_iter=2000, timed_iters=200),
    "paper600x595x1536": dict(dims=PAPER_MESH, recipe=RECIPE_IID, seed=0, rtol=1e-8,
                              max_iter=2000, timed_iters=100),
}

BATCH_SIDES = (24, 32, 48, 64, 96, 128)


def batch_shapes(nsys: int = 64, seed: int = 0):
    """Per-system mesh dims, each side uniform over BATCH_SIDES, plus per-system seeds."""
    u = uniform01(seed, AID_BATCH_SIDES, np.arange(3 * nsys))
    idx = np.minimum((u * len(BATCH_SIDES)).astype(np.int64), len(BATCH_SIDES) - 1)
    sides = np.array(BATCH_SIDES)[idx].reshape(nsys, 3)
    return [tuple(int(v) for v in row) for row in sides], [1000 + s for s in range(nsys)]


# the batched 2D 9-point workload: 64 meshes, each side uniform over these
BATCH_SIDES_2D9 = (96, 128, 192, 256, 384, 512)
AID_BATCH_SIDES_2D9 = 28


# planes of the paper's mesh at which a converged solution is checked on the host: the
# two faces, their inner neighbours, the middle plane, and 16 more drawn from the seed
AID_SAMPLE_PLANES = 32


def sample_planes(nz: int, extra: int = 16, seed: int = 0):
    """The fixed planes {0, 1, nz/2, nz-2, nz-1} and `extra` further distinct planes of
    [0, nz), drawn by hashing (seed, AID_SAMPLE_PLANES, draw) until enough are found."""
    planes = sorted({0, 1, nz // 2, nz - 2, nz - 1} & set(range(nz)))
    fixed = len(planes)
    draw = 0
    while len(planes) < min(nz, fixed + extra):
        k = int(uniform01(seed, AID_SAMPLE_PLANES, np.array([draw]))[0] * nz)
        draw += 1
        if k not in planes:
            planes.append(k)
    return sorted(planes)


def batch_shapes_2d9(nsys: int = 64, seed: int = 0):
    """Per-system 2D mesh sides (nx, ny), each uniform over BATCH_SIDES_2D9, plus
    per-system seeds 2000 + s."""
    u = uniform01(seed, AID_BATCH_SIDES_2D9, np.arange(2 * nsys))
    idx = np.minimum((u * len(BATCH_SIDES_2D9)).astype(np.int64), len(BATCH_SIDES_2D9) - 1)
    sides = np.array(BATCH_SIDES_2D9)[idx].reshape(nsys, 2)
    return [tuple(int(v) for v in row) for row in sides], [2000 + s for s in range(nsys)]


@dataclass
class Request:
    rid: int
    arrival_s: float
    dims: tuple
    mode: str  # "fp32" or "bf16_ir"
    rtol: float
    seed: int


def serve_stream(n: int = 10000, rate: float = 200.0, seed: int = 0, lo: int = 16, hi: int = 256):
    """Poisson arrivals, log-uniform sides per axis, 50/50 modes (FP32 1e-6, BF16+IR 1e-10)."""
    ids = np.arange(n)
    gaps = -np.log1p(-uniform01(seed, AID_SERVE_GAP, ids)) / rate
    t = np.cumsum(gaps)
    u = uniform01(seed, AID_SERVE_SIDE, np.arange(3 * n)).reshape(n, 3)
    sides = np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)
    modes = uniform01(seed, AID_SERVE_MODE, ids) < 0.5
    out = []
    for i in range(n):
        mode = "fp32" if modes[i] else "bf16_ir"
        out.append(Request(i, float(t[i]), tuple(int(v) for v in sides[i]), mode,
                           1e-6 if mode == "fp32" else 1e-10, 1_000_000 + i))
    return out


AID_SERVE2_GAP, AID_SERVE2_SIDE, AID_SERVE2_MODE = 29, 30, 31


def serve_stream_2d9(n: int = 200, rate: float = 200.0, seed: int = 0, lo: int = 64, hi: int = 1024):
    """2D 9-point requests: Poisson arrivals, sides (nx, ny) log-uniform in [lo, hi],
    50/50 modes (FP32 1e-6, BF16+IR 1e-10), seeds 3 * 10^6 + id."""
    ids = np.arange(n)
    gaps = -np.log1p(-uniform01(seed, AID_SERVE2_GAP, ids)) / rate
    t = np.cumsum(gaps)
    u = uniform01(seed, AID_SERVE2_SIDE, np.arange(2 * n)).reshape(n, 2)
    sides = np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)
    modes = uniform01(seed, AID_SERVE2_MODE, ids) < 0.5
    out = []
    for i in range(n):
        mode = "fp32" if modes[i] else "bf16_ir"
        out.append(Request(i, float(t[i]), tuple(int(v) for v in sides[i]), mode,
                           1e-6 if mode == "fp32" else 1e-10, 3_000_000 + i))
    return out
